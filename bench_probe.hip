// Throughput probes behind bench.py's peak figures (bench.py --peak-probe):
// chip-wide vector ALU issue rates (independent chains of v_add_u32,
// v_sad_u16 and v_fma_f32) and the LDS read bandwidth of conflict-free
// ds_read_b128 loops.  Measurement support only; not part of the library.
//
// Every access is in bounds: the LDS index is masked to the 64 KB buffer and
// each thread writes one word of an output of grid x block words.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kIters = 4096;
constexpr int kThreads = 512;

// OP 0: v_add_u32 (8 per iteration); 1: v_sad_u16; 2: v_fma_f32.
template <int OP>
__global__ __launch_bounds__(kThreads) void valu_kernel(unsigned* out, unsigned seed) {
  unsigned a[8];
  float f[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = seed + threadIdx.x * 8 + i;
    f[i] = (float)a[i];
  }
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (OP == 0) a[i] = a[i] + a[(i + 1) & 7];
      if constexpr (OP == 1) a[i] = __builtin_amdgcn_sad_u16(a[i], a[(i + 3) & 7], a[(i + 1) & 7]);
      if constexpr (OP == 2) f[i] = fmaf(f[i], 0.999f, f[(i + 1) & 7]);
    }
  }
  unsigned r = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) r ^= a[i] ^ __float_as_uint(f[i]);
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void lds_read_kernel(unsigned* out) {
  __shared__ uint4 buf[4096];   // 64 KB
  for (int i = threadIdx.x; i < 4096; i += blockDim.x) buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint4 v = buf[(threadIdx.x + (it * 8 + j) * 64) & 4095];
      acc.x ^= v.x;
      acc.y += v.y;
      acc.z ^= v.z;
      acc.w += v.w;
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

typedef short bf16x8_t __attribute__((ext_vector_type(8)));
typedef int i32x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// OP 0: v_mfma_f32_16x16x32_bf16; 1: v_mfma_scale_f32_16x16x128_f8f6f4 (E4M3
// operands, unit block scales).  Four independent accumulators per wave.
template <int OP>
__global__ __launch_bounds__(256) void mfma_kernel(float* out, int seed) {
  f32x4_t acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int t = threadIdx.x + seed;
  bf16x8_t a16, b16;
  i32x8_t a8, b8;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a16[i] = (short)(0x3F80 + ((t + i) & 7));
    b16[i] = (short)(0x3F80 + ((t * 3 + i) & 7));
    a8[i] = 0x38383838 + ((t + i) & 3);
    b8[i] = 0x38383838 + ((t * 5 + i) & 3);
  }
  for (int it = 0; it < kIters / 4; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if constexpr (OP == 0) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a16, b16, acc[i], 0, 0, 0);
      if constexpr (OP == 1)
        acc[i] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc[i], 0, 0, 0, 127, 0, 127);
    }
  }
  float r = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) r += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace

// Runs each probe twice and stores the second run's rates:
// out[0..2] = wave64 instructions per second of v_add_u32, v_sad_u16,
// v_fma_f32; out[3] = LDS bytes read per second; out[4] = compute units;
// out[5], out[6] = dense matrix-core flop per second of
// v_mfma_f32_16x16x32_bf16 and v_mfma_scale_f32_16x16x128_f8f6f4 (E4M3).
// Returns 0, or the HIP error code of the first failing call.
extern "C" int bench_probe_run(double* out) {
  int ncu = 0;
  hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0);
  if (e != hipSuccess) return (int)e;
  const int blocks = ncu * 8;
  unsigned* buf = nullptr;
  if ((e = hipMalloc(&buf, (size_t)blocks * kThreads * 4)) != hipSuccess) return (int)e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) rc = (int)e;
  for (int op = 0; op < 6 && !rc; ++op) {
    float ms = 0.f;
    for (int rep = 0; rep < 2 && !rc; ++rep) {
      if ((e = hipEventRecord(e0, 0)) != hipSuccess) { rc = (int)e; break; }
      if (op == 0) hipLaunchKernelGGL(valu_kernel<0>, dim3(blocks), dim3(kThreads), 0, 0, buf, 1u);
      if (op == 1) hipLaunchKernelGGL(valu_kernel<1>, dim3(blocks), dim3(kThreads), 0, 0, buf, 1u);
      if (op == 2) hipLaunchKernelGGL(valu_kernel<2>, dim3(blocks), dim3(kThreads), 0, 0, buf, 1u);
      if (op == 3) hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(kThreads), 0, 0, buf);
      if (op == 4) hipLaunchKernelGGL(mfma_kernel<0>, dim3(blocks), dim3(256), 0, 0, (float*)buf, 1);
      if (op == 5) hipLaunchKernelGGL(mfma_kernel<1>, dim3(blocks), dim3(256), 0, 0, (float*)buf, 1);
      if ((e = hipGetLastError()) != hipSuccess || (e = hipEventRecord(e1, 0)) != hipSuccess ||
          (e = hipEventSynchronize(e1)) != hipSuccess || (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        rc = (int)e;
    }
    if (rc) break;
    const double waves = (double)blocks * kThreads / 64.0;
    if (op < 3) out[op] = waves * kIters * 8 / (ms * 1e-3);
    else if (op == 3) out[3] = (double)blocks * kThreads * kIters * 8 * 16 / (ms * 1e-3);
    else out[op + 1] = (double)blocks * 4 * kIters * (op == 4 ? 16384.0 : 65536.0) / (ms * 1e-3);
  }
  out[4] = ncu;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return rc;
}

// Device helpers shared by the assignment kernels.
#pragma once
#include "dev_common.h"

namespace vqnnf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));


// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}


// Query storage of a kernel instance.
constexpr int kQBF16 = 0, kQF32 = 1, kQFP8 = 2, kQRGB8 = 3;

typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Eight E4M3FN codes (two words, element 0 in the low byte) to FP32, exactly
// (gfx950's conversion follows the OCP E4M3FN encoding).
__device__ __forceinline__ void fp8x8_to_f32(uint32_t w0, uint32_t w1, float (&x)[8]) {
  const f32x2_t a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w0, false);
  const f32x2_t b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w0, true);
  const f32x2_t c = __builtin_amdgcn_cvt_pk_f32_fp8((int)w1, false);
  const f32x2_t d = __builtin_amdgcn_cvt_pk_f32_fp8((int)w1, true);
  x[0] = a[0]; x[1] = a[1]; x[2] = b[0]; x[3] = b[1];
  x[4] = c[0]; x[5] = c[1]; x[6] = d[0]; x[7] = d[1];
}

__device__ __forceinline__ f32x4_t mfma_bf16(uint4 a, uint4 b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                 __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}


// Top-2 merge of (best value, best index, second value) triples; ties in the
// best value keep the lower index and make the second equal to the best.
// Branch-free: every lane takes the same path.
__device__ __forceinline__ void merge_top2_sel(float& v1, int& j1, float& v2, float o1, int oj1, float o2) {
  const bool take = o1 < v1 || (o1 == v1 && oj1 < j1);
  const float nv2 = take ? fminf(v1, o2) : fminf(v2, o1);
  v1 = take ? o1 : v1;
  j1 = take ? oj1 : j1;
  v2 = nv2;
}

// Lane l's partner value x[l ^ 16] and x[l ^ 32] for a full wave, with
// gfx950's row swaps (v_permlane16_swap: odd 16-lane rows of the first
// operand with even rows of the second; v_permlane32_swap: upper half of the
// first with lower half of the second) instead of an LDS permute.  Called
// with both operands equal, the first result holds the rows / half that
// moved into the first operand, the second those that moved out of it.
__device__ __forceinline__ uint32_t lane_xor16(uint32_t x, int lane) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  return (lane & 16) ? r[0] : r[1];
}
__device__ __forceinline__ uint32_t lane_xor32(uint32_t x, int lane) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (lane & 32) ? r[0] : r[1];
}
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int m, int lane) {
  return m == 16 ? lane_xor16(x, lane) : lane_xor32(x, lane);
}

constexpr int kWPB = 8;


typedef __attribute__((address_space(3))) void lds_void_t;

// Raw buffer resource over [base, base + 4 GiB): stride 0, 32-bit data
// format, so a load's address is base + voffset + soffset and the uniform part
// of every address stays in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}

// s_waitcnt with only the vector-memory counter limited to N (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt and lgkmcnt at their no-wait maxima).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}


}  // namespace vqnnf

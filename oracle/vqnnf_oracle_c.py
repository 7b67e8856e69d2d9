"""ctypes wrapper of the C variant of the FP64 oracle (vqnnf_oracle_c.c).

TEST INFRASTRUCTURE ONLY, like oracle/vqnnf_oracle.py: only the test suite,
the smoke check, the benchmark's CPU-baseline leg and the scripts that write
stored expected values use it.  It is built with gcc (no fast-math, no
contraction into FMA) into oracle/libvqnnf_oracle.so; `build()` compiles it
and the first use compiles it when the library is missing.

The functions return the same values as the Python oracle's, bit for bit
(pinned by tests/test_oracle_c.py):
  decode(dtype, data, scale)            == vqnnf_oracle.decode
  sq_distances_map(...)                 == vqnnf_oracle.sq_distances
  assign_map(dtype, data, scale, cb)    == vqnnf_oracle.assign_map
  kmeans_codebook(template, k, iters, seed) == vqnnf_oracle.kmeans_codebook
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vqnnf_oracle_c.c")
LIB = os.path.join(HERE, "libvqnnf_oracle.so")
# baseline x86-64 code (the library may run on another host than the one
# that built it); -ffp-contract=off: no FMA; no -ffast-math anywhere
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-pthread"]

_DT = {"f32": 0, "bf16": 1, "fp8": 2}
_lib = None
_lock = threading.Lock()


def build(out: Optional[str] = None) -> str:
    out = out or LIB
    tmp = out + f".tmp{os.getpid()}"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def lib() -> C.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            L = C.CDLL(LIB)
            vp, i32, i64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64
            L.vqo_e4m3fn_value.restype = C.c_double
            L.vqo_e4m3fn_value.argtypes = [i32]
            L.vqo_decode.restype = i32
            L.vqo_decode.argtypes = [vp, i32, i64, i64, i32, vp, vp]
            L.vqo_assign.restype = i32
            L.vqo_assign.argtypes = [vp, i32, i64, i64, i32, vp, vp, i32, vp, vp, i32]
            L.vqo_kmeans.restype = i32
            L.vqo_kmeans.argtypes = [vp, i64, i32, i32, i32, u64, vp, vp, i32]
            L.vqo_splitmix64.restype = None
            L.vqo_splitmix64.argtypes = [u64, i32, vp, vp]
            _lib = L
    return _lib


def _threads(n_threads: Optional[int]) -> int:
    if n_threads:
        return int(n_threads)
    return max(1, len(os.sched_getaffinity(0)))


def _map_args(dtype: str, data: np.ndarray, scale):
    if dtype == "f32":
        a = np.ascontiguousarray(data, dtype=np.float32)
    elif dtype == "bf16":
        a = np.ascontiguousarray(data, dtype=np.uint16)
    elif dtype == "fp8":
        a = np.ascontiguousarray(data, dtype=np.uint8)
    else:
        raise ValueError(dtype)
    D = a.shape[-1]
    n = a.size // D
    sc = None
    if dtype == "fp8":
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        assert sc.shape == (D,)
    return a, n, D, sc


def decode(dtype: str, data: np.ndarray, scale=None) -> np.ndarray:
    a, n, D, sc = _map_args(dtype, data, scale)
    out = np.empty(a.shape, dtype=np.float64)
    rc = lib().vqo_decode(a.ctypes.data, _DT[dtype], n, D, D, sc.ctypes.data if sc is not None else None,
                          out.ctypes.data)
    assert rc == 0
    return out


def _assign(dtype, data, scale, codebook, want_labels, want_dist, n_threads):
    a, n, D, sc = _map_args(dtype, data, scale)
    cb = np.ascontiguousarray(codebook, dtype=np.float64)
    k = cb.shape[0]
    assert cb.shape == (k, D)
    lab = np.empty(n, dtype=np.uint8) if want_labels else None
    dist = np.empty((n, k), dtype=np.float64) if want_dist else None
    rc = lib().vqo_assign(a.ctypes.data, _DT[dtype], n, D, D, sc.ctypes.data if sc is not None else None,
                          cb.ctypes.data, k, lab.ctypes.data if lab is not None else None,
                          dist.ctypes.data if dist is not None else None, _threads(n_threads))
    if rc != 0:
        raise RuntimeError(f"vqo_assign failed ({rc})")
    return lab, dist


def assign_map(dtype: str, data: np.ndarray, scale, codebook: np.ndarray,
               n_threads: Optional[int] = None) -> np.ndarray:
    """Alg. 1 on a stored map [H, W, D] (or [n, D]): uint8 labels of the same
    leading shape; codebook float64 (or exact FP32 values) [k, D]."""
    lab, _ = _assign(dtype, data, scale, codebook, True, False, n_threads)
    return lab.reshape(np.asarray(data).shape[:-1])


def sq_distances_map(dtype: str, data: np.ndarray, scale, codebook: np.ndarray,
                     n_threads: Optional[int] = None) -> np.ndarray:
    """FP64 squared distances [n, k] of every stored pixel to every codeword."""
    _, dist = _assign(dtype, data, scale, codebook, False, True, n_threads)
    return dist


def kmeans_codebook(template: np.ndarray, k: int, iters: int = 20, seed: int = 0,
                    return_f64: bool = False, n_threads: Optional[int] = None):
    """Codebook of a template [h, w, D] (FP32 values): k-means++ then `iters`
    Lloyd iterations in FP64, rounded to FP32."""
    t = np.ascontiguousarray(template, dtype=np.float32)
    D = t.shape[-1]
    l = t.size // D
    c64 = np.empty((k, D), dtype=np.float64)
    c32 = np.empty((k, D), dtype=np.float32)
    rc = lib().vqo_kmeans(t.ctypes.data, l, D, k, iters, seed & 0xFFFFFFFFFFFFFFFF, c64.ctypes.data,
                          c32.ctypes.data, _threads(n_threads))
    if rc != 0:
        raise RuntimeError(f"vqo_kmeans failed ({rc})")
    return (c32, c64) if return_f64 else c32


def splitmix64(seed: int, n: int):
    """First n outputs of the generator and of u01 from `seed`."""
    out = np.empty(n, dtype=np.uint64)
    u = np.empty(n, dtype=np.float64)
    lib().vqo_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, n, out.ctypes.data, u.ctypes.data)
    return out, u


def e4m3fn_value(code: int) -> float:
    return float(lib().vqo_e4m3fn_value(int(code)))

"""Thin Python binding of the vqnnf C ABI (include/vqnnf.h).

Argument marshalling only: every step of the hot path runs in the gfx950
kernels of libvqnnf.so.  Device buffers are torch tensors (their data_ptr()
is passed through); host arrays are numpy arrays.  Loading fails loudly when
the library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvqnnf.so")

VQNNF_OK, VQNNF_EINVAL, VQNNF_ENOMEM, VQNNF_EHIP, VQNNF_ENOTSUP, VQNNF_EHANDLE = range(6)
VQNNF_F32, VQNNF_BF16, VQNNF_FP8_E4M3, VQNNF_RGB8 = 0, 1, 2, 3
VQNNF_PREC_FP32_PLAIN, VQNNF_PREC_BF16_REFINED, VQNNF_PREC_FP8_REFINED = 0, 1, 2

EXPORTED = [
    "vqnnf_ctx_create", "vqnnf_ctx_create_host", "vqnnf_ctx_destroy", "vqnnf_codebook",
    "vqnnf_codebook_batched", "vqnnf_pca_fit", "vqnnf_pca_project",
    "vqnnf_template_from_codebook", "vqnnf_template_free", "vqnnf_template_info",
    "vqnnf_template_codebook", "vqnnf_template_labels", "vqnnf_template_counts",
    "vqnnf_template_weights", "vqnnf_template_responses", "vqnnf_paper_bank", "vqnnf_assign", "vqnnf_filter", "vqnnf_score",
    "vqnnf_score_integral", "vqnnf_match", "vqnnf_match_noalloc", "vqnnf_match_batched",
    "vqnnf_ctx_set_graph", "vqnnf_batched_labels", "vqnnf_ctx_set_debug_scores",
    "vqnnf_template_score_bound", "vqnnf_ctx_set_tune_file",
    "vqnnf_ctx_set_autotune",
    "vqnnf_ctx_set_timing", "vqnnf_ctx_kernel_times",
    "vqnnf_ctx_reset_times", "vqnnf_last_error", "vqnnf_version",
]


class VqnnfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vqnnf status {status}: {msg}")
        self.status = status


class FMap(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
                ("D", C.c_int32), ("pixel_stride", C.c_int64), ("channel_scale", C.c_void_p)]


class FilterDesc(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32),
                ("gx", C.c_int32), ("gy", C.c_int32), ("bin_weight", C.c_void_p),
                ("weight", C.c_float)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(no fallback implementation exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_int
    P = C.POINTER
    sig = {
        "vqnnf_ctx_create": (st, [vp, u64, P(vp)]),
        "vqnnf_ctx_create_host": (st, [u64, P(vp)]),
        "vqnnf_ctx_destroy": (None, [vp]),
        "vqnnf_codebook": (st, [vp, P(FMap), i32, i32, u64, P(FilterDesc), i32, P(vp)]),
        "vqnnf_template_from_codebook": (st, [vp, P(FMap), vp, i32, P(FilterDesc), i32, P(vp)]),
        "vqnnf_pca_fit": (st, [P(FMap), i32, vp, vp, vp]),
        "vqnnf_pca_project": (st, [vp, P(FMap), vp, vp, i32, vp]),
        "vqnnf_codebook_batched": (st, [vp, i32, P(P(FMap)), P(i32), i32, P(u64), P(P(FilterDesc)),
                                        P(i32), P(vp)]),
        "vqnnf_template_free": (None, [vp]),
        "vqnnf_template_info": (st, [vp, P(i32), P(i32), P(i32), P(i32), P(i32)]),
        "vqnnf_template_codebook": (st, [vp, vp]),
        "vqnnf_template_labels": (st, [vp, vp]),
        "vqnnf_template_counts": (st, [vp, vp]),
        "vqnnf_template_weights": (st, [vp, vp]),
        "vqnnf_template_responses": (st, [vp, vp]),
        "vqnnf_paper_bank": (st, [i32, i32, i32, i32, P(FilterDesc), vp, i32, P(i32)]),
        "vqnnf_assign": (st, [vp, vp, P(FMap), i32, vp, P(i64)]),
        "vqnnf_filter": (st, [vp, vp, vp, i32, i32, vp]),
        "vqnnf_score": (st, [vp, vp, vp, i32, i32, vp, P(i32), P(C.c_float)]),
        "vqnnf_score_integral": (st, [vp, vp, vp, i32, i32, vp, P(i32), P(C.c_float)]),
        "vqnnf_match": (st, [vp, vp, P(FMap), i32, vp, P(i32), P(C.c_float)]),
        "vqnnf_match_noalloc": (st, [vp, vp, P(FMap), i32, vp, P(i32), P(C.c_float)]),
        "vqnnf_match_batched": (st, [vp, i32, P(vp), P(P(FMap)), i32, P(vp), P(i32), P(C.c_float)]),
        "vqnnf_ctx_set_graph": (st, [vp, i32]),
        "vqnnf_batched_labels": (st, [vp, i32, vp]),
        "vqnnf_ctx_set_debug_scores": (st, [vp, vp, i64]),
        "vqnnf_template_score_bound": (st, [vp, i32, vp, vp]),
        "vqnnf_ctx_set_autotune": (st, [vp, i32]),
        "vqnnf_ctx_set_tune_file": (st, [vp, C.c_char_p]),
        "vqnnf_ctx_set_timing": (st, [vp, i32]),
        "vqnnf_ctx_kernel_times": (st, [vp, i32, P(C.c_char_p), P(i64), P(C.c_double), P(i32)]),
        "vqnnf_ctx_reset_times": (st, [vp]),
        "vqnnf_last_error": (C.c_char_p, []),
        "vqnnf_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != VQNNF_OK:
        raise VqnnfError(status, lib().vqnnf_last_error().decode())


def last_error() -> str:
    return lib().vqnnf_last_error().decode()


# ------------------------------------------------------------------ maps

_DT = {"f32": VQNNF_F32, "bf16": VQNNF_BF16, "fp8": VQNNF_FP8_E4M3, "rgb8": VQNNF_RGB8}


def host_fmap(arr: np.ndarray) -> Tuple[FMap, np.ndarray]:
    """Host map [H][W][D] as FP32, or a uint8 RGB image [H][W][3] (its 27
    colour features); the array is kept alive by the caller."""
    if arr.dtype == np.uint8 and arr.ndim == 3 and arr.shape[2] == 3:
        a = np.ascontiguousarray(arr)
        H, W, _ = a.shape
        return FMap(a.ctypes.data, VQNNF_RGB8, H, W, 27, 3, None), a
    a = np.ascontiguousarray(arr, dtype=np.float32)
    H, W, D = a.shape
    return FMap(a.ctypes.data, VQNNF_F32, H, W, D, D, None), a


def device_fmap(t, dtype: str, channel_scale: Optional[np.ndarray] = None) -> FMap:
    """Device map from a torch tensor [H][W][D] (float32 / uint16 bits /
    bfloat16 / uint8 E4M3FN codes with host FP32 channel_scale[D] / uint8 RGB
    pixels of S >= 3 bytes, "rgb8")."""
    H, W, S = t.shape[0], t.shape[1], t.shape[2]
    assert t.is_contiguous()
    if dtype == "rgb8":          # uint8 [H][W][S >= 3]: colour features, D = 27
        fm = FMap(t.data_ptr(), VQNNF_RGB8, H, W, 27, S, None)
        fm._tensor = t           # the device memory stays allocated while the map exists
        return fm
    scale = None
    if channel_scale is not None:
        channel_scale = np.ascontiguousarray(channel_scale, dtype=np.float32)
        scale = channel_scale.ctypes.data
    fm = FMap(t.data_ptr(), _DT[dtype], H, W, S, S, scale)
    fm._scale = channel_scale   # the host scales stay alive with the map
    fm._tensor = t              # and so does the device memory
    return fm


def bank_descs(bank):
    """Bank entries (x0, y0, x1, y1, gx, gy, weight[, bin_weight]) as C descs;
    bin_weight (gy x gx, or None) makes the entry one weighted filter.  The
    returned array keeps the weight arrays alive."""
    arr = (FilterDesc * len(bank))()
    keep = []
    for i, e in enumerate(bank):
        x0, y0, x1, y1, gx, gy, w = e[:7]
        bw = e[7] if len(e) > 7 else None
        ptr = None
        if bw is not None:
            a = np.ascontiguousarray(np.asarray(bw, dtype=np.float32).reshape(gy, gx))
            keep.append(a)
            ptr = a.ctypes.data
        arr[i] = FilterDesc(x0, y0, x1, y1, gx, gy, ptr, w)
    arr._keep = keep
    return arr


def default_bank(w: int, h: int, g: int):
    """Full window plus a g x g grid over it, each with weight 1."""
    return [(0, 0, w, h, 1, 1, 1.0), (0, 0, w, h, g, g, 1.0)]


VQNNF_BANK_GAUSS, VQNNF_BANK_2RECT, VQNNF_BANK_3RECT, VQNNF_BANK_23RECT = range(4)
_BANK_SETS = {"gauss": VQNNF_BANK_GAUSS, "2rect": VQNNF_BANK_2RECT, "3rect": VQNNF_BANK_3RECT,
              "23rect": VQNNF_BANK_23RECT}


def paper_bank(w: int, h: int, filter_set, n_scales: int):
    """vqnnf_paper_bank: the paper's Gaussian / Haar bank with sub-scales, as
    bank entries (x0, y0, x1, y1, 3, 3, weight, bin_weight[3][3])."""
    fs = _BANK_SETS[filter_set] if isinstance(filter_set, str) else int(filter_set)
    cap = 5 * max(n_scales, 1)
    arr = (FilterDesc * cap)()
    bw = np.zeros(9 * cap, dtype=np.float32)
    n = C.c_int32()
    _check(lib().vqnnf_paper_bank(w, h, fs, n_scales, arr, bw.ctypes.data, cap, C.byref(n)))
    return [(d.x0, d.y0, d.x1, d.y1, d.gx, d.gy, float(d.weight), bw[9 * i:9 * i + 9].reshape(3, 3).copy())
            for i, d in enumerate(arr[:n.value])]


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ------------------------------------------------------------------ handles

class Context:
    def __init__(self, stream=None, scratch_cap: int = 0, host: bool = False):
        h = C.c_void_p()
        if host:
            _check(lib().vqnnf_ctx_create_host(scratch_cap, C.byref(h)))
        else:
            _check(lib().vqnnf_ctx_create(_stream_ptr(stream), scratch_cap, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().vqnnf_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on: bool):
        _check(lib().vqnnf_ctx_set_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        n = 32
        names = (C.c_char_p * n)()
        launches = (C.c_int64 * n)()
        ms = (C.c_double * n)()
        cnt = C.c_int32()
        _check(lib().vqnnf_ctx_kernel_times(self.h, n, names, launches, ms, C.byref(cnt)))
        return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(min(n, cnt.value))}

    def reset_times(self):
        _check(lib().vqnnf_ctx_reset_times(self.h))


class Template:
    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx = ctx
        self.h = handle
        w, h, D, k, nf = (C.c_int32() for _ in range(5))
        _check(lib().vqnnf_template_info(handle, C.byref(w), C.byref(h), C.byref(D), C.byref(k),
                                         C.byref(nf)))
        self.w, self.h_, self.D, self.k, self.n_filters = w.value, h.value, D.value, k.value, nf.value

    @property
    def height(self):
        return self.h_

    def free(self):
        if self.h:
            lib().vqnnf_template_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def codebook(self) -> np.ndarray:
        out = np.empty((self.k, self.D), dtype=np.float32)
        _check(lib().vqnnf_template_codebook(self.h, out.ctypes.data))
        return out

    def labels(self) -> np.ndarray:
        out = np.empty((self.h_, self.w), dtype=np.uint8)
        _check(lib().vqnnf_template_labels(self.h, out.ctypes.data))
        return out

    def counts(self) -> np.ndarray:
        out = np.empty((self.n_filters, self.k), dtype=np.int32)
        _check(lib().vqnnf_template_counts(self.h, out.ctypes.data))
        return out

    def weights(self) -> np.ndarray:
        out = np.empty(self.n_filters, dtype=np.float32)
        _check(lib().vqnnf_template_weights(self.h, out.ctypes.data))
        return out

    def responses(self) -> np.ndarray:
        out = np.empty((self.n_filters, self.k), dtype=np.float32)
        _check(lib().vqnnf_template_responses(self.h, out.ctypes.data))
        return out


# ------------------------------------------------------------------ calls (C names)

def vqnnf_codebook(ctx: Context, template: np.ndarray, k: int, lloyd_iters: int, seed: int,
                   bank) -> Template:
    fm, keep = host_fmap(template)
    descs = bank_descs(bank)
    h = C.c_void_p()
    _check(lib().vqnnf_codebook(ctx.h, C.byref(fm), k, lloyd_iters, seed, descs, len(bank),
                                C.byref(h)))
    return Template(ctx, h)


def vqnnf_pca_fit(template: np.ndarray, d: int):
    """vqnnf_pca_fit: (mean [D], basis [d][D], variances [d]) of a host template."""
    fm, keep = host_fmap(template)
    mean = np.empty(fm.D, np.float32)
    basis = np.empty((d, fm.D), np.float32)
    var = np.empty(d, np.float32)
    _check(lib().vqnnf_pca_fit(C.byref(fm), d, mean.ctypes.data, basis.ctypes.data, var.ctypes.data))
    return mean, basis, var


def vqnnf_pca_project(ctx: Context, query: FMap, mean: np.ndarray, basis: np.ndarray, out) -> None:
    """vqnnf_pca_project into the device tensor `out` ([H][W][d] float32)."""
    m = np.ascontiguousarray(mean, np.float32)
    b = np.ascontiguousarray(basis, np.float32)
    _check(lib().vqnnf_pca_project(ctx.h, C.byref(query), m.ctypes.data, b.ctypes.data, b.shape[0],
                                   out.data_ptr()))


def vqnnf_codebook_batched(ctx: Context, templates: Sequence[np.ndarray], ks: Sequence[int],
                           lloyd_iters: int, seeds: Sequence[int], banks) -> list:
    """vqnnf_codebook_batched: one handle per template (host FP32 [h][w][D])."""
    n = len(templates)
    maps = [host_fmap(t) for t in templates]
    fms = (C.POINTER(FMap) * n)(*[C.pointer(m[0]) for m in maps])
    descs = [bank_descs(b) for b in banks]
    dps = (C.POINTER(FilterDesc) * n)(*[C.cast(d, C.POINTER(FilterDesc)) for d in descs])
    kk = (C.c_int32 * n)(*ks)
    ss = (C.c_uint64 * n)(*seeds)
    nd = (C.c_int32 * n)(*[len(b) for b in banks])
    out = (C.c_void_p * n)()
    _check(lib().vqnnf_codebook_batched(ctx.h, n, fms, kk, lloyd_iters, ss, dps, nd, out))
    return [Template(ctx, C.c_void_p(out[i])) for i in range(n)]


def vqnnf_template_from_codebook(ctx: Context, template: np.ndarray, codebook: np.ndarray,
                                 bank) -> Template:
    fm, keep = host_fmap(template)
    cb = np.ascontiguousarray(codebook, dtype=np.float32)
    descs = bank_descs(bank)
    h = C.c_void_p()
    _check(lib().vqnnf_template_from_codebook(ctx.h, C.byref(fm), cb.ctypes.data, cb.shape[0],
                                              descs, len(bank), C.byref(h)))
    return Template(ctx, h)


def vqnnf_assign(ctx: Context, tpl: Template, query: FMap, prec: int, labels) -> int:
    n = C.c_int64()
    _check(lib().vqnnf_assign(ctx.h, tpl.h, C.byref(query), prec, C.c_void_p(labels.data_ptr()),
                              C.byref(n)))
    return int(n.value)


def vqnnf_filter(ctx: Context, tpl: Template, labels, H: int, W: int, integral) -> None:
    _check(lib().vqnnf_filter(ctx.h, tpl.h, C.c_void_p(labels.data_ptr()), H, W,
                              C.c_void_p(integral.data_ptr())))


def _best_out(st, xy, sc):
    _check(st)
    return (int(xy[0]), int(xy[1])), float(sc.value)


def vqnnf_score(ctx: Context, tpl: Template, labels, H: int, W: int, heatmap):
    xy = (C.c_int32 * 2)()
    sc = C.c_float()
    st = lib().vqnnf_score(ctx.h, tpl.h, C.c_void_p(labels.data_ptr()), H, W,
                           C.c_void_p(heatmap.data_ptr()), xy, C.byref(sc))
    return _best_out(st, xy, sc)


def vqnnf_score_integral(ctx: Context, tpl: Template, integral, H: int, W: int, heatmap):
    xy = (C.c_int32 * 2)()
    sc = C.c_float()
    st = lib().vqnnf_score_integral(ctx.h, tpl.h, C.c_void_p(integral.data_ptr()), H, W,
                                    C.c_void_p(heatmap.data_ptr()), xy, C.byref(sc))
    return _best_out(st, xy, sc)


def vqnnf_match(ctx: Context, tpl: Template, query: FMap, prec: int, heatmap, want_best=True):
    if not want_best:
        _check(lib().vqnnf_match(ctx.h, tpl.h, C.byref(query), prec,
                                 C.c_void_p(heatmap.data_ptr()), None, None))
        return None
    xy = (C.c_int32 * 2)()
    sc = C.c_float()
    st = lib().vqnnf_match(ctx.h, tpl.h, C.byref(query), prec, C.c_void_p(heatmap.data_ptr()),
                           xy, C.byref(sc))
    return _best_out(st, xy, sc)


def vqnnf_match_noalloc(ctx: Context, tpl: Template, query: FMap, prec: int, heatmap, want_best=True):
    """vqnnf_match with every intermediate in the library's fixed device
    array (no device allocation); same results."""
    if not want_best:
        _check(lib().vqnnf_match_noalloc(ctx.h, tpl.h, C.byref(query), prec,
                                         C.c_void_p(heatmap.data_ptr()), None, None))
        return None
    xy = (C.c_int32 * 2)()
    sc = C.c_float()
    st = lib().vqnnf_match_noalloc(ctx.h, tpl.h, C.byref(query), prec, C.c_void_p(heatmap.data_ptr()),
                                   xy, C.byref(sc))
    return _best_out(st, xy, sc)


NOALLOC_SCRATCH_BYTES = 64 << 20


def vqnnf_ctx_set_debug_scores(ctx: Context, scores=None):
    """Test support: refined assignments on ctx also write their FP32 scores
    into the float32 device tensor `scores` ([n_pix][kpad]); None turns it off."""
    if scores is None:
        _check(lib().vqnnf_ctx_set_debug_scores(ctx.h, None, 0))
    else:
        _check(lib().vqnnf_ctx_set_debug_scores(ctx.h, C.c_void_p(scores.data_ptr()), scores.numel()))


def vqnnf_template_score_bound(tpl: Template, dtype: str, channel_scale=None):
    """(a0, a1, a2, A0, A1) of the refined search's bound for maps of `dtype`."""
    out = np.zeros(5, dtype=np.float64)
    sc = None if channel_scale is None else np.ascontiguousarray(channel_scale, dtype=np.float32)
    _check(lib().vqnnf_template_score_bound(tpl.h, _DT[dtype], sc.ctypes.data if sc is not None else None,
                                            out.ctypes.data))
    return tuple(float(v) for v in out)


def vqnnf_ctx_set_tune_file(ctx: Context, path):
    """Persist (and load) the context's tuning results in a text file."""
    _check(lib().vqnnf_ctx_set_tune_file(ctx.h, None if path is None else str(path).encode()))


def vqnnf_batched_labels(ctx: Context, pair: int, labels):
    """Copies pair `pair`'s label map of the last batched call into the
    device tensor `labels` (uint8, H*W), on the context stream."""
    _check(lib().vqnnf_batched_labels(ctx.h, pair, C.c_void_p(labels.data_ptr())))


def vqnnf_match_batched(ctx: Context, templates: Sequence[Template], queries: Sequence[FMap],
                        prec: int, heatmaps, want_best=True):
    """Pairs (templates[i], queries[i]) -> heatmaps[i]; returns [((x, y), score)] or None."""
    n = len(templates)
    if len(queries) != n or len(heatmaps) != n:
        raise ValueError("templates, queries and heatmaps must have the same length")
    th = (C.c_void_p * n)(*[t.h for t in templates])
    qarr = (FMap * n)(*queries)
    qp = (C.POINTER(FMap) * n)(*[C.pointer(qarr[i]) for i in range(n)])
    hp = (C.c_void_p * n)(*[h.data_ptr() for h in heatmaps])
    if not want_best:
        _check(lib().vqnnf_match_batched(ctx.h, n, th, qp, prec, hp, None, None))
        return None
    xy = (C.c_int32 * (2 * n))()
    sc = (C.c_float * n)()
    _check(lib().vqnnf_match_batched(ctx.h, n, th, qp, prec, hp, xy, sc))
    return [((xy[2 * i], xy[2 * i + 1]), sc[i]) for i in range(n)]


def vqnnf_ctx_set_autotune(ctx: Context, enable: bool) -> None:
    _check(lib().vqnnf_ctx_set_autotune(ctx.h, 1 if enable else 0))


def vqnnf_ctx_set_graph(ctx: Context, enable: bool) -> None:
    _check(lib().vqnnf_ctx_set_graph(ctx.h, 1 if enable else 0))


def vqnnf_version() -> str:
    return lib().vqnnf_version().decode()

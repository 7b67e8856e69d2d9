"""Seeded synthetic workloads for VQ-NNF template matching.

This module only draws inputs: feature maps from a spatially smooth Gaussian
mixture, their storage encodings (FP32, BF16, FP8 E4M3FN with per-channel
scales) and template crops planted at seeded offsets.  It holds none of the
matching method's arithmetic (no distances, no integral images, no scores), so
the product path and the FP64 oracle can both consume its output without
sharing any of the computation they are compared on.

The paper measures on BBS (320x480 / 320x240 frames, colour D=27 or ResNet-18
D=512 features) and TinyTLP / TLPattr (1280x720) (Sec. 5.1, 5.2).  Those
datasets are not available; these generators stand in for them with the shapes
of the paper's low- and high-resolution workloads.

Recipe (every random draw comes from numpy PCG64 streams spawned from one
master seed, so a (config, seed) pair fixes every byte):
  1. mixture means mu_m ~ N(0, I_D), m < M;
  2. a component label field: z0 ~ U{0..M-1} per pixel, then each pixel takes
     the component with the largest count in its 5x5 neighbourhood (clipped at
     the border); ties are broken by a seeded hash jitter in [0, 0.5);
  3. features q = mu_z + sigma * eps, eps ~ N(0, I_D), in FP32;
  4. storage encoding (RNE): FP32, BF16, or FP8 E4M3FN with a per-channel
     scale s_d = max|q_d| / 448;
  5. templates are crops of the *decoded* query at seeded offsets, optionally
     rotated by a multiple of 90 degrees, plus N(0, 0.1^2) noise, stored FP32.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

MASTER_SEED = 230615010

_MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser on a uint64 array (used only as a tie-break hash)."""
    with np.errstate(over="ignore"):
        x = (x + np.uint64(0x9E3779B97F4A7C15)) & _MASK64
        x = ((x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _MASK64
        x = ((x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _MASK64
        return x ^ (x >> np.uint64(31))


def smooth_label_field(H: int, W: int, M: int, rng: np.random.Generator) -> np.ndarray:
    """Spatially smooth component labels (int32 [H][W]).

    z0 is drawn per pixel; every pixel then takes the component with the most
    occurrences of z0 in its 5x5 window (zero padding: outside pixels do not
    count), with a seeded jitter in [0, 0.5) per (pixel, component) breaking
    ties without reordering unequal counts.
    """
    z0 = rng.integers(0, M, size=(H, W), dtype=np.int32)
    key = np.uint64(int(rng.integers(0, 2**63 - 1)))
    pad = np.full((H + 4, W + 4), -1, dtype=np.int32)
    pad[2:-2, 2:-2] = z0
    cands = [pad[dy:dy + H, dx:dx + W] for dy in range(5) for dx in range(5)]
    pix = (np.arange(H, dtype=np.uint64)[:, None] * np.uint64(W)
           + np.arange(W, dtype=np.uint64)[None, :])
    best_score = np.full((H, W), -1.0, dtype=np.float64)
    best = np.zeros((H, W), dtype=np.int32)
    for c in cands:
        cnt = np.zeros((H, W), dtype=np.int32)
        for o in cands:
            cnt += (o == c)
        valid = c >= 0
        h = _mix64(key ^ (pix * np.uint64(M) + np.where(valid, c, 0).astype(np.uint64)))
        jit = (h >> np.uint64(11)).astype(np.float64) * (0.5 / 2.0**53)
        score = np.where(valid, cnt + jit, -1.0)
        upd = score > best_score
        best_score = np.where(upd, score, best_score)
        best = np.where(upd, c, best)
    return best


def mixture_features(z: np.ndarray, means: np.ndarray, sigma: float,
                     rng: np.random.Generator) -> np.ndarray:
    """q = mu_z + sigma * eps in FP32, HWC layout."""
    H, W = z.shape
    D = means.shape[1]
    out = np.empty((H, W, D), dtype=np.float32)
    mu32 = means.astype(np.float32)
    rows = max(1, (1 << 22) // max(1, W * D))
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        eps = rng.standard_normal(size=(y1 - y0, W, D), dtype=np.float32)
        np.multiply(eps, np.float32(sigma), out=eps)
        np.add(np.take(mu32, z[y0:y1], axis=0), eps, out=out[y0:y1])
    return out


# ---------------------------------------------------------------- encodings

def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 to BF16 (round to nearest even); returns the uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    r = (u + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def _e4m3_values() -> np.ndarray:
    """Value of each E4M3FN code 0..255 (NaN for 0x7F/0xFF), float64."""
    v = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            v[code] = np.nan
        elif e == 0:
            v[code] = s * (m / 8.0) * 2.0 ** -6
        else:
            v[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return v


_E4M3 = _e4m3_values()
_E4M3_POS = _E4M3[:0x7F]  # codes 0x00..0x7E, increasing, 0 .. 448


def f32_to_e4m3fn(x: np.ndarray) -> np.ndarray:
    """Encode finite values to OCP E4M3FN codes: round to nearest even,
    saturating at +-448.  |x| >= 2^-6 (normal codes): the binary64 pattern
    rounded to 3 mantissa bits, ties to even, by integer addition (a carry
    out of the mantissa moves into the exponent), exponent rebiased from 1023
    to 7; |x| < 2^-6: rint(|x| * 2^9) on the subnormal 2^-9 grid.  Returns
    the same codes as the frexp form below, several times faster."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    np.minimum(a, 448.0, out=a)
    b = a.view(np.int64)
    r = b >> 49
    r &= 1
    r += b
    r += (1 << 48) - 1
    r >>= 49
    r -= (1023 - 7) << 3
    small = a < 2.0 ** -6
    if small.any():
        r[small] = np.rint(a[small] * 512.0).astype(np.int64)
    code = r.astype(np.uint8)            # every code is in 0..0x7E here
    code[(x < 0) & (code != 0)] |= np.uint8(0x80)
    return code


def f32_to_e4m3fn_frexp(x: np.ndarray) -> np.ndarray:
    """The same encoding written with frexp: |x| = m * 2^e with m in [1, 2):
    normal codes (e >= -6) keep rint(8m) in [8, 16] (16 carries into the
    exponent), subnormals rint(|x| * 2^9) on the 2^-9 grid."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    m, e = np.frexp(a)                          # a = m * 2^e, m in [0.5, 1)
    e = e - 1
    q = np.rint(np.ldexp(m, 4))                 # 8 * (2m), in [8, 16]
    carry = q == 16
    q = np.where(carry, 8, q).astype(np.int64)
    e = np.where(carry, e + 1, e)
    code = np.where(e >= -6, ((e + 7) << 3) + (q - 8), np.rint(np.ldexp(a, 9)).astype(np.int64))
    code = np.where(a == 0, 0, np.minimum(code, 0x7E)).astype(np.uint8)
    neg = (x < 0) & (code != 0)
    return np.where(neg, code | np.uint8(0x80), code).astype(np.uint8)


def e4m3fn_to_f64(code: np.ndarray) -> np.ndarray:
    return _E4M3[np.asarray(code, dtype=np.uint8)]


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass
class QueryMap:
    """One query feature map in its storage encoding (HWC)."""
    H: int
    W: int
    D: int
    dtype: str                    # "f32" | "bf16" | "fp8"
    data: np.ndarray              # f32 [H,W,D] | uint16 bits | uint8 codes
    scale: Optional[np.ndarray]   # fp8 only: float32 [D]

    def decoded_f32(self) -> np.ndarray:
        """Decoded values as float32 where exact (f32/bf16); fp8 values may
        need more than 24 bits (scale * code) and are given as float64."""
        if self.dtype == "f32":
            return self.data
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.data)
        return e4m3fn_to_f64(self.data) * self.scale.astype(np.float64)


@dataclasses.dataclass
class Template:
    data: np.ndarray              # float32 [h][w][D]
    x0: int                       # planted offset in its query map
    y0: int
    rot: int                      # multiple of 90 degrees applied
    k: int
    grid: int


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    maps: List[QueryMap]
    templates: List[List[Template]]   # templates[i] are matched against maps[i]
    lloyd_iters: int = 20


def encode(q: np.ndarray, dtype: str) -> QueryMap:
    H, W, D = q.shape
    if dtype == "f32":
        return QueryMap(H, W, D, "f32", np.ascontiguousarray(q, dtype=np.float32), None)
    if dtype == "bf16":
        return QueryMap(H, W, D, "bf16", f32_to_bf16_bits(q), None)
    if dtype == "fp8":
        amax = np.abs(q).reshape(-1, D).max(axis=0).astype(np.float64)
        scale = np.where(amax > 0, amax / 448.0, 1.0).astype(np.float32)
        codes = np.empty((H, W, D), dtype=np.uint8)
        s64 = scale.astype(np.float64)
        for y in range(H):
            codes[y] = f32_to_e4m3fn(q[y].astype(np.float64) / s64)
        return QueryMap(H, W, D, "fp8", codes, scale)
    raise ValueError(dtype)


def _crop(qm: QueryMap, x0: int, y0: int, w: int, h: int) -> np.ndarray:
    if qm.dtype == "f32":
        return qm.data[y0:y0 + h, x0:x0 + w].astype(np.float32)
    if qm.dtype == "bf16":
        return bf16_bits_to_f32(qm.data[y0:y0 + h, x0:x0 + w])
    v = e4m3fn_to_f64(qm.data[y0:y0 + h, x0:x0 + w]) * qm.scale.astype(np.float64)
    return v.astype(np.float32)


def _streams(seed: int, n: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def make_single(name: str, seed: int, H: int, W: int, D: int, M: int, sigma: float,
                dtype: str, side: int, k: int, grid: int, noise: float = 0.1,
                rotate: bool = False, occlude: float = 0.0) -> Workload:
    """One query map, one planted template."""
    r_means, r_lab, r_feat, r_place, r_tnoise, r_occ = _streams(seed, 6)
    means = r_means.standard_normal(size=(M, D))
    z = smooth_label_field(H, W, M, r_lab)
    q = mixture_features(z, means, sigma, r_feat)
    qm = encode(q, dtype)
    x0 = int(r_place.integers(0, W - side + 1))
    y0 = int(r_place.integers(0, H - side + 1))
    t = _crop(qm, x0, y0, side, side)
    rot = 0
    if rotate:
        rot = int(r_place.integers(0, 4))
        t = np.ascontiguousarray(np.rot90(t, rot, axes=(0, 1)))
    if noise > 0:
        t = (t + np.float32(noise) * r_tnoise.standard_normal(size=t.shape, dtype=np.float32))
    t = np.ascontiguousarray(t, dtype=np.float32)
    if occlude > 0:
        n = side * side
        m = int(round(occlude * n))
        idx = r_occ.choice(n, size=m, replace=False)
        comp = r_occ.integers(0, M, size=m)
        vals = (means[comp].astype(np.float32)
                + np.float32(sigma) * r_occ.standard_normal(size=(m, D), dtype=np.float32))
        enc = encode(vals.reshape(m, 1, D), dtype) if dtype != "fp8" else None
        ys = y0 + idx // side
        xs = x0 + idx % side
        if dtype == "fp8":
            s64 = qm.scale.astype(np.float64)
            qm.data[ys, xs] = f32_to_e4m3fn(vals.astype(np.float64) / s64)
        else:
            qm.data[ys, xs] = enc.data[:, 0, :]
    tpl = Template(t, x0, y0, rot, k, grid)
    return Workload(name, seed, [qm], [[tpl]])


CONFIGS = ("c1", "c2", "c3", "c4", "c5")


def make_config(name: str, seed: Optional[int] = None, scale_down: int = 1, progress=None,
                maps: Optional[List[int]] = None) -> Workload:
    """Workloads shaped like the five benchmark configurations.

    c1: 64x64, D=27, FP32, 32 components, 16x16 template, k=8, full + 2x2 grid.
    c2: 512x512, D=64, FP32, 64 components, 48x48 template rotated by a seeded
        multiple of 90 degrees, k=32, full + 3x3 grid.
    c3: 1024x1024, D=512, BF16, 128 components, 96x96 template planted with 20%
        of the crop's query pixels replaced by occluder draws, k=128, full + 3x3.
    c4: 1024x1024, D=256, BF16; 64 templates, sides U{24..160}, k in
        {16,32,64,128}, full + 2x2 grid.
    c5: 32 maps with sides U{256,320,...,2048}, D=256, FP8 E4M3FN with
        per-channel scales, 128 components; 4 templates per map, sides
        U{32..128}, k=64, full + 3x3 grid.
    `scale_down` divides map sides (tests use it for reduced-size variants);
    `progress(done, total)`, if given, is called as the maps of c5 are made;
    `maps` (c5 only) makes just those maps (each map has its own streams, so a
    subset is the same bytes as in the whole set).
    """
    idx = CONFIGS.index(name)
    if seed is None:
        seed = MASTER_SEED + idx
    s = scale_down
    if name == "c1":
        return make_single("c1", seed, 64 // s, 64 // s, 27, 32, 0.3, "f32", 16, 8, 2)
    if name == "c2":
        return make_single("c2", seed, 512 // s, 512 // s, 64, 64, 0.3, "f32", 48, 32, 3,
                           rotate=True)
    if name == "c3":
        return make_single("c3", seed, 1024 // s, 1024 // s, 512, 128, 0.3, "bf16", 96, 128, 3,
                           noise=0.0, occlude=0.2)
    if name == "c4":
        return make_multi_template(seed, 1024 // s, 1024 // s, 256, 128, 0.3, "bf16", 64,
                                   (24, 160), (16, 32, 64, 128), 2)
    if name == "c5":
        return make_multi_map(seed, 32, (256 // s, 2048 // s), 256, 128, 0.3, "fp8", 4,
                              (32, 128), 64, 3, progress=progress, only=maps)
    raise ValueError(name)


def make_multi_template(seed, H, W, D, M, sigma, dtype, n_t, side_rng, k_choices, grid,
                        noise=0.1) -> Workload:
    r_means, r_lab, r_feat, r_place, r_tnoise = _streams(seed, 5)
    means = r_means.standard_normal(size=(M, D))
    z = smooth_label_field(H, W, M, r_lab)
    qm = encode(mixture_features(z, means, sigma, r_feat), dtype)
    tpls = []
    lo, hi = side_rng
    hi = min(hi, H, W)
    lo = min(lo, hi)
    for _ in range(n_t):
        side = int(r_place.integers(lo, hi + 1))
        k = int(r_place.choice(np.asarray(k_choices)))
        x0 = int(r_place.integers(0, W - side + 1))
        y0 = int(r_place.integers(0, H - side + 1))
        t = _crop(qm, x0, y0, side, side)
        t = t + np.float32(noise) * r_tnoise.standard_normal(size=t.shape, dtype=np.float32)
        tpls.append(Template(np.ascontiguousarray(t, dtype=np.float32), x0, y0, 0, k, grid))
    return Workload("c4", seed, [qm], [tpls])


def _multi_map_one(job):
    """One map of make_multi_map and its templates (a process-pool job)."""
    map_seed, H, W, D, M, sigma, dtype, means, t_per_map, tside_rng, k, grid, noise = job
    r_lab, r_feat, r_place, r_tnoise = _streams(map_seed, 4)
    z = smooth_label_field(H, W, M, r_lab)
    qm = encode(mixture_features(z, means, sigma, r_feat), dtype)
    row = []
    tlo, thi = tside_rng
    thi = min(thi, H, W)
    tlo = min(tlo, thi)
    for _ in range(t_per_map):
        side = int(r_place.integers(tlo, thi + 1))
        x0 = int(r_place.integers(0, W - side + 1))
        y0 = int(r_place.integers(0, H - side + 1))
        t = _crop(qm, x0, y0, side, side)
        t = t + np.float32(noise) * r_tnoise.standard_normal(size=t.shape, dtype=np.float32)
        row.append(Template(np.ascontiguousarray(t, dtype=np.float32), x0, y0, 0, k, grid))
    return qm, row


def make_multi_map(seed, n_maps, side_rng, D, M, sigma, dtype, t_per_map, tside_rng, k, grid,
                   noise=0.1, progress=None, only=None) -> Workload:
    r_means, r_sizes, *r_maps = _streams(seed, 2 + n_maps)
    means = r_means.standard_normal(size=(M, D))
    lo, hi = side_rng
    sides = np.arange(lo, hi + 1, 64) if lo % 64 == 0 and hi % 64 == 0 else np.arange(lo, hi + 1)
    jobs = []
    for i in range(n_maps):
        H = int(r_sizes.choice(sides))
        W = int(r_sizes.choice(sides))
        jobs.append((int(r_maps[i].integers(0, 2**62)), H, W, D, M, sigma, dtype, means, t_per_map,
                     tside_rng, k, grid, noise))
    if only is not None:
        jobs = [jobs[i] for i in only]
        n_maps = len(jobs)
    # every map has its own streams, so maps can be made in any order; large
    # workloads use a pool of fresh interpreters
    total = sum(j[1] * j[2] for j in jobs) * D
    if total > (1 << 28) and n_maps > 1:
        import multiprocessing as mp
        import os
        n = max(1, min(16, len(os.sched_getaffinity(0)), n_maps))
        with mp.get_context("spawn").Pool(n) as pool:
            done = []
            for d in pool.imap(_multi_map_one, jobs, chunksize=1):
                done.append(d)
                if progress:
                    progress(len(done), n_maps)
    else:
        done = []
        for j in jobs:
            done.append(_multi_map_one(j))
            if progress:
                progress(len(done), n_maps)
    maps = [d[0] for d in done]
    tpls = [d[1] for d in done]
    return Workload("c5", seed, maps, tpls)


def random_map(H: int, W: int, D: int, dtype: str, seed: int, M: int = 16,
               sigma: float = 0.3) -> QueryMap:
    """A small smooth-mixture map for unit tests."""
    r_means, r_lab, r_feat = _streams(seed, 3)
    means = r_means.standard_normal(size=(M, D))
    z = smooth_label_field(H, W, M, r_lab)
    return encode(mixture_features(z, means, sigma, r_feat), dtype)


def rgb_image(H: int, W: int, seed: int, M: int = 12, noise: float = 8.0, cell: int = 8) -> np.ndarray:
    """A seeded uint8 RGB image [H, W, 3] of colour regions: the component
    field of the feature maps drawn at 1/cell resolution and enlarged to
    cell x cell blocks, one palette colour per component, plus Gaussian
    noise, clipped to 0..255 (stand-in for the colour images of the
    colour-feature workloads)."""
    r_pal, r_lab, r_noise = _streams(seed, 3)
    palette = r_pal.uniform(20.0, 235.0, size=(M, 3))
    zc = smooth_label_field(-(-H // cell), -(-W // cell), M, r_lab)
    z = np.repeat(np.repeat(zc, cell, axis=0), cell, axis=1)[:H, :W]
    img = palette[z] + noise * r_noise.standard_normal(size=(H, W, 3))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)

"""FP64 CPU oracle for VQ-NNF template matching (Gupta & Sintorn, arXiv 2306.15010).

TEST INFRASTRUCTURE ONLY.  This module is the parity target for the GPU path.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does.  It shares no code, tables or helpers
with the GPU library and imports nothing from it.

It is deliberately plain and slow: every quantity is computed from its
definition in float64 (or exact integers), in the order stated below, with
numpy elementwise operations (each correctly rounded) and explicit loops where
the order of a floating-point sum matters.  numpy reductions such as `sum` are
never used on floats, since they sum pairwise.

Contents and the passages they follow:
  O1  decode of stored values (FP32 / BF16 / FP8 E4M3FN x per-channel scale;
      RGB images as 3x3 colour patches, Sec. 5.2 "Feature Extraction");
      O1b PCA reduction of the features (Sec. 5.5)
  O2  k-means codebook: seeded k-means++ then Lloyd (Sec. 3.1, Sec. 4 "K-means
      computation", Sec. 5.2 "Codebook and NNF Generation")
  O3  nearest-codeword assignment (Alg. 1, Sec. 3.1; exact L2 NN, Sec. 5.2)
  O4  one-hot integral image (Sec. 3.1; Supp. S.2, definition and box sum)
  O5  filter regions and Alg. 2's dilation filter (Sec. 3.2.1, Supp. S.4);
      O5b the paper's Gaussian / Haar coarse filters and sub-scale regions
      (Sec. 3.2.2, Sec. 3.3, Sec. 5.2 "Filtering")
  O6  template representation R(tau) (Sec. 3.3)
  O7  similarity, eq. 2 (Sec. 3.3)
  O8  localisation: argmax of the heatmap (Sec. 4 "Target Localization")

Readings where the paper is silent or ambiguous (each also listed in the
design notes):
  * distance is the squared L2 norm (same argmin as L2);
  * nearest-neighbour ties go to the lowest codeword index;
  * FP64 distance order: d = sum_t (q_t - c_t)^2, accumulated sequentially in
    t starting from 0, with separate subtract, multiply and add (no FMA);
  * the integral image is stored exclusive and zero padded: P[y][x][j] counts
    label j over rows < y and columns < x, so the paper's inclusive value at
    (x, y) is P[y+1][x+1] and a box [x0,x1) x [y0,y1) is
    P[y1][x1] - P[y0][x1] - P[y1][x0] + P[y0][x0];
  * heatmap entries are indexed by the window's top-left corner and only
    windows fully inside the query are scored: (H-h+1) x (W-w+1);
  * grid bins of a region of width w split at floor(a*w/g), a = 0..g;
  * |.| in eq. 2 is the L1 norm over the k channels;
  * an indicator bin's weight is the filter weight divided by
    (number of bins x bin area), so each term compares two distributions;
  * localisation ties go to the lowest y, then the lowest x.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# O1: decoding stored values.  Every stored element has an exact float64 value.

def decode_f32(x: np.ndarray) -> np.ndarray:
    """FP32 -> float64 (exact)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def decode_bf16(bits: np.ndarray) -> np.ndarray:
    """BF16 bit patterns -> float64 (exact): a BF16 value is the FP32 value
    whose upper 16 bits are the pattern and whose lower 16 bits are zero."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def e4m3fn_value(code: int) -> float:
    """Value of one OCP E4M3FN code: 1 sign bit, 4 exponent bits (bias 7),
    3 mantissa bits; exponent field 0 is subnormal; S.1111.111 is NaN and
    there are no infinities, so the largest finite magnitude is 448."""
    sign = -1.0 if (code >> 7) & 1 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return math.nan
    if e == 0:
        return sign * math.ldexp(m, -9)          # m/8 * 2^-6
    return sign * math.ldexp(8 + m, e - 10)      # (1 + m/8) * 2^(e-7)


E4M3FN_TABLE = np.array([e4m3fn_value(c) for c in range(256)], dtype=np.float64)


def decode_e4m3fn(codes: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """FP8 element value = double(scale[d]) * double(e4m3fn(code)).  The
    product of a 24-bit and a 4-bit significand fits in 53 bits: exact."""
    v = E4M3FN_TABLE[np.asarray(codes, dtype=np.uint8)]
    return v * np.asarray(scale, dtype=np.float32).astype(np.float64)


def rgb_patch_features(img: np.ndarray) -> np.ndarray:
    """Colour features (Sec. 5.2 "Feature Extraction"): every pixel's 3x3
    neighbourhood of RGB values, 27 per pixel.  img: uint8 [H, W, 3].
    Readings: feature t = (3*dy + dx)*3 + c holds channel c of the pixel at
    offset (dx - 1, dy - 1), dx, dy in {0, 1, 2}; neighbours outside the image
    take the nearest pixel inside (edge replication); values are the raw
    0..255 integers (exact).  Returns float64 [H, W, 27]."""
    im = np.asarray(img, dtype=np.uint8)
    H, W, C = im.shape
    if C != 3:
        raise ValueError("RGB image expected")
    out = np.zeros((H, W, 27), dtype=np.float64)
    for dy in range(3):
        ys = np.clip(np.arange(H) + dy - 1, 0, H - 1)
        for dx in range(3):
            xs = np.clip(np.arange(W) + dx - 1, 0, W - 1)
            for c in range(3):
                out[:, :, (3 * dy + dx) * 3 + c] = im[ys][:, xs, c].astype(np.float64)
    return out


def decode(dtype: str, data: np.ndarray, scale: Optional[np.ndarray] = None) -> np.ndarray:
    if dtype == "f32":
        return decode_f32(data)
    if dtype == "bf16":
        return decode_bf16(data)
    if dtype == "fp8":
        return decode_e4m3fn(data, scale)
    if dtype == "rgb8":
        return rgb_patch_features(data)
    raise ValueError(dtype)


# --------------------------------------------------------------------------
# O1b: dimensionality reduction (Sec. 5.5): PCA of the template's features.
#
# Readings (the paper names only "PCA" and the target sizes 9 and 18): the
# principal axes are fitted on the template's pixels (mean-centred, covariance
# normalised by the pixel count), the d axes of largest variance in
# decreasing order, each with its largest-magnitude component positive (the
# first such component on ties); template and query are both projected onto
# them after subtracting the template mean.

def pca_fit(x: np.ndarray, d: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """x: float64 [n, D] -> (mean [D], basis [d, D], variances [d])."""
    x = np.asarray(x, dtype=np.float64)
    n, D = x.shape
    mean = np.zeros(D)
    for i in range(n):                      # sequential sum in point order
        mean = mean + x[i]
    mean = mean / float(n)
    xc = x - mean
    cov = (xc.T @ xc) / float(n)            # library matmul: a step, not the method
    w, v = np.linalg.eigh(cov)              # ascending eigenvalues
    order = np.argsort(-w, kind="stable")[:d]
    basis = v[:, order].T.copy()
    for r in range(d):
        j = int(np.argmax(np.abs(basis[r])))
        if basis[r, j] < 0:
            basis[r] = -basis[r]
    return mean, basis, w[order]


def pca_project(x: np.ndarray, mean: np.ndarray, basis: np.ndarray) -> np.ndarray:
    """(x - mean) . basis^T for every row of x [..., D] -> [..., d]."""
    return (np.asarray(x, dtype=np.float64) - mean) @ np.asarray(basis, dtype=np.float64).T


# --------------------------------------------------------------------------
# O3: squared distances in the fixed FP64 order, and the NN assignment.

def sq_distances(points: np.ndarray, centres: np.ndarray) -> np.ndarray:
    """d[p, j] = sum_t (x[p,t] - c[j,t])^2, float64, accumulated sequentially
    over t from 0 with separate subtract, multiply and add.

    points: float64 [n, D]; centres: float64 [k, D] -> float64 [n, k].
    """
    x = np.asarray(points, dtype=np.float64)
    c = np.asarray(centres, dtype=np.float64)
    n, D = x.shape
    k = c.shape[0]
    acc = np.zeros((n, k), dtype=np.float64)
    for t in range(D):
        diff = x[:, t:t + 1] - c[None, :, t]
        sq = diff * diff
        acc = acc + sq
    return acc


def assign(points: np.ndarray, codebook: np.ndarray, chunk: int = 16384) -> np.ndarray:
    """Alg. 1: index of the nearest codeword of every point (lowest index on
    ties).  points float64 [n, D]; codebook float64 [k, D] -> int64 [n]."""
    x = np.asarray(points, dtype=np.float64)
    out = np.empty(x.shape[0], dtype=np.int64)
    for s in range(0, x.shape[0], chunk):
        d = sq_distances(x[s:s + chunk], codebook)
        out[s:s + chunk] = np.argmin(d, axis=1)   # first minimum = lowest index
    return out


def assign_map(fmap: np.ndarray, codebook: np.ndarray) -> np.ndarray:
    """NNF of a feature map: fmap float64 [H, W, D] -> labels int64 [H, W]."""
    H, W, D = fmap.shape
    return assign(fmap.reshape(H * W, D), codebook).reshape(H, W)


# --------------------------------------------------------------------------
# O2: k-means codebook.

class SplitMix64:
    """Vigna's splitmix64 generator; u01() = (next >> 11) * 2^-53."""

    def __init__(self, seed: int):
        self.state = seed & 0xFFFFFFFFFFFFFFFF

    def next(self) -> int:
        m = 0xFFFFFFFFFFFFFFFF
        self.state = (self.state + 0x9E3779B97F4A7C15) & m
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        return z ^ (z >> 31)

    def u01(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53


def _uniform_index(u: float, n: int) -> int:
    return min(int(math.floor(u * n)), n - 1)


def _seq_sum(v: np.ndarray) -> float:
    """Sequential float64 sum from 0 (np.add.accumulate is a running sum)."""
    if v.size == 0:
        return 0.0
    return float(np.add.accumulate(np.asarray(v, dtype=np.float64))[-1])


def kmeans_pp_init(x: np.ndarray, k: int, rng: SplitMix64) -> np.ndarray:
    """k-means++ seeding: the first centre uniformly; each next centre is the
    point i drawn with probability proportional to D^2(x_i), the squared
    distance to the nearest chosen centre.  The draw takes u = rng.u01() and
    returns the smallest i whose sequential running sum of D^2 exceeds u * S,
    S being the sequential total.  If S == 0 the point is drawn uniformly."""
    n = x.shape[0]
    centres = np.empty((k, x.shape[1]), dtype=np.float64)
    first = _uniform_index(rng.u01(), n)
    centres[0] = x[first]
    d2 = sq_distances(x, centres[0:1])[:, 0]
    for i in range(1, k):
        csum = np.add.accumulate(d2)
        total = float(csum[-1])
        u = rng.u01()
        if total == 0.0:
            idx = _uniform_index(u, n)
        else:
            target = u * total
            hit = np.nonzero(csum > target)[0]
            idx = int(hit[0]) if hit.size else int(np.nonzero(d2 > 0)[0][-1])
        centres[i] = x[idx]
        d_new = sq_distances(x, centres[i:i + 1])[:, 0]
        d2 = np.minimum(d2, d_new)
    return centres


def lloyd(x: np.ndarray, centres: np.ndarray, iters: int,
          history: Optional[list] = None) -> np.ndarray:
    """`iters` Lloyd iterations: assign every point with O3's rule, then move
    each centre to the sequential FP64 mean of its points in point order (sum
    from 0, then one division by the count).  An empty cluster keeps its
    centre.  If `history` is a list, the k-means objective (sequential sum of
    each point's squared distance to its centre) before every update and
    after the last is appended."""
    c = np.array(centres, dtype=np.float64, copy=True)
    for _ in range(iters):
        d = sq_distances(x, c)
        lab = np.argmin(d, axis=1)
        if history is not None:
            history.append(_seq_sum(d[np.arange(x.shape[0]), lab]))
        for j in range(c.shape[0]):
            idx = np.nonzero(lab == j)[0]
            if idx.size == 0:
                continue
            s = np.add.accumulate(x[idx], axis=0)[-1]
            c[j] = s / float(idx.size)
    if history is not None:
        d = sq_distances(x, c)
        history.append(_seq_sum(d.min(axis=1)))
    return c


def kmeans_codebook(template: np.ndarray, k: int, iters: int = 20, seed: int = 0,
                    return_f64: bool = False):
    """Codebook of a template (Sec. 3.1): k-means of its w*h feature vectors,
    taken in row-major order, from seeded k-means++ and `iters` Lloyd
    iterations, rounded to FP32 at the end.  template: float [h, w, D]."""
    t = np.asarray(template, dtype=np.float32).astype(np.float64)
    x = t.reshape(-1, t.shape[-1])
    rng = SplitMix64(seed)
    c0 = kmeans_pp_init(x, k, rng)
    c = lloyd(x, c0, iters)
    c32 = c.astype(np.float32)
    return (c32, c) if return_f64 else c32


# --------------------------------------------------------------------------
# O4: integral image of the one-hot label map.

def one_hot(labels: np.ndarray, k: int) -> np.ndarray:
    lab = np.asarray(labels)
    return (lab[..., None] == np.arange(k)[None, None, :]).astype(np.int64)


def integral_image(labels: np.ndarray, k: int) -> np.ndarray:
    """P[y][x][j] = #{(x', y') : y' < y, x' < x, label(x', y') = j}, int64,
    shape (H+1, W+1, k).  Supp. S.2 defines the inclusive sum; P is its
    exclusive, zero-padded form (the paper's value at (x, y) is P[y+1][x+1])."""
    oh = one_hot(labels, k)
    H, W = oh.shape[:2]
    P = np.zeros((H + 1, W + 1, k), dtype=np.int64)
    P[1:, 1:] = np.cumsum(np.cumsum(oh, axis=0), axis=1)
    return P


def box_sum(P: np.ndarray, x0: int, y0: int, x1: int, y1: int) -> np.ndarray:
    """Supp. S.2 box sum over columns [x0, x1) and rows [y0, y1)."""
    return P[y1, x1] - P[y0, x1] - P[y1, x0] + P[y0, x0]


# --------------------------------------------------------------------------
# O5: filter regions, indicator bins and Alg. 2.

@dataclass
class FilterDesc:
    """A rectangular region of the template, [x0, x1) x [y0, y1), split into a
    gx x gy grid.  bin_weight None: every bin is its own indicator filter with
    weight `weight / (gx*gy*area(bin))`.  Otherwise one filter whose response
    is sum_bins bin_weight[b][a] * count(bin) / area(region) (eq. 1's
    normaliser), scored with weight `weight`."""
    x0: int
    y0: int
    x1: int
    y1: int
    gx: int = 1
    gy: int = 1
    bin_weight: Optional[np.ndarray] = None
    weight: float = 1.0


def grid_edges(lo: int, hi: int, g: int) -> List[int]:
    """Bin boundaries lo + floor(a*(hi-lo)/g), a = 0..g (an exact partition)."""
    n = hi - lo
    return [lo + (a * n) // g for a in range(g + 1)]


@dataclass
class Filter:
    """One expanded filter: a list of (coefficient, x0, y0, x1, y1) boxes."""
    boxes: List[Tuple[float, int, int, int, int]]
    weight: float
    integer: bool          # response is an integer count (single box, coef 1)


def default_bank(w: int, h: int, g: int) -> List[FilterDesc]:
    """The benchmark bank: the full window plus a g x g grid of sub-windows."""
    return [FilterDesc(0, 0, w, h, 1, 1, None, 1.0), FilterDesc(0, 0, w, h, g, g, None, 1.0)]


def expand_bank(bank: Sequence[FilterDesc]) -> List[Filter]:
    out: List[Filter] = []
    for d in bank:
        xs = grid_edges(d.x0, d.x1, d.gx)
        ys = grid_edges(d.y0, d.y1, d.gy)
        if d.bin_weight is None:
            for b in range(d.gy):
                for a in range(d.gx):
                    area = (xs[a + 1] - xs[a]) * (ys[b + 1] - ys[b])
                    wt = float(d.weight) / float(d.gx * d.gy * area)
                    out.append(Filter([(1.0, xs[a], ys[b], xs[a + 1], ys[b + 1])], wt, True))
        else:
            bw = np.asarray(d.bin_weight, dtype=np.float64).reshape(d.gy, d.gx)
            region = float((d.x1 - d.x0) * (d.y1 - d.y0))
            boxes = [(bw[b, a] / region, xs[a], ys[b], xs[a + 1], ys[b + 1])
                     for b in range(d.gy) for a in range(d.gx)]
            out.append(Filter(boxes, float(d.weight), False))
    return out


def dilation_filter(coarse: np.ndarray) -> np.ndarray:
    """Alg. 2: the (r_h+1) x (r_w+1) dilation filter on the integral image for
    a coarse filter f_i of r_h x r_w bins.  Every bin weight is spread over
    the 2x2 block of taps at its corners with the multiplier [[1,-1],[-1,1]].
    Indexing: fd[b][a] is the tap at (row edge b, column edge a)."""
    f = np.asarray(coarse, dtype=np.float64)
    rh, rw = f.shape
    fd = np.zeros((rh + 1, rw + 1), dtype=np.float64)
    m = np.array([[1.0, -1.0], [-1.0, 1.0]])
    for b in range(rh):
        for a in range(rw):
            fd[b:b + 2, a:a + 2] += f[b, a] * m
    return fd


def dilated_response(P: np.ndarray, x: int, y: int, fd: np.ndarray,
                     xs: Sequence[int], ys: Sequence[int]) -> np.ndarray:
    """Eq. 1 on the integral image with Alg. 2's filter: the response at the
    window whose top-left is (x, y) is sum_{b,a} fd[b][a] * P[y+Y_b][x+X_a],
    where the taps sit on the bin edges (the dilation), per channel.  Taps
    are applied in the exclusive P (reading of the corner convention)."""
    out = np.zeros(P.shape[-1], dtype=np.float64)
    # With P exclusive, bin (a, b) = +P[Y_b][X_a] - P[Y_b][X_a+1]
    # - P[Y_b+1][X_a] + P[Y_b+1][X_a+1]: exactly the multiplier's pattern
    # placed at taps [b..b+1][a..a+1].
    for b in range(fd.shape[0]):
        for a in range(fd.shape[1]):
            if fd[b, a] != 0.0:
                out = out + fd[b, a] * P[y + ys[b], x + xs[a]].astype(np.float64)
    return out


# --------------------------------------------------------------------------
# O5b: the paper's coarse filters and sub-scale aggregation (Sec. 3.2.2,
# Sec. 3.3, Sec. 5.2 "Filtering"; Supp. S.3 option c).
#
# Readings (the paper gives names and sigma only):
#   * the Gaussian is the unnormalised 3x3 kernel exp(-(a^2 + b^2) / (2 sigma^2))
#     at a, b in {-1, 0, 1}, sigma = 2;
#   * Haar-2x has column factors [+1, 0, -1] and Haar-3x [+1, -2, +1], each
#     multiplied elementwise by the Gaussian; the y filters are the transposes;
#   * scale s uses the centred sub-window of floor(w/s) x floor(h/s) starting at
#     (floor((w - floor(w/s)) / 2), floor((h - floor(h/s)) / 2)) with a 3x3 grid;
#   * w_{s,f} = w_f / s with w_f = 1 for the Gaussian and 0.25 for Haar filters;
#   * a filter's response is sum_bins f(a,b) * count(bin) / area(region).

PAPER_FILTER_SETS = {
    "gauss": ("gauss",),
    "2rect": ("gauss", "haar2x", "haar2y"),
    "3rect": ("gauss", "haar3x", "haar3y"),
    "23rect": ("gauss", "haar2x", "haar2y", "haar3x", "haar3y"),
}


def gaussian_coarse(sigma: float = 2.0) -> np.ndarray:
    """3x3 coarse Gaussian, indexed [row b][column a], centre 1."""
    g = np.zeros((3, 3), dtype=np.float64)
    for b in range(3):
        for a in range(3):
            g[b, a] = np.exp(-float((a - 1) ** 2 + (b - 1) ** 2) / (2.0 * sigma * sigma))
    return g


def coarse_filter(name: str) -> np.ndarray:
    """The 3x3 coarse filter of a filter name, indexed [row b][column a]."""
    g = gaussian_coarse()
    if name == "gauss":
        return g
    cols = {"haar2": np.array([1.0, 0.0, -1.0]), "haar3": np.array([1.0, -2.0, 1.0])}[name[:5]]
    hx = g * cols[None, :]            # varies along x (columns)
    if name.endswith("x"):
        return hx
    if name.endswith("y"):
        return g * cols[:, None]      # varies along y (rows)
    raise ValueError(name)


def subscale_region(w: int, h: int, s: int) -> Tuple[int, int, int, int]:
    """Centred sub-window of scale s: (x0, y0, x1, y1)."""
    rw, rh = w // s, h // s
    x0, y0 = (w - rw) // 2, (h - rh) // 2
    return x0, y0, x0 + rw, y0 + rh


def paper_bank(w: int, h: int, filter_set: str, n_scales: int) -> List[FilterDesc]:
    """The filter bank of Sec. 5.2: every filter of the set at every scale
    s = 1..n_scales, scale-major, each one weighted filter over a 3x3 grid."""
    names = PAPER_FILTER_SETS[filter_set]
    out: List[FilterDesc] = []
    for s in range(1, n_scales + 1):
        x0, y0, x1, y1 = subscale_region(w, h, s)
        if x1 - x0 < 3 or y1 - y0 < 3:
            raise ValueError(f"scale {s}: sub-window {x1 - x0}x{y1 - y0} has empty bins")
        for name in names:
            wf = 1.0 if name == "gauss" else 0.25
            out.append(FilterDesc(x0, y0, x1, y1, 3, 3, coarse_filter(name), wf / float(s)))
    return out


# --------------------------------------------------------------------------
# O6 / O7: filter responses, template representation and the similarity map.

def filter_responses(P: np.ndarray, x: int, y: int, filters: Sequence[Filter]) -> np.ndarray:
    """Responses of every filter at the window with top-left (x, y):
    float64 [n_filters, k] (exact integers for indicator filters)."""
    k = P.shape[-1]
    out = np.zeros((len(filters), k), dtype=np.float64)
    for i, f in enumerate(filters):
        acc = np.zeros(k, dtype=np.float64)
        for coef, bx0, by0, bx1, by1 in f.boxes:
            cnt = box_sum(P, x + bx0, y + by0, x + bx1, y + by1).astype(np.float64)
            acc = acc + coef * cnt
        out[i] = acc
    return out


def template_representation(template_labels: np.ndarray, k: int,
                            filters: Sequence[Filter]) -> np.ndarray:
    """R(tau): the same filters on the template's own NNF (Sec. 3.3)."""
    P = integral_image(template_labels, k)
    return filter_responses(P, 0, 0, filters)


def l1_per_filter(rt: np.ndarray, rq: np.ndarray) -> np.ndarray:
    """sum_j |R_f,j(tau) - R_f,j(q)| per filter, summed sequentially in j."""
    d = np.abs(rt - rq)
    acc = np.zeros(d.shape[0], dtype=np.float64)
    for j in range(d.shape[1]):
        acc = acc + d[:, j]
    return acc


def similarity_map(query_labels: np.ndarray, k: int, w: int, h: int,
                   filters: Sequence[Filter], rt: np.ndarray,
                   region: Optional[Tuple[int, int, int, int]] = None) -> np.ndarray:
    """Eq. 2 for every valid window: sim = -sum_f w_f * |R_f(tau) - R_f(q)|_1.

    Returns float64 [(H-h+1), (W-w+1)], or only the windows with top-left in
    region = (wx0, wy0, wx1, wy1) (others NaN) when given.  Integer L1s are
    exact; the weighted sum runs over filters in order."""
    H, W = query_labels.shape
    P = integral_image(query_labels, k)
    oh, ow = H - h + 1, W - w + 1
    out = np.full((oh, ow), np.nan, dtype=np.float64)
    wx0, wy0, wx1, wy1 = region if region is not None else (0, 0, ow, oh)
    wts = np.array([f.weight for f in filters], dtype=np.float64)
    for y in range(wy0, wy1):
        for x in range(wx0, wx1):
            l1 = l1_per_filter(rt, filter_responses(P, x, y, filters))
            s = 0.0
            for i in range(len(filters)):
                s = s + wts[i] * l1[i]
            out[y, x] = -s
    return out


def similarity_map_fast(query_labels: np.ndarray, k: int, w: int, h: int,
                        filters: Sequence[Filter], rt: np.ndarray) -> np.ndarray:
    """Same values as similarity_map (indicator or weighted filters),
    vectorised over windows: per-filter box sums of P for all windows at once,
    with the boxes, the L1 over channels and the weighted sum in the same
    order, so every window's value is the same float64 result."""
    H, W = query_labels.shape
    P = integral_image(query_labels, k)
    oh, ow = H - h + 1, W - w + 1
    total = np.zeros((oh, ow), dtype=np.float64)
    for i, f in enumerate(filters):
        resp = np.zeros((oh, ow, k), dtype=np.float64)
        for coef, bx0, by0, bx1, by1 in f.boxes:
            cnt = (P[by1:by1 + oh, bx1:bx1 + ow] - P[by0:by0 + oh, bx1:bx1 + ow]
                   - P[by1:by1 + oh, bx0:bx0 + ow] + P[by0:by0 + oh, bx0:bx0 + ow])
            resp = resp + coef * cnt.astype(np.float64)
        d = np.abs(resp - rt[i][None, None, :])
        l1 = np.zeros((oh, ow), dtype=np.float64)
        for j in range(k):
            l1 = l1 + d[:, :, j]
        total = total + f.weight * l1
    return -total


# --------------------------------------------------------------------------
# O8: localisation.

def localise(sim: np.ndarray) -> Tuple[int, int, float]:
    """argmax of the heatmap; ties to the lowest y, then the lowest x
    (row-major first).  Returns (x, y, score)."""
    flat = np.asarray(sim, dtype=np.float64).reshape(-1)
    i = int(np.argmax(flat))       # first maximum in row-major order
    ow = sim.shape[1]
    return i % ow, i // ow, float(flat[i])


# --------------------------------------------------------------------------
# Whole pipeline for one (template, query) pair.

@dataclass
class MatchResult:
    codebook: np.ndarray          # float32 [k, D]
    template_labels: np.ndarray   # int64 [h, w]
    rt: np.ndarray                # float64 [n_filters, k]
    query_labels: np.ndarray      # int64 [H, W]
    sim: np.ndarray               # float64 [H-h+1, W-w+1]
    best: Tuple[int, int, float]


def match(template: np.ndarray, query: np.ndarray, k: int, bank: Sequence[FilterDesc],
          codebook: Optional[np.ndarray] = None, iters: int = 20, seed: int = 0) -> MatchResult:
    """The full method on one pair (Sec. 3): codebook, NNFs, filtering,
    similarity and localisation.  template float [h, w, D] (FP32 values);
    query float64 [H, W, D] (decoded with O1)."""
    h, w, D = template.shape
    if codebook is None:
        codebook = kmeans_codebook(template, k, iters, seed)
    cb = np.asarray(codebook, dtype=np.float32).astype(np.float64)
    tl = assign_map(np.asarray(template, dtype=np.float32).astype(np.float64), cb)
    filters = expand_bank(bank)
    rt = template_representation(tl, k, filters)
    ql = assign_map(np.asarray(query, dtype=np.float64), cb)
    sim = similarity_map_fast(ql, k, w, h, filters, rt)
    return MatchResult(np.asarray(codebook, dtype=np.float32), tl, rt, ql, sim, localise(sim))

"""Benchmark of the VQ-NNF hot path on one MI355X.

One step = one vqnnf_match call: nearest-codeword assignment (BF16 matrix
cores + FP64 re-score of near ties), the on-chip one-hot integral images, the
full-window + 3x3-grid filter bank, eq. 2 scores for every window and the
argmax, on device-resident inputs.  The default workload is the 1024x1024
query map with D=512 BF16 features, k=128 codewords and a 96x96 template.

Prints one JSON line.  `value` is query pixels per second of the refined path;
the plain FP32 path is timed on the same workload beside it, and a bounded
sample of the FP64 CPU oracle gives the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query px/s for VQ-NNF assign+filter+score, BF16-refined vs FP32, labels exact"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# LDS read bandwidth: 256 bytes per clock per CU x 256 CUs x 2.4 GHz = 157.3
# TB/s (gfx950 doubles the 128 B/clock of earlier CDNA LDS; a conflict-free
# ds_read_b128 loop over the whole chip measured 114 TB/s = 186 B per clock
# per CU, more than 128 could deliver)
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12
# vector ALU issue: two wave64 instructions per clock per CU (4 SIMDs, a
# full-rate 32-bit operation takes 2 clocks) = 256 x 128 lanes x 2.4 GHz =
# 78.6 T lane-ops/s, the FP32 vector peak of 157.3 TFLOP/s with an FMA as one
# lane-op (a chip-wide loop of independent v_fma_f32 measured 1.62 wave
# instructions per clock per CU; v_sad_u16 issues at half that rate)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_desc(name, wl):
    qm, t = wl.maps[0], wl.templates[0][0]
    h, w, D = t.data.shape
    return (f"{name}: {qm.H}x{qm.W} query, D={qm.D} {qm.dtype}, k={t.k}, {w}x{h} template, "
            f"full+{t.grid}x{t.grid} bank")


def score_lds_bytes(H, W, w, h, g, kpad):
    """Bytes the on-chip score tile kernel moves through LDS for one (template,
    map) pair: per window row of a tile and 8 channels, the g band prefix rows
    (nseg segments of 7 columns, 16-byte entries) are read from the column
    histograms and written (2 x 16 B per entry), and every window reads
    g(g+1) 16-byte taps.  Tile widths follow the kernel's plan (at most 256
    windows, balanced over the map); the block width and tile height do not
    change the total."""
    kSL, kNSeg = 7, 53
    ow, oh = W - w + 1, H - h + 1
    txw_max = min(256, kSL * kNSeg - kSL + 1 - w)
    nx = -(-ow // txw_max)
    txw = -(-ow // nx)
    total = 0
    for bx in range(nx):
        txv = min(txw, ow - bx * txw)
        nseg = (txv + w - 1) // kSL + 1
        total += oh * (kpad // 8) * (g * nseg * kSL * 32 + txv * g * (g + 1) * 16)
    return total


def kpad_of(k):
    """Padded codebook size: blocks of 16 codewords, rounded to 1-4, 8 or 16 blocks."""
    kb = (k + 15) // 16
    return 16 * (8 if 4 < kb <= 8 else 16 if kb > 8 else kb)


def kernel_roofline(name, avg_ms, n_pix, D, qbytes, k, terms, lds_bytes=None):
    """Algorithmic work of one launch of `name` and the bound it is held to."""
    s = avg_ms / 1e3
    if name in ("assign_bf16_refined", "assign_fp32_plain"):
        # bytes: every query element once + one label byte per pixel
        by = n_pix * (D * qbytes + 1)
        return {"bound": "hbm", "achieved": by / s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": by / s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": by,
                "mfma_tflops": 2.0 * n_pix * k * D * terms / s / 1e12}
    if name == "score_partial" and lds_bytes:
        ach = lds_bytes / s / 1e12
        return {"bound": "lds", "achieved": ach, "peak": LDS_PEAK_TBS, "unit": "TB/s",
                "frac": ach / LDS_PEAK_TBS, "algorithmic_bytes": lds_bytes}
    return None


def kernel_source_sha(kernel):
    """sha256 of the source file that holds `kernel` (traffic figures are tied to it)."""
    import hashlib
    src = {"assign_bf16_refined": "k_assign.hip", "assign_fp32_plain": "k_assign.hip",
           "score_partial": "k_score.hip", "score_combine": "k_score.hip"}.get(kernel)
    if src is None:
        return None
    path = os.path.join(ROOT, "paper_2306_15010_amd", "csrc", src)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain copy of known
    size), or None when there is none or the kernel source changed since."""
    import glob
    import re
    for path in glob.glob(os.path.join(ROOT, "profiles", f"traffic__{kernel}__{workload}*.md")):
        text = open(path).read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        if not m:
            continue
        d = json.loads(m.group(1))
        if d.get("kernel_source_sha256") != kernel_source_sha(kernel):
            return None
        return d.get("hbm_bytes_per_launch")
    return None


def copy_probe(n_bytes=1 << 30, reps=3):
    """A plain device copy of known size: the reference the HBM byte counters
    are scaled by (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE on this run)."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n_bytes, "reps": reps}), flush=True)


def read_probe(n_bytes=1 << 30, reps=3):
    """A read-only pass over a buffer of known size (a sum over 1 GiB): the
    reference for the HBM read counters of read-mostly kernels."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    for _ in range(reps):
        a.sum()
    torch.cuda.synchronize()
    print(json.dumps({"read_probe_bytes": n_bytes, "reps": reps}), flush=True)


def peak_probe():
    """Chip-wide throughput probes (bench_probe.hip): wave64 VALU instructions
    per clock per CU for v_add_u32, v_sad_u16 and v_fma_f32, LDS bytes read per
    clock per CU with conflict-free ds_read_b128 (both at the 2.4 GHz peak
    clock), and the dense matrix-core rates of the BF16 and block-scaled FP8
    instructions."""
    import ctypes
    import torch
    torch.cuda.init()
    lib = ctypes.CDLL(os.path.join(ROOT, "bench_probe.so"))
    lib.bench_probe_run.argtypes = [ctypes.POINTER(ctypes.c_double)]
    out = (ctypes.c_double * 7)()
    rc = lib.bench_probe_run(out)
    if rc:
        raise RuntimeError(f"bench_probe_run: HIP error {rc}")
    ncu = out[4]
    per_clock = lambda v: v / (ncu * 2.4e9)
    print(json.dumps({"compute_units": int(ncu),
                      "valu_wave_instr_per_cu_clock": {"v_add_u32": per_clock(out[0]),
                                                       "v_sad_u16": per_clock(out[1]),
                                                       "v_fma_f32": per_clock(out[2])},
                      "lds_read_tbs": out[3] / 1e12, "lds_read_bytes_per_cu_clock": per_clock(out[3]),
                      "mfma_dense_tflops": {"bf16_16x16x32": out[5] / 1e12,
                                            "fp8_e4m3_scaled_16x16x128": out[6] / 1e12}}),
          flush=True)


def secondary(name, ctx, B, synth, steps):
    """Both paths on another workload (device-resident, same timing as the main line)."""
    import torch
    wl = synth.make_config(name)
    qm, t = wl.maps[0], wl.templates[0][0]
    h, w, D = t.data.shape
    tpl = B.vqnnf_codebook(ctx, t.data, t.k, 20, 0, B.default_bank(w, h, t.grid))
    if qm.dtype == "f32":
        qd = torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()
    else:
        qd = torch.from_numpy(qm.data.view(np.int16)).cuda()
    fm = B.device_fmap(qd, qm.dtype)
    heat = torch.empty((qm.H - h + 1) * (qm.W - w + 1), device="cuda")
    out = {"workload": workload_desc(name, wl)}
    for key, prec in (("bf16_refined", B.VQNNF_PREC_BF16_REFINED), ("fp32_plain", B.VQNNF_PREC_FP32_PLAIN)):
        for _ in range(3):
            B.vqnnf_match(ctx, tpl, fm, prec, heat, want_best=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.vqnnf_match(ctx, tpl, fm, prec, heat, want_best=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[key] = {"value": qm.H * qm.W / (ms / 1e3), "ms_per_step": ms}
    best, _ = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
    out["best"] = {"x": best[0], "y": best[1], "planted": [t.x0, t.y0]}
    return out


def bank_ops_per_window(bank, k):
    """Algorithmic lane-ops of the bank kernel per window: per region group
    (one per scale here) the tap differences and count conversions
    (gx(gy+1) + 2 gx gy per channel), per filter one FMA per non-zero bin plus
    |difference| and accumulation (3) per channel."""
    ops = 0
    prev = None
    for e in bank:
        gx, gy, bw = e[4], e[5], np.asarray(e[7])
        if tuple(e[:6]) != prev:            # consecutive filters of one region share its counts
            ops += k * (gx * (gy + 1) + 2 * gx * gy)
        prev = tuple(e[:6])
        ops += k * (int(np.count_nonzero(bw)) + 3)
    return ops


def paper_bank_leg(ctx, B, t, fm, qm, steps, torch):
    """The paper's own filter bank (Gaussian + Haar 2x/2y/3x/3y at scales
    1..3: 15 weighted filters, Sec. 5.2) on the same map and template:
    assignment, integral image in HBM, bank kernel, localisation."""
    h, w, _ = t.data.shape
    bank = B.paper_bank(w, h, "23rect", 3)
    tpl = B.vqnnf_codebook(ctx, t.data, t.k, 20, 0, bank)
    oh, ow = qm.H - h + 1, qm.W - w + 1
    heat = torch.empty(oh * ow, device="cuda")
    P = B.VQNNF_PREC_BF16_REFINED
    for _ in range(3):
        B.vqnnf_match(ctx, tpl, fm, P, heat, want_best=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.vqnnf_match(ctx, tpl, fm, P, heat, want_best=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ctx.reset_times()
    ctx.set_timing(True)
    for _ in range(steps):
        B.vqnnf_match(ctx, tpl, fm, P, heat, want_best=False)
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    best, _ = B.vqnnf_match(ctx, tpl, fm, P, heat)
    avg = {k: v[1] / max(1, v[0]) for k, v in kt.items()}
    out = {"workload": f"same map and template, paper bank F_2,3-rect at S=3 ({len(bank)} weighted filters)",
           "value": qm.H * qm.W / (ms / 1e3), "unit": "px/s", "ms_per_step": ms,
           "kernels_avg_ms": {k: round(v, 4) for k, v in avg.items()},
           "best": {"x": best[0], "y": best[1], "planted": [t.x0, t.y0]}}
    if "score_bank" in avg:
        ops = bank_ops_per_window(bank, t.k) * oh * ow
        ach = ops / (avg["score_bank"] * 1e-3) / 1e12
        out["score_bank_roofline"] = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                                      "unit": "Tops/s", "frac": ach / VALU_PEAK_TOPS,
                                      "ops_per_window": bank_ops_per_window(bank, t.k)}
    if "integral_main" in avg:
        # weighted banks read the integral image mod 2^16: 2 bytes per entry
        pbytes = (qm.H + 1) * (qm.W + 1) * (t.k + t.k % 2) * 2 + qm.H * qm.W
        out["integral_hbm_tbs"] = pbytes / (avg["integral_main"] * 1e-3) / 1e12
    return out


def _timed(fn, steps, torch):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def _kernel_avgs(ctx, fn, steps):
    ctx.reset_times()
    ctx.set_timing(True)
    for _ in range(steps):
        fn()
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    return {k: round(v[1] / max(1, v[0]), 4) for k, v in kt.items()}


def low_d_leg(ctx, B, t, qd, qm, steps, torch):
    """The same map and template reduced to d = 18 and 9 principal axes of the
    template (Sec. 5.5): the timed step is the query projection plus the
    whole matching path at D = d; the template's PCA and k-means are
    preparation."""
    h, w, D = t.data.shape
    out = {}
    for d in (18, 9):
        mean, basis, _ = B.vqnnf_pca_fit(t.data, d)
        tp = torch.empty((h, w, d), dtype=torch.float32, device="cuda")
        B.vqnnf_pca_project(ctx, B.device_fmap(torch.from_numpy(np.ascontiguousarray(t.data)).cuda(), "f32"),
                            mean, basis, tp)
        tpl = B.vqnnf_codebook(ctx, tp.cpu().numpy(), t.k, 20, 0, B.default_bank(w, h, t.grid))
        qp = torch.empty((qm.H, qm.W, d), dtype=torch.float32, device="cuda")
        heat = torch.empty((qm.H - h + 1) * (qm.W - w + 1), device="cuda")
        fm_in = B.device_fmap(qd, qm.dtype)
        fm = B.device_fmap(qp, "f32")

        def step():
            B.vqnnf_pca_project(ctx, fm_in, mean, basis, qp)
            B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat, want_best=False)

        ms = _timed(step, steps, torch)
        best, _ = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
        out[f"d{d}"] = {"value": qm.H * qm.W / (ms / 1e3), "unit": "px/s", "ms_per_step": ms,
                        "kernels_avg_ms": _kernel_avgs(ctx, step, steps),
                        "best": {"x": best[0], "y": best[1], "planted": [t.x0, t.y0]}}
    out["workload"] = "same map and template, PCA of the template to d = 18 / 9, projection timed"
    return out


def colour_leg(ctx, B, synth, steps, torch):
    """Colour features (Sec. 5.2): a 1280x720 RGB image (the long-video frame
    size), a 100x100 crop as template, k = 128; features are 3x3 RGB patches
    built inside the assignment; the full-window + 3x3 grid bank and the
    paper's best colour bank (F_2,3-rect at S = 4, 20 filters)."""
    H, W, side, k = 720, 1280, 100, 128
    img = synth.rgb_image(H, W, seed=230615014)
    rng = np.random.default_rng(230615014)
    x0, y0 = int(rng.integers(0, W - side + 1)), int(rng.integers(0, H - side + 1))
    crop = np.ascontiguousarray(img[y0:y0 + side, x0:x0 + side])
    fm = B.device_fmap(torch.from_numpy(img).cuda(), "rgb8")
    heat = torch.empty((H - side + 1) * (W - side + 1), device="cuda")
    out = {"workload": f"{W}x{H} RGB, colour features D=27, {side}x{side} template, k={k}"}
    for name, bank in (("full_3x3", B.default_bank(side, side, 3)),
                       ("paper_23rect_S4", B.paper_bank(side, side, "23rect", 4))):
        tpl = B.vqnnf_codebook(ctx, crop, k, 20, 0, bank)

        def step():
            B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat, want_best=False)

        ms = _timed(step, steps, torch)
        best, _ = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
        out[name] = {"value": H * W / (ms / 1e3), "unit": "px/s", "ms_per_step": ms,
                     "kernels_avg_ms": _kernel_avgs(ctx, step, steps),
                     "best": {"x": best[0], "y": best[1], "planted": [x0, y0]}}
    return out


def stored_label_hashes(workload):
    """Per-pair SHA-256 of the oracle's full-size label maps (written by
    tests/golden/make_fullsize_golden.py from the oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_labels.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f).get(workload)
    if not g:
        return None
    return [p["labels_sha256"] for m in g["maps"] for p in m["pairs"]]


def batched_leg(workload, scale_down, steps, warmup, ctx, B, synth, torch, with_cpu=False):
    """Batched workloads: every (template, map) pair in one vqnnf_match_batched
    call, replayed as one captured HIP graph, against the same pairs as
    sequential vqnnf_match calls."""
    import hashlib
    log(f"generating workload {workload} (map sides / {scale_down})")
    t0 = time.perf_counter()
    wl = synth.make_config(workload, scale_down=scale_down,
                           progress=lambda i, n: log(f"  map {i} of {n} made"))
    log(f"  {time.perf_counter() - t0:.1f} s")
    tpls, fms, heats, devs = [], [], [], []
    flat = [t for row in wl.templates for t in row]
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    # every template's k-means (and NNF) in one batched call on the GPU
    tpls = B.vqnnf_codebook_batched(ctx, [t.data for t in flat], [t.k for t in flat], 20,
                                    list(range(len(flat))),
                                    [B.default_bank(t.data.shape[1], t.data.shape[0], t.grid) for t in flat])
    prep_s = time.perf_counter() - tp0
    for qm, row in zip(wl.maps, wl.templates):
        if qm.dtype == "f32":
            dev = torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()
        elif qm.dtype == "bf16":
            dev = torch.from_numpy(qm.data.view(np.int16)).cuda()
        else:
            dev = torch.from_numpy(qm.data).cuda()
        devs.append(dev)
        for t in row:
            h, w, _ = t.data.shape
            fms.append(B.device_fmap(dev, qm.dtype, qm.scale))
            heats.append(torch.empty((qm.H - h + 1) * (qm.W - w + 1), device="cuda"))
    log(f"  {len(tpls)} templates prepared in {prep_s:.1f} s")
    pair_px = sum(qm.H * qm.W * len(row) for qm, row in zip(wl.maps, wl.templates))
    map_px = sum(qm.H * qm.W for qm in wl.maps)
    P = B.VQNNF_PREC_BF16_REFINED

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    def seq():
        for tp, fm, ht in zip(tpls, fms, heats):
            B.vqnnf_match(ctx, tp, fm, P, ht, want_best=False)

    def bat():
        B.vqnnf_match_batched(ctx, tpls, fms, P, heats, want_best=False)

    log("timing: graph-captured batch")
    B.vqnnf_ctx_set_graph(ctx, True)
    ms_graph = timed(bat, steps, warmup)
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    B.vqnnf_ctx_set_graph(ctx, False)
    # the batch's label maps against the oracle's (stored hashes, full size only)
    stored = stored_label_hashes(workload) if scale_down == 1 else None
    labels_ok = None
    if stored is not None and len(stored) == len(tpls):
        labels_ok = 0
        pi = 0
        for qm, row in zip(wl.maps, wl.templates):
            lab = torch.empty(qm.H * qm.W, dtype=torch.uint8, device="cuda")
            for _ in row:
                B.vqnnf_batched_labels(ctx, pi, lab)
                torch.cuda.synchronize()
                labels_ok += hashlib.sha256(lab.cpu().numpy().tobytes()).hexdigest() == stored[pi]
                pi += 1
    log("timing: eager batch")
    ms_eager = timed(bat, steps, warmup)
    log("timing: sequential vqnnf_match calls")
    ms_seq = timed(seq, steps, warmup)
    ctx.reset_times()
    ctx.set_timing(True)
    bat()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    found = 0
    i = 0
    for row in wl.templates:
        for t in row:
            found += int(out[i][0] == (t.x0, t.y0))
            i += 1
    cpu = None
    if with_cpu:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline_sample(wl)
    # dominant kernel of the batch: the fused multi-template assignment, a
    # dense contraction of 2*k*D flop per (pixel, template); the refined path
    # executes it twice (high and low BF16 terms of the codebook)
    roof = None
    if "assign_multi" in kt and kt["assign_multi"][0] > 0:
        alg = sum(2.0 * t.k * qm.D * qm.H * qm.W for qm, row in zip(wl.maps, wl.templates) for t in row)
        ms_am = kt["assign_multi"][1]
        ach = alg / (ms_am / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": 2500.0, "unit": "TFLOP/s", "frac": ach / 2500.0,
                "traffic": None, "kernel": "assign_multi", "algorithmic_flop": alg,
                "executed_tflops": 2.0 * ach, "kernel_ms_per_batch": ms_am}
    # the batch's tile score, held to the LDS bound
    score_roof = None
    if "score_partial" in kt and kt["score_partial"][0] > 0:
        lds = sum(score_lds_bytes(qm.H, qm.W, t.data.shape[1], t.data.shape[0], t.grid, kpad_of(t.k))
                  for qm, row in zip(wl.maps, wl.templates) for t in row)
        ach = lds / (kt["score_partial"][1] / 1e3) / 1e12
        score_roof = {"bound": "lds", "achieved": ach, "peak": LDS_PEAK_TBS, "unit": "TB/s",
                      "frac": ach / LDS_PEAK_TBS, "algorithmic_bytes": lds,
                      "kernel_ms_per_batch": kt["score_partial"][1]}
    value = pair_px / (ms_graph / 1e3)
    res = {
        "metric": METRIC, "value": value, "unit": "px/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms_graph, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp8" if wl.maps[0].dtype == "fp8" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"{workload}: {len(wl.maps)} map(s), {len(tpls)} (template, map) "
                               f"pairs, D={wl.maps[0].D} {wl.maps[0].dtype}, map sides / {scale_down}",
                   "global_batch": len(tpls), "pair_pixels": pair_px, "map_pixels": map_px,
                   "prec": "bf16_refined"},
        "roofline": roof,
        "score_roofline": score_roof,
        "cpu_baseline": cpu,
        "map_px_per_s": map_px / (ms_graph / 1e3),
        "graph_batch_ms": ms_graph, "eager_batch_ms": ms_eager, "sequential_ms": ms_seq,
        "sequential_value": pair_px / (ms_seq / 1e3),
        "speedup_vs_sequential": ms_seq / ms_graph,
        "labels_equal_to_oracle": (f"{labels_ok} of {len(tpls)} pairs (stored oracle hashes)"
                                   if labels_ok is not None else None),
        "planted_found": f"{found} of {len(tpls)}",
        "kernels_total_ms": {k: round(v[1], 4) for k, v in kt.items()},
        "kernel_launches": {k: v[0] for k, v in kt.items()},
        "template_prep_s": prep_s,
    }
    for tp in tpls:
        tp.free()
    return res


def cpu_baseline_sample(wl, budget_px=256 * 256):
    """The oracle as it stands on a bounded sample of the same workload: the
    top-left 256x256 pixels of the query (assign, integral image, filter bank,
    scores of every window inside the sample, argmax).  Batched workloads use
    the pair with the smallest template (its k-means is not timed)."""
    from oracle import vqnnf_oracle as O
    pairs = [(qm, t) for qm, row in zip(wl.maps, wl.templates) for t in row]
    qm, t = min(pairs, key=lambda p: p[1].data.size * p[1].k)
    h, w, D = t.data.shape
    side = int(np.sqrt(budget_px))
    side = max(side, max(h, w))
    q = O.decode(qm.dtype, qm.data[:side, :side], qm.scale)
    cb = O.kmeans_codebook(t.data, t.k, 20, seed=0) if D * t.k * h * w <= 2e7 else None
    if cb is None:
        cb_path = os.path.join(ROOT, "tests", "golden", f"{wl.name}_codebook.npy")
        cb = np.load(cb_path) if os.path.exists(cb_path) else O.kmeans_codebook(t.data, t.k, 20, 0)
    bank = O.default_bank(w, h, t.grid)
    filters = O.expand_bank(bank)
    cb64 = cb.astype(np.float64)
    tl = O.assign_map(t.data.astype(np.float64), cb64)
    rt = O.template_representation(tl, t.k, filters)
    t0 = time.perf_counter()
    ql = O.assign_map(q, cb64)
    sim = O.similarity_map_fast(ql, t.k, w, h, filters, rt)
    O.localise(sim)
    dt = time.perf_counter() - t0
    n = side * side
    return {"value": n / dt, "unit": "px/s", "cores": 1, "kind": "oracle",
            "sample": f"top-left {side}x{side} pixels of the query map ({n} px, "
                      f"{sim.size} windows), FP64 numpy, single thread, {dt:.1f} s"}


def oracle_heatmap_bands(O, labels, k, w, h, filters, rt, n_threads, band=64):
    """The oracle's eq. 2 for every window from row bands of the label map (a
    window depends only on the labels inside it), bands on n_threads threads."""
    from concurrent.futures import ThreadPoolExecutor
    H, W = labels.shape
    oh = H - h + 1
    out = np.empty((oh, W - w + 1))

    def one(y0):
        y1 = min(oh, y0 + band)
        out[y0:y1] = O.similarity_map_fast(labels[y0:y1 + h - 1], k, w, h, filters, rt)

    with ThreadPoolExecutor(max_workers=n_threads) as ex:
        list(ex.map(one, range(0, oh, band)))
    return out


def cpu_baseline_full(qm, t, gpu_labels, gpu_heat):
    """The oracle on the whole workload, on every host core the process may
    use: FP64 assignment of every pixel (the oracle's C variant, bit-identical
    to the Python oracle), integral images, filter bank, eq. 2 for every
    window and the argmax (the Python oracle over row bands).  Template prep
    (k-means, template NNF and counts) is not timed, as on the GPU.  Also
    reports the GPU's label mismatches and heatmap error against it."""
    from oracle import vqnnf_oracle as O
    from oracle import vqnnf_oracle_c as OC
    cores = len(os.sched_getaffinity(0))
    h, w, D = t.data.shape
    cb64 = OC.kmeans_codebook(t.data, t.k, 20, seed=0).astype(np.float64)
    filters = O.expand_bank(O.default_bank(w, h, t.grid))
    tl = O.assign_map(t.data.astype(np.float64), cb64)
    rt = O.template_representation(tl, t.k, filters)
    t0 = time.perf_counter()
    ql = OC.assign_map(qm.dtype, qm.data, qm.scale, cb64, n_threads=cores)
    t1 = time.perf_counter()
    sim = oracle_heatmap_bands(O, ql.astype(np.int64), t.k, w, h, filters, rt, cores)
    bx, by, _ = O.localise(sim)
    t2 = time.perf_counter()
    n = qm.H * qm.W
    err = np.abs(gpu_heat.reshape(sim.shape).astype(np.float64) - sim)
    rel = err / np.maximum(np.abs(sim), 2.0 ** -24)
    return {"value": n / (t2 - t0), "unit": "px/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole workload: all {n} query pixels and {sim.size} windows; FP64 "
                      f"assignment (oracle C variant, {cores} threads) {t1 - t0:.1f} s, integral "
                      f"images + filter bank + eq. 2 + argmax (Python oracle, {cores} threads over "
                      f"row bands) {t2 - t1:.1f} s",
            "seconds": t2 - t0,
            "label_mismatches_vs_gpu": int((ql.reshape(-1) != gpu_labels.reshape(-1)).sum()),
            "similarity_abs_err_max": float(err.max()),
            "similarity_abs_err_p999": float(np.quantile(err, 0.999)),
            "similarity_rel_err_max": float(rel.max()),
            "oracle_best": [int(bx), int(by)]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 100 timed steps: the fixed cost of restarting the stream after the
    # synchronisation that opens the timed region (about 0.5 ms) stays near 1%
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--scale-down", type=int, default=1,
                    help="batched workloads: divide map sides by this factor")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--read-probe", action="store_true",
                    help="only run a read-only pass over 1 GiB (counter calibration)")
    ap.add_argument("--peak-probe", action="store_true",
                    help="only run the VALU issue and LDS bandwidth probes (bench_probe.so)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hot path would shard "
              "into independent (template, map) pairs and row bands of a map, but no multi-GPU "
              "launch is implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_15010_amd import binding as B
    from paper_2306_15010_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    if args.read_probe:
        read_probe()
        return
    if args.peak_probe:
        peak_probe()
        return
    if args.workload in ("c4", "c5"):
        # the full batches need more scratch than the default cap (re-score
        # worklists and partial sums of every pair at once)
        res = batched_leg(args.workload, args.scale_down, args.steps, args.warmup,
                          B.Context(stream=torch.cuda.current_stream(), scratch_cap=64 << 30), B, synth,
                          torch, with_cpu=not args.no_cpu_baseline)
        print(json.dumps(res), flush=True)
        return
    log(f"generating workload {args.workload}")
    wl = synth.make_config(args.workload)
    qm, t = wl.maps[0], wl.templates[0][0]
    h, w, D = t.data.shape
    log(workload_desc(args.workload, wl))
    stream = torch.cuda.current_stream()
    ctx = B.Context(stream=stream)
    tp0 = time.perf_counter()
    tpl = B.vqnnf_codebook(ctx, t.data, t.k, 20, 0, B.default_bank(w, h, t.grid))
    prep_s = time.perf_counter() - tp0
    if qm.dtype == "f32":
        qd = torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()
    else:
        qd = torch.from_numpy(qm.data.view(np.int16)).cuda()
    fm = B.device_fmap(qd, qm.dtype)
    oh, ow = qm.H - h + 1, qm.W - w + 1
    heat = torch.empty(oh * ow, device="cuda")
    n_pix = qm.H * qm.W
    qbytes = {"f32": 4, "bf16": 2}[qm.dtype]

    def run(prec, steps, warmup, timing):
        for _ in range(warmup):
            B.vqnnf_match(ctx, tpl, fm, prec, heat, want_best=False)
        torch.cuda.synchronize()
        if timing:
            ctx.reset_times()
            ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            B.vqnnf_match(ctx, tpl, fm, prec, heat, want_best=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = None
        if timing:
            kt = ctx.kernel_times()
            ctx.set_timing(False)
        return dt / steps * 1e3, kt

    P = B.VQNNF_PREC_BF16_REFINED
    log("timing refined path")
    ms, _ = run(P, args.steps, args.warmup, False)
    ms_ev, kt = run(P, args.steps, 1, True)
    best, bscore = B.vqnnf_match(ctx, tpl, fm, P, heat)
    lab = torch.empty(n_pix, dtype=torch.uint8, device="cuda")
    n_flag = B.vqnnf_assign(ctx, tpl, fm, P, lab)
    # the refined path's results, kept for the oracle comparison (later legs
    # reuse the heatmap buffer)
    gpu_heat, gpu_lab = heat.cpu().numpy(), lab.cpu().numpy()
    value = n_pix / (ms / 1e3)

    kernels = {k: {"launches": v[0], "avg_ms": v[1] / max(1, v[0])} for k, v in kt.items()}
    per_step = {k: v[1] / args.steps for k, v in kt.items()}
    dom = max(per_step, key=per_step.get)
    lds = score_lds_bytes(qm.H, qm.W, w, h, t.grid, kpad_of(t.k))
    roof = kernel_roofline(dom, kernels[dom]["avg_ms"], n_pix, D, qbytes, t.k, 2, lds)
    roof = dict(roof) if roof else {}
    roof["kernel"] = dom
    roof["duration_source"] = (f"HIP events on the context stream around each launch, mean of "
                               f"{kernels[dom]['launches']} launches")
    roof["avg_ms"] = kernels[dom]["avg_ms"]
    roof["traffic"] = measured_traffic(dom, args.workload)
    others = {}
    for k2 in kernels:
        r2 = kernel_roofline(k2, kernels[k2]["avg_ms"], n_pix, D, qbytes, t.k, 2, lds)
        if r2:
            others[k2] = {"frac": round(r2["frac"], 4), "achieved": round(r2["achieved"], 2),
                          "unit": r2["unit"], "bound": r2["bound"]}

    fp32 = None
    if not args.no_fp32:
        log("timing plain FP32 path")
        ms32, _ = run(B.VQNNF_PREC_FP32_PLAIN, args.steps, args.warmup, False)
        _, kt32 = run(B.VQNNF_PREC_FP32_PLAIN, max(3, args.steps // 4), 1, True)
        lab32 = torch.empty_like(lab)
        B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_FP32_PLAIN, lab32)
        mism = int((lab32 != lab).sum().item())
        fp32 = {"value": n_pix / (ms32 / 1e3), "ms_per_step": ms32,
                "label_mismatches_vs_refined": mism,
                "kernels_avg_ms": {k: v[1] / max(1, v[0]) for k, v in kt32.items()}}

    sec = None
    if not args.no_secondary and args.workload == "c3":
        log("timing the 512x512 D=64 FP32 workload (both paths)")
        sec = secondary("c2", ctx, B, synth, max(5, args.steps))
        log("timing the paper's filter bank on the same map")
        sec = {"c2": sec, "paper_bank": paper_bank_leg(ctx, B, t, fm, qm, max(5, args.steps // 2), torch)}
        log("timing the low-dimensional (PCA) and colour-feature workloads")
        sec["low_d"] = low_d_leg(ctx, B, t, qd, qm, max(5, args.steps // 2), torch)
        sec["colour"] = colour_leg(ctx, B, synth, max(5, args.steps // 2), torch)
        log("timing the 64-template batch (c4): graph, eager, sequential")
        bctx = B.Context(stream=stream, scratch_cap=64 << 30)
        sec["c4_batched"] = batched_leg("c4", 1, max(5, args.steps // 2), 2, bctx, B, synth, torch)
        bctx.close()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the whole workload (all host cores)")
        cpu = cpu_baseline_full(qm, t, gpu_lab, gpu_heat)

    out = {
        "metric": METRIC, "value": value, "unit": "px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": workload_desc(args.workload, wl), "global_batch": 1,
                   "query_pixels": n_pix, "windows": oh * ow, "prec": "bf16_refined"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_plain": fp32,
        "speedup_vs_fp32_plain": (value / fp32["value"]) if fp32 else None,
        "flagged_pixels": n_flag, "flagged_fraction": n_flag / n_pix,
        "best": {"x": best[0], "y": best[1], "score": bscore, "planted": [t.x0, t.y0]},
        "kernels_avg_ms": {k: round(v["avg_ms"], 4) for k, v in kernels.items()},
        "kernel_rooflines": others,
        "ms_per_step_with_kernel_events": ms_ev,
        "template_prep_s": prep_s,
        "secondary": sec,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12    # 32-bit integer lane-ops per second (39.3 T)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_desc(name, wl):
    qm, t = wl.maps[0], wl.templates[0][0]
    h, w, D = t.data.shape
    return (f"{name}: {qm.H}x{qm.W} query, D={qm.D} {qm.dtype}, k={t.k}, {w}x{h} template, "
            f"full+{t.grid}x{t.grid} bank")


def kernel_roofline(name, avg_ms, n_pix, D, qbytes, k, terms, n_win, n_f):
    """Algorithmic work of one launch of `name` and the bound it is held to."""
    s = avg_ms / 1e3
    if name in ("assign_bf16_refined", "assign_fp32_plain"):
        # bytes: every query element once + one label byte per pixel
        by = n_pix * (D * qbytes + 1)
        return {"bound": "hbm", "achieved": by / s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": by / s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": by,
                "mfma_tflops": 2.0 * n_pix * k * D * terms / s / 1e12}
    if name == "score_partial":
        # per window, filter and channel: |T - C| and its accumulation (2 ops)
        # plus the box count from the integral-image taps (3 ops)
        ops = n_win * n_f * k * 5
        return {"bound": "alu", "achieved": ops / s / 1e12, "peak": ALU_PEAK_TOPS,
                "unit": "Tops/s", "frac": ops / s / 1e12 / ALU_PEAK_TOPS, "algorithmic_ops": ops}
    return None


def cpu_baseline(wl, budget_px=256 * 256):
    """The oracle as it stands on a bounded sample of the same workload: the
    top-left 256x256 pixels of the query (assign, integral image, filter bank,
    scores of every window inside the sample, argmax)."""
    from oracle import vqnnf_oracle as O
    qm, t = wl.maps[0], wl.templates[0][0]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the hot path shards "
              "into independent (template, map) pairs and row bands, but multi-GPU runs are not "
              "part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_15010_amd import binding as B
    from paper_2306_15010_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
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
    value = n_pix / (ms / 1e3)

    kernels = {k: {"launches": v[0], "avg_ms": v[1] / max(1, v[0])} for k, v in kt.items()}
    per_step = {k: v[1] / args.steps for k, v in kt.items()}
    dom = max(per_step, key=per_step.get)
    n_f = 1 + t.grid * t.grid
    roof = kernel_roofline(dom, kernels[dom]["avg_ms"], n_pix, D, qbytes, t.k, 2, oh * ow, n_f)
    roof = dict(roof) if roof else {}
    roof["kernel"] = dom
    roof["traffic"] = None
    others = {}
    for k2 in kernels:
        r2 = kernel_roofline(k2, kernels[k2]["avg_ms"], n_pix, D, qbytes, t.k, 2, oh * ow, n_f)
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

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(wl)

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
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

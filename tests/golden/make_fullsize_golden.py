"""Writes the full-size expected label maps of the three benchmark workloads,
using only the oracle (its C variant, bit-identical to the Python oracle)
and the seeded input generator for its inputs.

For every (template, map) pair of
  c3: the 1024x1024 D=512 BF16 map, one 96x96 template, k = 128, seed 0;
  c4: the 1024x1024 D=256 BF16 map, 64 templates (sides 24..160, k in
      {16, 32, 64, 128}), k-means seed = template index;
  c5: 32 FP8 maps with sides 256..2048 (full size), 4 templates each
      (sides 32..128, k = 64), k-means seed = pair index (map-major);
it runs the oracle's k-means (seeded k-means++, 20 Lloyd iterations, FP32
codebook) on the template and the oracle's assignment (exact FP64
nearest codeword, lowest index on ties) on the whole map, and records
SHA-256 hashes of the template, the map, the codebook and the uint8 label
map in fullsize_labels.json.  The c3 label map itself is stored in
c3_query_labels.npz (zlib-compressed) so a test can compare it element by
element and compute the oracle's heatmap from it.

Run: python tests/golden/make_fullsize_golden.py [c3] [c4] [c5]
(all three by default; about 10 minutes on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import vqnnf_oracle_c as OC  # noqa: E402
from paper_2306_15010_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize_labels.json")
ITERS = 20


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def log(*a):
    print(*a, flush=True)


def pair_record(qm, t, seed):
    t0 = time.time()
    cb = OC.kmeans_codebook(t.data, t.k, ITERS, seed=seed)
    t1 = time.time()
    lab = OC.assign_map(qm.dtype, qm.data, qm.scale, cb.astype(np.float64))
    t2 = time.time()
    rec = {"k": t.k, "w": int(t.data.shape[1]), "h": int(t.data.shape[0]), "x0": t.x0, "y0": t.y0,
           "seed": seed, "template_sha256": sha(t.data.astype(np.float32)), "codebook_sha256": sha(cb),
           "labels_sha256": sha(lab)}
    return rec, lab, (t1 - t0, t2 - t1)


def map_record(qm):
    return {"H": qm.H, "W": qm.W, "D": qm.D, "dtype": qm.dtype, "map_sha256": sha(qm.data),
            "scale_sha256": sha(qm.scale) if qm.scale is not None else None}


def run(name, out):
    t0 = time.time()
    wl = synth.make_config(name, progress=lambda i, n: log(f"  {name}: map {i} of {n} made"))
    log(f"{name}: generated in {time.time() - t0:.0f} s")
    maps = []
    seed = 0
    for mi, (qm, row) in enumerate(zip(wl.maps, wl.templates)):
        mrec = map_record(qm)
        mrec["pairs"] = []
        for t in row:
            s = 0 if name == "c3" else seed
            rec, lab, (tk, ta) = pair_record(qm, t, s)
            mrec["pairs"].append(rec)
            log(f"{name}: map {mi} ({qm.W}x{qm.H}) template {t.data.shape[1]}x{t.data.shape[0]} k={t.k} "
                f"seed {s}: k-means {tk:.1f} s, labels {ta:.1f} s")
            if name == "c3":
                np.savez_compressed(os.path.join(HERE, "c3_query_labels.npz"), labels=lab)
            seed += 1
        maps.append(mrec)
    out[name] = {"seed": wl.seed, "lloyd_iters": ITERS, "maps": maps}


def main():
    names = sys.argv[1:] or ["c3", "c4", "c5"]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    for name in names:
        run(name, out)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
        log(f"wrote {OUT} ({name})")


if __name__ == "__main__":
    main()

"""Writes the stored expected values under tests/golden/ using only the
oracle (and the seeded input generator for its inputs).

  c3_codebook.npy : oracle k-means codebook (seeded k-means++, 20 Lloyd
                    iterations, FP32) of the 1024x1024 / D=512 / k=128
                    workload's 96x96 template, seed 0.
  c3_template_sha256.txt : hash of that template's FP32 bytes, so a test can
                    tell whether the generator still produces the same input.

Run: python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import vqnnf_oracle as O  # noqa: E402
from paper_2306_15010_amd import synth  # noqa: E402


def main():
    wl = synth.make_config("c3")
    t = wl.templates[0][0]
    cb = O.kmeans_codebook(t.data, t.k, 20, seed=0)
    np.save(os.path.join(HERE, "c3_codebook.npy"), cb)
    h = hashlib.sha256(np.ascontiguousarray(t.data, dtype=np.float32).tobytes()).hexdigest()
    with open(os.path.join(HERE, "c3_template_sha256.txt"), "w") as f:
        f.write(h + "\n")
    print("wrote c3 golden codebook", cb.shape, h)


if __name__ == "__main__":
    main()

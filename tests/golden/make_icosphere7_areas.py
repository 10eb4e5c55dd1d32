"""Writes icosphere7_areas_oracle.npz: the FP64 oracle's 40-iteration Alg. 3
run (treecode of Alg. 4, c = 2, D = 15, widths 0.002 -> 0.016, zero
initialization; the defaults of Sec. 5.1.1) on the 163,842 vertices of the
level-7 icosphere, the sphere of Table 5 (Sec. 6.1.2), for the GPU test of
the solved-area output.

It calls only the oracle and the seeded generator.  Stored:
* `area`: the oracle's solved areas |mu_i| / s^2 (FP32 rounding of the FP64
  values; s the normalization scale, so the areas are in the unit-sphere
  frame of Table 5);
* `n16`: the oracle's unit normals as int16 (x 32767);
* `points_sha256`: digest of the FP32 input points.

Run from the repository root: ``python tests/golden/make_icosphere7_areas.py``.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "icosphere7_areas_oracle.npz")


def main():
    s = synth.icosphere(7)
    x, _, sc = oracle.normalize(s.points)
    t0 = time.time()
    mu = oracle.orient(x, iters=40, w1=0.002, w2=0.016, backend="tree")
    nm = np.linalg.norm(mu, axis=1)
    area = (nm / sc ** 2).astype(np.float32)
    n16 = np.round(mu / nm[:, None] * 32767.0).astype(np.int16)
    sha = hashlib.sha256(np.ascontiguousarray(s.points, np.float32).tobytes()).hexdigest()
    np.savez_compressed(OUT, area=area, n16=n16, points_sha256=np.array(sha))
    print(f"wrote {OUT} in {time.time() - t0:.0f} s: total {area.astype(np.float64).sum():.6f} "
          f"mean {area.mean():.6e}")


if __name__ == "__main__":
    main()

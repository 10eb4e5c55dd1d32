"""Writes knot500k_orient_oracle.npz: the FP64 oracle's 40-iteration Alg. 3
run (treecode of Alg. 4, c = 2, D = 15, widths 0.002 -> 0.016 as in
Sec. 5.1.1, zero initialization) on the 500k-point torus knot of the
benchmark (seed 3, 2 % outliers), for the end-to-end GPU parity test.

It calls only the oracle and the seeded generator.  Stored:
* `n16`: the oracle's unit normals mu_i / |mu_i| as int16 (x 32767), enough
  to count sign flips n_gpu . n_oracle <= 0 (a stored component is within
  1.6e-5 of the FP64 value);
* `E`, `alpha`, `w`: per iteration the energy of the incoming mu, the step
  length of Alg. 2 and the width;
* `points_sha256`: digest of the FP32 input points, so that a change of
  the generator is seen instead of compared.

Run from the repository root: ``python tests/golden/make_knot500k_orient.py``
(about 5 minutes on 8 cores).
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "knot500k_orient_oracle.npz")


def main():
    cloud = synth.torus_knot(500000, 3)
    x, _, _ = oracle.normalize(cloud.points)
    E, alpha, w = [], [], []

    def cb(i, mu, info):
        E.append(info["E"])
        alpha.append(info["alpha"])
        w.append(info["w"])
        print(f"iteration {i}: w={info['w']:.5f} E={info['E']:.6e} alpha={info['alpha']:.4e}",
              flush=True)

    t0 = time.time()
    mu = oracle.orient(x, iters=40, w1=0.002, w2=0.016, backend="tree", callback=cb)
    nrm = mu / np.linalg.norm(mu, axis=1, keepdims=True)
    assert np.all(np.isfinite(nrm))
    n16 = np.round(nrm * 32767.0).astype(np.int16)
    sha = hashlib.sha256(np.ascontiguousarray(cloud.points, np.float32).tobytes()).hexdigest()
    np.savez_compressed(OUT, n16=n16, E=np.array(E), alpha=np.array(alpha), w=np.array(w),
                        points_sha256=np.array(sha))
    print(f"wrote {OUT} in {time.time() - t0:.0f} s ({oracle.num_threads()} threads)")


if __name__ == "__main__":
    main()

"""Compile the HIP sources into the in-tree shared library libwnnc.so (gfx950).

Run ``python -m paper_2405_16634_amd.build``.  The library is built in place
so that it travels with the source tree.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwnnc.so")
# the hardware-rate probes: a library of their own, not part of libwnnc.so
RATES_SRC = os.path.join(HERE, "hwrates", "rates.hip")
RATES_LIB = os.path.join(HERE, "libwnnc_rates.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("WNNC_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # only the explicit fmaf() calls fuse: results then do not depend on how
    # the compiler shapes each template instance (bit-identical tile shapes)
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src):
    os.makedirs(OBJ, exist_ok=True)
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (p.stderr or "").splitlines()
                     if "is not a recognized feature for this target" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj, errs


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs) + 1)) as ex:
        results = list(ex.map(_compile, srcs + [RATES_SRC]))
    objs = [o for o, _ in results]
    if verbose:
        for o, e in results:
            if e.strip():
                print(e)
    _link(objs[:-1], LIB)
    _link(objs[-1:], RATES_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

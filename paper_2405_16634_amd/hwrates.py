"""Measured throughput of one GPU's vector ALU and HBM (``libwnnc_rates.so``).

The traversal is priced against the chip's published peaks; these probes
measure, on the card at hand, the rates those peaks stand for:

* ``fma``, ``mul``: FP32 vector instructions (wave64) per second.  With one
  wave64 instruction per 4 cycles per SIMD, the issue ceiling is
  256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G/s, i.e. 78.6 TFLOP/s of
  non-packed FP32 FMA;
* ``rsq``: the hardware reciprocal square root, one per pair term;
* ``add64``: FP64 adds (the per-target sums);
* ``acc64``: an FP32 FMA, its conversion to FP64 and an FP64 add: the step
  that adds one FP32 term to an FP64 sum, in instructions per second;
* ``copy``, ``read``: HBM bytes per second of a float4 stream copy (read +
  write) and of a float4 stream read.

``python -m paper_2405_16634_amd.hwrates`` prints one JSON object.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libwnnc_rates.so")

KINDS = {"fma": 0, "mul": 1, "rsq": 2, "add64": 3, "acc64": 4, "copy": 5, "read": 6}
# vector instructions each ALU probe issues per chain step
INSTS_PER_STEP = {"fma": 1, "mul": 1, "rsq": 1, "add64": 1, "acc64": 3}
# the chip's published figures these are compared with
PUBLISHED = {"valu_issue_per_s": 256 * 4 * 2.4e9 / 4, "hbm_bytes_per_s": 8.0e12}


def load():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built (python -m paper_2405_16634_amd.build)")
    lib = ctypes.CDLL(LIB)
    lib.wnnc_rates_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_float)]
    lib.wnnc_rates_run.restype = ctypes.c_int
    lib.wnnc_rates_block.restype = ctypes.c_int
    lib.wnnc_rates_chains.restype = ctypes.c_int
    return lib


def run_alu(lib, kind: str, blocks: int, iters: int) -> dict:
    import torch
    block, chains = lib.wnnc_rates_block(), lib.wnnc_rates_chains()
    out = torch.empty(blocks * block, dtype=torch.float32, device="cuda:0")
    ms = ctypes.c_float()
    rc = lib.wnnc_rates_run(KINDS[kind], blocks, iters, ctypes.c_void_p(out.data_ptr()),
                            ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"probe {kind}: HIP error {rc}")
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError(f"probe {kind}: non-finite chain values")
    waves = blocks * block // 64
    insts = waves * iters * chains * INSTS_PER_STEP[kind]
    rate = insts / (ms.value * 1e-3)
    return {"ms": round(ms.value, 4), "wave_insts": insts, "insts_per_s": rate,
            "frac_of_issue_ceiling": rate / PUBLISHED["valu_issue_per_s"]}


def run_stream(lib, kind: str, blocks: int, mib: int) -> dict:
    import torch
    n = mib * (1 << 20) // 16  # float4 elements per direction
    # copy: source then destination; read: source then one float per thread
    extra = 2 * n * 4 if kind == "copy" else n * 4 + blocks * 256
    buf = torch.ones(extra, dtype=torch.float32, device="cuda:0")
    ms = ctypes.c_float()
    rc = lib.wnnc_rates_run(KINDS[kind], blocks, n, ctypes.c_void_p(buf.data_ptr()),
                            ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"probe {kind}: HIP error {rc}")
    nbytes = n * 16 * (2 if kind == "copy" else 1)
    rate = nbytes / (ms.value * 1e-3)
    return {"ms": round(ms.value, 4), "bytes": nbytes, "bytes_per_s": rate,
            "frac_of_published": rate / PUBLISHED["hbm_bytes_per_s"]}


def measure(blocks: int = 8192, iters: int = 4096, mib: int = 1024) -> dict:
    lib = load()
    res = {"published": PUBLISHED, "blocks": blocks, "block": lib.wnnc_rates_block(),
           "chains": lib.wnnc_rates_chains(), "iters": iters}
    for k in INSTS_PER_STEP:
        res[k] = run_alu(lib, k, blocks, iters)
    for k in ("copy", "read"):
        res[k] = run_stream(lib, k, 4096, mib)
    res["stream_mib"] = mib
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=8192)
    ap.add_argument("--iters", type=int, default=4096)
    ap.add_argument("--mib", type=int, default=1024)
    args = ap.parse_args()
    print(json.dumps(measure(args.blocks, args.iters, args.mib)), flush=True)


if __name__ == "__main__":
    main()

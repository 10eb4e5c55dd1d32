"""Calibration workload for hardware traffic counters.

Copies a device buffer of known size a few times with torch's plain copy
kernel, so that what FETCH_SIZE and WRITE_SIZE read for it can be compared
with the bytes the copy must move (each copy reads and writes ``--mb`` MiB).
Run under ``rocprofv3 --pmc FETCH_SIZE`` (and then ``WRITE_SIZE``).
"""
from __future__ import annotations

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mb", type=int, default=512)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mb * (1 << 20) // 4
    src = torch.arange(n, device="cuda:0", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.mb} MiB x {args.reps}", flush=True)


if __name__ == "__main__":
    main()

"""The hardware-rate probes on the device: each reports a finite rate, and
the FP32 FMA probe stays within the chip's vector-issue ceiling (one wave64
instruction per 4 cycles per SIMD at the 2.4 GHz peak clock)."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_are_finite_and_bounded():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_16634_amd import hwrates
    print("[case] hardware-rate probes, small sizes", flush=True)
    lib = hwrates.load()
    for kind in hwrates.INSTS_PER_STEP:
        r = hwrates.run_alu(lib, kind, 2048, 512)
        print(f"  {kind}: {r['insts_per_s'] / 1e9:.1f} G/s", flush=True)
        assert math.isfinite(r["insts_per_s"]) and r["insts_per_s"] > 0
        assert r["frac_of_issue_ceiling"] <= 1.02
    fma = hwrates.run_alu(lib, "fma", 8192, 1024)
    assert fma["frac_of_issue_ceiling"] > 0.3
    for kind in ("copy", "read"):
        r = hwrates.run_stream(lib, kind, 4096, 64)
        print(f"  {kind}: {r['bytes_per_s'] / 1e9:.0f} GB/s", flush=True)
        assert math.isfinite(r["bytes_per_s"]) and r["bytes_per_s"] > 0

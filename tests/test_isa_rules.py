"""The device code as compiled: every HIP source of the library and of the
rate probes, built with the library's flags to gfx950 assembly, holds no
scalar-memory store, atomic, write-back or discard (every store goes through
vector memory) and no packed FP32 arithmetic (the flags disable it).  CPU
only: hipcc cross-compiles."""
import glob
import os
import re
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2405_16634_amd import build as B

FORBIDDEN = re.compile(r"^\s*(s_store\w*|s_buffer_store\w*|s_scratch_store\w*|s_atomic\w*|"
                       r"s_buffer_atomic\w*|s_dcache_wb\w*|s_dcache_discard\w*|"
                       r"v_pk_add_f32|v_pk_mul_f32|v_pk_fma_f32)\b", re.M)


def _asm(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    flags = [f for f in B.FLAGS if f not in ("-fPIC",)]
    p = subprocess.run([B.HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", out],
                       capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-2000:]
    return src, open(out).read()


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_device_code_has_no_scalar_stores_and_no_packed_fp32():
    srcs = B.sources() + [B.RATES_SRC]
    with tempfile.TemporaryDirectory() as d, ThreadPoolExecutor(max_workers=8) as ex:
        results = list(ex.map(lambda s: _asm(s, d), srcs))
    # real device code: the traversal's template instances alone are hundreds
    assert sum(text.count("s_endpgm") for _, text in results) > 300
    for src, text in results:
        hits = FORBIDDEN.findall(text)
        assert not hits, (os.path.basename(src), sorted(set(hits)))


def test_the_scan_finds_what_it_looks_for():
    sample = "\tv_add_f32_e32 v1, v2, v3\n\ts_store_dword s4, s[0:1], 0x0\n\tv_pk_fma_f32 v[0:1], v[2:3], v[4:5], v[6:7]\n"
    assert sorted(FORBIDDEN.findall(sample)) == ["s_store_dword", "v_pk_fma_f32"]
    assert not FORBIDDEN.findall("\ts_load_dwordx16 s[8:23], s[52:53], s6\n\tglobal_store_dword v[0:1], v2, off\n")

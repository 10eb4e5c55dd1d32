"""The device code as compiled: every HIP source of the library and of the
rate probes, built with the library's flags to gfx950 assembly, holds no
scalar-memory store, atomic, write-back or discard (every store goes through
vector memory), no packed FP32 arithmetic (the flags disable it) and no
kernel with private (scratch) memory, whose spills would be extra memory
traffic and a per-launch set-up; and the record loads that the prefetching
walk issues by inline assembly are left alone while in flight (no
instruction names their registers before the wait, and no branch leaves
that span).  CPU only: hipcc cross-compiles."""
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


_KERNEL_META = re.compile(r"^\s*\.name:\s+(\S+)\s*$|^\s*\.private_segment_fixed_size:\s+(\d+)",
                          re.M)


def private_sizes(text):
    """{kernel symbol: private segment bytes per lane} from the metadata."""
    out, name = {}, None
    for m in _KERNEL_META.finditer(text):
        if m.group(1) is not None:
            name = m.group(1)
        elif name is not None:
            out[name] = int(m.group(2))
    return out


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_device_code_has_no_scalar_stores_no_packed_fp32_and_no_scratch():
    srcs = B.sources() + [B.RATES_SRC]
    with tempfile.TemporaryDirectory() as d, ThreadPoolExecutor(max_workers=8) as ex:
        results = list(ex.map(lambda s: _asm(s, d), srcs))
    # real device code: the traversal's template instances alone are hundreds
    assert sum(text.count("s_endpgm") for _, text in results) > 300
    kernels = 0
    for src, text in results:
        hits = FORBIDDEN.findall(text)
        assert not hits, (os.path.basename(src), sorted(set(hits)))
        sizes = private_sizes(text)
        kernels += len(sizes)
        scratch = {k: v for k, v in sizes.items() if v}
        assert not scratch, (os.path.basename(src), scratch)
    assert kernels > 300


def test_the_private_size_scan_reads_the_metadata():
    meta = ("    .name:           _Z3fooPf\n    .private_segment_fixed_size: 0\n"
            "    .name:           _Z3barPf\n    .private_segment_fixed_size: 16\n")
    assert private_sizes(meta) == {"_Z3fooPf": 0, "_Z3barPf": 16}


def test_the_scan_finds_what_it_looks_for():
    sample = "\tv_add_f32_e32 v1, v2, v3\n\ts_store_dword s4, s[0:1], 0x0\n\tv_pk_fma_f32 v[0:1], v[2:3], v[4:5], v[6:7]\n"
    assert sorted(FORBIDDEN.findall(sample)) == ["s_store_dword", "v_pk_fma_f32"]
    assert not FORBIDDEN.findall("\ts_load_dwordx16 s[8:23], s[52:53], s6\n\tglobal_store_dword v[0:1], v2, off\n")


_SREG = re.compile(r"\bs\[(\d+):(\d+)\]|\bs(\d+)\b")
_BRANCH = re.compile(r"^\s*(s_branch|s_cbranch_\w+)\s+(\S+)")
_LABEL = re.compile(r"^([.\w$]+):")


def _sgprs(operands):
    regs = set()
    for m in _SREG.finditer(operands):
        if m.group(3) is not None:
            regs.add(int(m.group(3)))
        else:
            regs.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return regs


def inline_load_violations(text):
    """For every record load issued by inline assembly (s_load_dwordx16
    between ;;#ASMSTART and ;;#ASMEND), the instructions in layout order up
    to the next inline s_waitcnt lgkmcnt(0): none may name a register of the
    load's destination, and every branch among them must land between the
    load and the wait (the load is still in flight there: a read would see a
    stale value, a write would be overwritten).  Returns (count, problems)."""
    lines = text.split("\n")
    inside, loads, problems = False, 0, []
    for i, line in enumerate(lines):
        t = line.strip()
        if t.startswith(";;#ASMSTART"):
            inside = True
            continue
        if t.startswith(";;#ASMEND"):
            inside = False
            continue
        if not (inside and t.startswith("s_load_dwordx16")):
            continue
        loads += 1
        dest = _sgprs(t.split(None, 1)[1].split(",")[0])
        labels, branches, end, ins = {}, [], None, False
        for j in range(i + 1, len(lines)):
            u = lines[j].strip()
            if u.startswith(";;#ASMSTART"):
                ins = True
                continue
            if u.startswith(";;#ASMEND"):
                ins = False
                continue
            if ins and u.startswith("s_waitcnt") and "lgkmcnt(0)" in u:
                end = j
                break
            lab = _LABEL.match(u)
            if lab:
                labels[lab.group(1)] = j
                continue
            if not u or u.startswith(";") or u.startswith("."):
                continue
            b = _BRANCH.match(u)
            if b:
                branches.append((j, b.group(2)))
            ops = u.split(None, 1)[1] if " " in u else ""
            hit = dest & _sgprs(ops.split(";")[0])
            if hit:
                problems.append((i, j, u, sorted(hit)))
        if end is None:
            problems.append((i, None, "no wait after the load", []))
            continue
        # every branch inside the span goes to a label inside the span
        for j, target in branches:
            if target not in labels:
                problems.append((i, j, f"branch to {target} leaves the span", []))
    return loads, problems


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_inline_record_loads_are_not_touched_in_flight():
    src = os.path.join(os.path.dirname(B.__file__), "csrc", "traverse.hip")
    with tempfile.TemporaryDirectory() as d:
        _, text = _asm(src, d)
    loads, problems = inline_load_violations(text)
    assert loads > 50  # the prefetching walk's template instances
    assert not problems, problems[:5]


def test_the_in_flight_check_finds_what_it_looks_for():
    ok = ("\t;;#ASMSTART\n\ts_load_dwordx16 s[8:23], s[2:3], s4\n\t;;#ASMEND\n"
          "\tv_add_f32_e32 v1, s30, v2\n\ts_cbranch_scc1 .LBB0_2\n.LBB0_2:\n"
          "\t;;#ASMSTART\n\ts_waitcnt lgkmcnt(0)\n\t;;#ASMEND\n\tv_add_f32_e32 v1, s9, v2\n")
    assert inline_load_violations(ok) == (1, [])
    reads = ok.replace("v_add_f32_e32 v1, s30, v2", "s_mov_b32 s40, s12")
    assert len(inline_load_violations(reads)[1]) == 1
    leaves = ok.replace("s_cbranch_scc1 .LBB0_2", "s_cbranch_scc1 .LBB0_9")
    assert len(inline_load_violations(leaves)[1]) == 1

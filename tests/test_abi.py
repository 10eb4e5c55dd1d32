"""The C-ABI library loads and exports every entry point include/wnnc.h
declares (no device calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wnnc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wnnc_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("wnnc_create", "wnnc_destroy", "wnnc_normalize", "wnnc_build",
                     "wnnc_winding", "wnnc_gradient", "wnnc_adjoint", "wnnc_orient",
                     "wnnc_normals", "wnnc_stats", "wnnc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2405_16634_amd as w
    lib = w.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(w.EXPORTED) == declared_functions()
    assert "gfx950" in w.wnnc_version()


def test_library_is_built_for_gfx950_only():
    import re as _re
    import paper_2405_16634_amd as w
    data = open(w.LIB_PATH, "rb").read()
    targets = set(_re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-f]+)", data))
    assert targets == {b"gfx950"}


def test_errors_are_reported_without_a_device():
    """Argument checks that fail before any device work return EINVAL with
    a message (a NULL output pointer for the context)."""
    import paper_2405_16634_amd as w
    lib = w.load_library()
    st = lib.wnnc_create(None, 0, None)
    assert st == w.WNNC_EINVAL
    assert "null" in w.wnnc_last_error()
    assert lib.wnnc_build(None, None, 0, None) == w.WNNC_EINVAL


def test_orient_presets_are_the_papers_parameter_sets():
    """Host-only: the experiment presets (Sec. 5.1.1 defaults, Sec. 5.2.5
    noise levels with w2 = 4 w1, Sec. 5.2.6 scans, Sec. 5.2.3 high genus)."""
    import numpy as np
    import paper_2405_16634_amd as w
    want = {"default": (40, 0.002, 0.016), "noise_0.25": (40, 0.02, 0.08),
            "noise_0.5": (40, 0.03, 0.12), "noise_1": (40, 0.04, 0.16),
            "scan": (40, 0.01, 0.04), "high_genus": (300, 0.002, 0.016)}
    assert set(want) == set(w.PRESETS)
    for name, (it, w1, w2) in want.items():
        p = w.wnnc_orient_preset(name)
        assert p["iters"] == it
        # the widths are FP32 in the options struct
        assert p["w1"] == float(np.float32(w1)) and p["w2"] == float(np.float32(w2))
    o = w.OrientOpts()
    assert w.load_library().wnnc_orient_preset(6, ctypes.byref(o)) == w.WNNC_EINVAL
    assert "preset" in w.wnnc_last_error()


def test_rate_probe_library_is_separate_and_loads():
    """The hardware-rate probes live in a library of their own (not part of
    the boundary): it loads without a device and exports its three calls."""
    from paper_2405_16634_amd import hwrates
    import paper_2405_16634_amd as w
    lib = hwrates.load()
    assert lib.wnnc_rates_block() == 256 and lib.wnnc_rates_chains() == 8
    data = open(hwrates.LIB, "rb").read()
    assert set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-f]+)", data)) == {b"gfx950"}
    main = w.load_library()
    assert not hasattr(main, "wnnc_rates_run")

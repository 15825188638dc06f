"""Host-side checks of the C-ABI library (no GPU needed, no compute calls).

* libwt.so loads and exports every function include/wt.h declares;
* argument validation fails with WT_ERR_ARG before any device work;
* the Python binding refuses host tensors instead of falling back to the CPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "wt.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(wt_[a-z_]+)\s*\(", text))
    # function-pointer typedefs are not exported functions
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def wt():
    import paper_2505_03372_amd as wt
    if not os.path.exists(wt.LIB_PATH):
        from paper_2505_03372_amd import buildlib as b
        b.build()
    return wt


def test_library_exports_every_declared_function(wt):
    L = wt.lib()
    declared = _header_functions()
    assert set(declared) == set(wt.ABI_FUNCTIONS)
    for name in declared:
        assert hasattr(L, name), name
    assert b"gfx950" in L.wt_version()


def test_build_rejects_bad_arguments_before_touching_the_device(wt):
    L = wt.lib()
    out = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        (dummy, 10, 3, 256),          # symbol width
        (dummy, 10, 5, 0),            # symbol width, alphabet to extract
        (ctypes.c_void_p(0), 10, 4, 0),  # null symbols, alphabet to extract
        (dummy, 10, 1, 257),          # sigma beyond the width
        (dummy, 10, 4, (1 << 24) + 1),  # sigma beyond the node-table limit
        (ctypes.c_void_p(0), 10, 1, 4),  # null symbols with n > 0
    ]
    for ptr, n, w, sigma in cases:
        st = L.wt_build(ptr, n, w, sigma, None, None, ctypes.byref(out))
        assert st == wt.WT_ERR_ARG, (n, w, sigma)
        assert out.value is None
        assert L.wt_last_error()
    bad = wt.BuildOpts(300, 4096, 0, 0)
    assert L.wt_build(dummy, 10, 1, 4, ctypes.byref(bad), None, ctypes.byref(out)) == wt.WT_ERR_ARG
    bad = wt.BuildOpts(512, 3000, 0, 0)
    assert L.wt_build(dummy, 10, 1, 4, ctypes.byref(bad), None, ctypes.byref(out)) == wt.WT_ERR_ARG
    # the extraction path (sigma = 0) checks the options before its first device call
    assert L.wt_build(dummy, 10, 1, 0, ctypes.byref(bad), None, ctypes.byref(out)) == wt.WT_ERR_ARG
    assert L.wt_build(dummy, 10, 1, 4, None, None, None) == wt.WT_ERR_ARG


def test_queries_reject_null_tree(wt):
    L = wt.lib()
    assert L.wt_access(None, None, 5, None, None) == wt.WT_ERR_ARG
    assert L.wt_rank(None, None, None, 5, None, None) == wt.WT_ERR_ARG
    assert L.wt_select(None, None, None, 5, None, None) == wt.WT_ERR_ARG
    assert L.wt_free(None) == wt.WT_OK
    assert L.wt_set_allocator(ctypes.c_void_p(1), None, None) == wt.WT_ERR_ARG


def test_binding_refuses_host_tensors(wt):
    import torch
    with pytest.raises(ValueError):
        wt.build(torch.zeros(8, dtype=torch.uint8), sigma=4)
    with pytest.raises(TypeError):
        wt.build(torch.zeros(8, dtype=torch.int64), sigma=4)


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2505_03372_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(dirpath, fn)) as f:
                    text = f.read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "wt_oracle" not in text, fn


def test_tune_table_json_roundtrip(tmp_path):
    import paper_2505_03372_amd as wt
    entries = {(5, 0): (256, 4096), (12, 3): (1024, 16384), (20, 6): (512, 1024)}
    tt = wt.make_tune_table(entries)
    path = str(tmp_path / "t.json")
    wt.save_tune(tt, path)
    tt2 = wt.load_tune(path)
    assert bytes(tt2) == bytes(tt)
    for (nb, sb), (l2, s) in entries.items():
        assert (tt2.l2_bits[nb][sb], tt2.sample_rate[nb][sb]) == (l2, s)


def test_tune_bucket():
    import paper_2505_03372_amd as wt
    assert wt.tune_bucket(1, 1) == (0, 0)
    assert wt.tune_bucket(1 << 10, 4) == (5, 0)
    assert wt.tune_bucket((1 << 24) - 1, 1 << 16) == (11, 4)
    assert wt.tune_bucket(1 << 24, (1 << 16) - 1) == (12, 3)
    assert wt.tune_bucket(1 << 60, 1 << 40) == (wt.TUNE_NB - 1, wt.TUNE_SB - 1)

"""CPU checks of the seeded bit-array generator of the rank/select workload (thesis Section 6.1: fill
rates 10/50/90 %, uniform, or adversarial with 99 % of the ones in the last fill fraction) and of the
bit-vector build's argument checks (no GPU)."""
import ctypes

import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("fill", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("adversarial", [False, True])
def test_bit_array_fill_and_placement(fill, adversarial):
    n = (1 << 21) + 37
    w = workloads.bit_words(0xB175, n, fill, adversarial)
    assert w.size == (n + 63) // 64
    b = workloads.unpack_bits(w, n)
    assert b.size == n and set(np.unique(b)) <= {0, 1}
    # bits past n are zero
    assert (np.unpackbits(w.view(np.uint8), bitorder="little")[n:] == 0).all()
    ones = int(b.sum())
    assert abs(ones / n - fill) < 0.005
    head = int(b[: int(round((1 - fill) * n))].sum())
    if adversarial:
        assert abs(head / ones - 0.01) < 0.002  # 1 % of the ones before the last fill fraction
    else:
        assert abs(head / ones - (1 - fill)) < 0.01  # spread evenly


def test_bit_array_is_seeded():
    a = workloads.bit_words(5, 100_000, 0.5, False)
    b = workloads.bit_words(5, 100_000, 0.5, False)
    c = workloads.bit_words(6, 100_000, 0.5, False)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_bitvector_build_rejects_bad_arguments():
    import paper_2505_03372_amd as wt
    L = wt.lib()
    out = ctypes.c_void_p(0)
    assert L.wt_bv_build(None, 10, None, None, ctypes.byref(out)) == wt.WT_ERR_ARG
    assert L.wt_bv_build(ctypes.c_void_p(0x1000), 1 << 40, None, None, ctypes.byref(out)) == wt.WT_ERR_ARG
    bad = wt.BuildOpts(300, 4096, 0, 0)
    assert L.wt_bv_build(ctypes.c_void_p(0x1000), 10, ctypes.byref(bad), None, ctypes.byref(out)) == wt.WT_ERR_ARG
    assert L.wt_bv_build(ctypes.c_void_p(0x1000), 10, None, None, None) == wt.WT_ERR_ARG
    assert out.value is None

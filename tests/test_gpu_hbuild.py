"""GPU tests of the build from host memory in chunks (wt_build_host; the chunked construction of the
thesis's Conclusion): the tree equals the one wt_build makes from a device copy, part by part (level
sizes and ones, bits, L1/L2, samples, node tables, cumulative histogram), and the oracle's tree; its
answers equal the oracle's. One pass and two passes; page-locked and pageable arrays; one chunk, many
chunks with a ragged last one; reduced codes, 2- and 4-byte symbols, an alphabet above the dense
histogram, full-width codes, sigma = 1, and a level of more than 1024 tiles.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import gpu_cases as G
from tests.test_gpu_parity import make_seq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_03372_amd as wt
    wt.lib()


def _pinned(a):
    import torch
    t = torch.empty(a.size, dtype=getattr(torch, str(a.dtype)), pin_memory=True)
    t.numpy()[:] = a
    return t.numpy(), t


def same_tree(th, td):
    """Every part of two trees of the same sequence is equal."""
    import paper_2505_03372_amd as wt
    a, b = th.info, td.info
    for k in ("levels", "level_n", "level_ones", "n", "sigma", "bytes_total"):
        assert a[k] == b[k], (k, a[k], b[k])
    np.testing.assert_array_equal(th.export(wt.PART_CUM_HIST), td.export(wt.PART_CUM_HIST))
    for l in range(a["levels"]):
        for part in (wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START,
                     wt.PART_NODE_R0):
            x, y = th.export(part, l), td.export(part, l)
            if not np.array_equal(x, y):
                bad = np.nonzero(x != y)[0]
                raise AssertionError("part %d level %d differs at %d places, first %d" % (part, l, bad.size, bad[0]))


# (width, sigma, n, kind, chunk, pinned, two_pass)
CASES = [
    (1, 256, (1 << 21) + 777, "zipf", 1 << 16, True, False),
    (1, 256, (1 << 21) + 777, "zipf", 1 << 16, False, False),
    (1, 256, (1 << 21) + 777, "zipf", 1 << 16, True, True),
    (1, 256, (1 << 21) + 777, "zipf", 1 << 16, False, True),
    (1, 5, 300001, "zipf", 65537, True, False),
    (1, 5, 300001, "zipf", 65537, True, True),
    (1, 200, 250000, "runs", 1 << 20, False, False),       # one chunk
    (1, 7, 40000, "uniform", 1 << 16, True, True),         # fewer symbols than one chunk
    (2, 1000, 1 << 20, "zipf", 100003, True, False),
    (2, 65536, 400000, "uniform", 1 << 17, False, True),
    (4, 1 << 20, 1 << 21, "zipf12", 1 << 19, True, False),  # alphabet above the dense histogram
    (4, 1 << 20, 1 << 21, "zipf12", 1 << 19, True, True),
    (4, 12345, 300000, "sparse", 70000, False, False),
    (1, 1, 100000, "equal", 1 << 16, True, False),         # sigma = 1: no level
]


@pytest.mark.parametrize("width,sigma,n,kind,chunk,pinned,two_pass", CASES)
def test_host_build_equals_device_build(width, sigma, n, kind, chunk, pinned, two_pass):
    import paper_2505_03372_amd as wt
    G.log("host build: width=%d sigma=%d n=%d %s chunk=%d pinned=%s two_pass=%s"
          % (width, sigma, n, kind, chunk, pinned, two_pass))
    S = make_seq(kind, n, sigma, width, 0x4B10 + n + sigma)
    keep = None
    Sh = S
    if pinned:
        Sh, keep = _pinned(S)
    th, st = wt.build_host(Sh, sigma, chunk=chunk, two_pass=two_pass)
    td = G.gpu_build(S, sigma)
    try:
        assert st["chunks"] == -(-n // min(chunk, n)) and st["pinned"] == int(pinned)
        assert st["passes"] == (2 if two_pass or sigma == 1 else 1)
        same_tree(th, td)
        G.compare_structure(th, oracle.OracleTree(S, sigma))
        G.compare_queries(th, S, sigma, *G.edge_queries(S, sigma))
        G.compare_queries(th, S, sigma, *G.random_queries(S, sigma, 4096, 0x4B11 + n))
    finally:
        th.free()
        td.free()
    del keep


def test_host_build_wide_codes_and_options():
    import paper_2505_03372_amd as wt
    n, sigma = 1 << 20, 60000
    G.log("host build: full-width codes, |L2| 1024, s 1024")
    S = make_seq("zipf", n, sigma, 2, 0x4B12)
    th, _ = wt.build_host(S, sigma, chunk=1 << 17, wide=True, l2_bits=1024, sample_rate=1024)
    td = G.gpu_build(S, sigma, l2_bits=1024, sample_rate=1024)
    try:
        same_tree(th, td)
    finally:
        th.free()
        td.free()


def test_host_build_more_than_1024_tiles():
    """2^24 + 123 u8 symbols in chunks of 2^22 (five chunks): 1025 tiles per level, every part equal to
    the device build's; binned queries against the oracle on a sample."""
    import paper_2505_03372_amd as wt
    n, sigma = (1 << 24) + 123, 256
    G.log("host build: n=%d u8 (1025 tiles per level), chunks of 2^22" % n)
    S = make_seq("zipf", n, sigma, 1, 0x4B13)
    Sh, keep = _pinned(S)
    th, st = wt.build_host(Sh, sigma, chunk=1 << 22)
    t2, st2 = wt.build_host(Sh, sigma, chunk=1 << 22, two_pass=True)
    td = G.gpu_build(S, sigma)
    try:
        assert st["chunks"] == 5 and st["passes"] == 1 and st2["passes"] == 2
        same_tree(t2, td)
        same_tree(th, td)
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, 1 << 17, 0x4B14)
        smp = workloads.uniform(0x4B15, 4096, 1 << 17).astype(np.int64)
        np.testing.assert_array_equal(G.host(th.select(G.dev(sc), G.dev(sk)))[smp],
                                      oracle.select(S, sigma, sc[smp], sk[smp]))
        np.testing.assert_array_equal(G.host(th.rank(G.dev(rc), G.dev(ri)))[smp],
                                      oracle.rank(S, sigma, rc[smp], ri[smp]))
    finally:
        th.free()
        t2.free()
        td.free()
    del keep


def test_host_build_refusals():
    import paper_2505_03372_amd as wt
    S = workloads.uniform(0x4B16, 100000, 10, 1)
    with pytest.raises(wt.WTError):
        wt.build_host(S, 0)
    with pytest.raises(wt.WTError):
        wt.build_host(S, 10, chunk=1000)
    bad = S.copy()
    bad[99999] = 10
    with pytest.raises(wt.WTError):
        wt.build_host(bad, 10, chunk=1 << 16)
    t, st = wt.build_host(np.zeros(0, np.uint8), 10)
    try:
        assert t.info["n"] == 0
    finally:
        t.free()

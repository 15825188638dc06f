"""GPU parity of the wavelet matrix (wt_build with WT_BUILD_MATRIX; the layout the thesis's Conclusion
names as further work), bit-exact against the oracle.

* every level's bits, L1/L2 directory and select samples, the ones per level and every symbol's start
  below the last level equal the oracle matrix's (plain definition: per level, S stably sorted by the
  reversed top bits of the symbols), for widths 1/2/4, alphabets that are powers of two and not, from
  1 to 2^20, lengths around the word, L2, tile and L1 boundaries, and one level of more than 1024 tiles;
* access / rank / select answers, random and at the boundaries, equal the oracle's (answers do not
  depend on the layout), in unbinned and binned batches, through wt_select_noalloc too;
* the matrix of an extracted alphabet (sigma = 0) answers in the caller's values;
* the calls that need the tree's node table refuse a matrix.
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


def compare_matrix(t, om: "oracle.OracleMatrix"):
    import paper_2505_03372_amd as wt
    info = t.info
    assert info["matrix"] and info["levels"] == om.L
    assert info["level_n"] == [om.n] * om.L
    assert info["level_ones"] == om.ones, (info["level_ones"], om.ones)
    assert [om.n - o for o in info["level_ones"]] == om.zeros
    np.testing.assert_array_equal(t.export(wt.PART_WM_STARTS), om.starts)
    parts = {"bits": (wt.PART_BITS, om.bits), "L1": (wt.PART_L1, om.L1), "L2": (wt.PART_L2, om.L2),
             "samples1": (wt.PART_SAMPLES1, om.samples1), "samples0": (wt.PART_SAMPLES0, om.samples0)}
    for l in range(om.L):
        for name, (part, ref) in parts.items():
            got, exp = t.export(part, l), ref[l]
            assert got.shape == exp.shape, (name, l, got.shape, exp.shape)
            if not np.array_equal(got, exp):
                bad = np.nonzero(got != exp)[0]
                raise AssertionError("%s level %d differs at %d places, first %d: got %d expected %d"
                                     % (name, l, bad.size, bad[0], got[bad[0]], exp[bad[0]]))


# (width, sigma, n, kind, l2_bits, sample_rate)
CASES = [
    (1, 256, 1 << 20, "uniform", 512, 4096),
    (1, 256, 300001, "zipf", 512, 4096),
    (1, 2, 100003, "uniform", 512, 512),
    (1, 3, 65537, "uniform", 512, 4096),
    (1, 5, 70000, "zipf", 512, 512),
    (1, 6, 16385, "alternate", 512, 512),
    (1, 7, 131073, "runs", 512, 512),
    (1, 200, 250000, "zipf", 256, 1024),
    (1, 255, 99999, "uniform", 1024, 2048),
    (1, 256, 200000, "equal", 2048, 512),
    (1, 4, 1, "uniform", 512, 4096),
    (1, 11, 63, "uniform", 512, 4096),
    (1, 11, 65, "uniform", 512, 4096),
    (1, 13, 513, "zipf", 512, 4096),
    (1, 16, 16384, "uniform", 512, 4096),
    (1, 9, 65536, "uniform", 512, 512),
    (1, 1, 1000, "equal", 512, 4096),
    (1, 4, 0, "uniform", 512, 4096),
    (2, 65536, 400000, "zipf", 512, 4096),
    (2, 25, 200000, "zipf", 512, 4096),
    (2, 40000, 300000, "uniform", 512, 2048),
    (2, 60001, 100000, "sparse", 512, 4096),
    (4, 1 << 20, 1 << 21, "zipf12", 512, 4096),
    (4, 12345, 200000, "uniform", 256, 4096),
    (4, 3, 100001, "alternate", 512, 512),
    (4, 1000003, 300000, "sparse", 512, 4096),
]


@pytest.mark.parametrize("width,sigma,n,kind,l2,s", CASES)
def test_matrix_structure_and_queries(width, sigma, n, kind, l2, s):
    G.log("matrix: width=%d sigma=%d n=%d %s l2=%d s=%d" % (width, sigma, n, kind, l2, s))
    S = make_seq(kind, n, sigma, width, 0x3A70 + n + sigma)
    t = G.gpu_build(S, sigma, l2_bits=l2, sample_rate=s, matrix=True)
    try:
        compare_matrix(t, oracle.OracleMatrix(S, sigma, l2_bits=l2, sample_rate=s))
        G.compare_queries(t, S, sigma, *G.edge_queries(S, sigma))
        G.compare_queries(t, S, sigma, *G.random_queries(S, sigma, 4096, 0x3A71 + n))
    finally:
        t.free()


def test_matrix_more_than_1024_tiles_per_level():
    """2^24 + 123 u8 symbols: 1025 tiles per level (the chunked tile prefix), every part and a sample of
    binned queries of each kind."""
    n, sigma = (1 << 24) + 123, 256
    G.log("matrix: n=%d u8 sigma=%d (1025 tiles per level)" % (n, sigma))
    S = make_seq("zipf", n, sigma, 1, 0x3A72)
    t = G.gpu_build(S, sigma, matrix=True)
    try:
        compare_matrix(t, oracle.OracleMatrix(S, sigma))
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, 1 << 18, 0x3A73)
        smp = workloads.uniform(0x3A74, 8192, 1 << 18).astype(np.int64)
        acc = G.host(t.access(G.dev(pos)))
        rk = G.host(t.rank(G.dev(rc), G.dev(ri)))
        sl = G.host(t.select(G.dev(sc), G.dev(sk)))
        np.testing.assert_array_equal(acc[smp], oracle.access(S, pos[smp]))
        np.testing.assert_array_equal(rk[smp], oracle.rank(S, sigma, rc[smp], ri[smp]))
        np.testing.assert_array_equal(sl[smp], oracle.select(S, sigma, sc[smp], sk[smp]))
        # whole-batch properties: access reproduces S, select inverts rank
        np.testing.assert_array_equal(acc, S[pos.astype(np.int64)])
        np.testing.assert_array_equal(G.host(t.access(G.dev(sl))), sc)
        np.testing.assert_array_equal(G.host(t.rank(G.dev(sc), G.dev(sl))), sk - 1)
    finally:
        t.free()


@pytest.mark.parametrize("width,sigma,n", [(1, 256, (1 << 21) + 777), (2, 1000, 1 << 20), (4, 1 << 20, 1 << 20)])
def test_matrix_binned_batches_equal_tree(width, sigma, n):
    """Batches of 2^17 queries (binned) on a matrix and on the tree of the same sequence give the same
    answers, which equal the oracle on a sample; select also through wt_select_noalloc."""
    import torch
    G.log("matrix vs tree, binned: width=%d sigma=%d n=%d" % (width, sigma, n))
    S = make_seq("zipf", n, sigma, width, 0x3A75 + sigma)
    tm = G.gpu_build(S, sigma, matrix=True)
    tt = G.gpu_build(S, sigma)
    try:
        q = 1 << 17
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, q, 0x3A76 + sigma)
        dpos, drc, dri, dsc, dsk = (G.dev(a) for a in (pos, rc, ri, sc, sk))
        for name, fm, ft in (("access", lambda t: t.access(dpos), None),
                             ("rank", lambda t: t.rank(drc, dri), None),
                             ("select", lambda t: t.select(dsc, dsk), None)):
            got, exp = G.host(fm(tm)), G.host(fm(tt))
            assert np.array_equal(got, exp), "%s: matrix and tree differ at %d places" % (
                name, int(np.count_nonzero(got != exp)))
        out = torch.empty(q, dtype=torch.uint64, device="cuda")
        tm.select_noalloc(dsc, dsk, out)
        np.testing.assert_array_equal(G.host(out), G.host(tt.select(dsc, dsk)))
        smp = workloads.uniform(0x3A77, 2048, q).astype(np.int64)
        np.testing.assert_array_equal(G.host(out)[smp], oracle.select(S, sigma, sc[smp], sk[smp]))
    finally:
        tm.free()
        tt.free()


def test_matrix_extracted_alphabet():
    import paper_2505_03372_amd as wt
    n, d = 300000, 300
    G.log("matrix: extracted alphabet of %d u32 values" % d)
    vals = np.sort(np.unique(workloads.raw(0x3A78, 0, 4 * d) % np.uint64(1 << 31)))[:d].astype(np.uint32)
    idx = workloads.zipf(0x3A79, n, vals.size, 1.0, 4, workloads.permutation(0x3A7A, vals.size))
    S = vals[idx.astype(np.int64)].astype(np.uint32)
    t = wt.build(G.dev(S), 0, matrix=True)
    try:
        assert t.info["matrix"] and t.info["alphabet_extracted"] and t.info["sigma"] == vals.size
        np.testing.assert_array_equal(t.export(wt.PART_ALPHABET), vals)
        codes = np.searchsorted(vals, S).astype(np.uint32)
        compare_matrix(t, oracle.OracleMatrix(codes, int(vals.size)))
        pos, rc, ri, sc, sk = G.random_queries(codes, int(vals.size), 4096, 0x3A7B)
        np.testing.assert_array_equal(G.host(t.access(G.dev(pos))), vals[oracle.access(codes, pos).astype(np.int64)])
        np.testing.assert_array_equal(G.host(t.rank(G.dev(vals[rc.astype(np.int64)]), G.dev(ri))),
                                      oracle.rank(codes, int(vals.size), rc, ri))
        np.testing.assert_array_equal(G.host(t.select(G.dev(vals[sc.astype(np.int64)]), G.dev(sk))),
                                      oracle.select(codes, int(vals.size), sc, sk))
    finally:
        t.free()


def test_matrix_refuses_node_table_calls():
    import paper_2505_03372_amd as wt
    S = workloads.uniform(0x3A7C, 5000, 10, 1)
    t = G.gpu_build(S, 10, matrix=True)
    try:
        with pytest.raises(wt.WTError):
            t.export(wt.PART_NODE_START, 0)
        with pytest.raises(wt.WTError):
            t.learn_select()
    finally:
        t.free()
    t2 = G.gpu_build(S, 10)
    try:
        with pytest.raises(wt.WTError):
            t2.export(wt.PART_WM_STARTS)
    finally:
        t2.free()

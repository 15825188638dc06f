"""GPU parity of the Huffman-shaped tree (wt_build with WT_BUILD_HUFFMAN), bit-exact against the oracle.

* the code table (length and code of every symbol), the number of levels, every level's size, ones,
  bits, L1/L2 directory, select samples and node table, and the cumulative histogram equal the
  oracle's Huffman-shaped tree (package-merge lengths, canonical codes with the longer codes left),
  for widths 1/2/4, codes of 1, 2 and 4 bytes (up to 20 bits), alphabets with absent symbols, two
  and one occurring symbols, the empty sequence, lengths around the word, L2, tile and L1 boundaries,
  and a first level of more than 1024 tiles;
* access / rank / select answers (random and at the boundaries) equal the oracle's, in unbinned and
  binned batches, through wt_select_noalloc and the host-sourced pipeline too;
* narrow and full-width carried codes give the same tree; an extracted alphabet answers in the
  caller's values; the learned index and WT_BUILD_MATRIX refuse the Huffman shape.
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


def skewed(seed, n, sigma, width, alpha):
    """Zipf(alpha) symbols over a shuffled alphabet (long codes for the rare symbols)."""
    return workloads.zipf(seed, n, sigma, alpha, width, workloads.permutation(seed + 1, sigma))


def geometric(seed, n, sigma, width):
    """Counts halving from symbol to symbol (the code lengths reach the length limit), shuffled."""
    cnt = np.maximum(1, (n // 2) >> np.arange(sigma)).astype(np.int64)
    cnt[0] += n - int(cnt.sum())
    S = np.repeat(np.arange(sigma), cnt)
    return S[workloads.permutation(seed, S.size)].astype(workloads.dtype_for(width))


def compare_huffman(t, S, sigma, l2=512, s=4096):
    import paper_2505_03372_amd as wt
    ot = oracle.OracleTree(S, sigma, l2_bits=l2, sample_rate=s, huffman=True)
    info = t.info
    assert info["huffman"] and not info["matrix"]
    codes = t.export(wt.PART_HUFF_CODES)
    ln = (codes >> np.uint64(32)).astype(np.uint32)
    right = (codes & np.uint64(0xFFFFFFFF))
    np.testing.assert_array_equal(ln, ot.lens)
    shift = np.where(ot.lens > 0, ot.L - ot.lens.astype(np.int64), 0).astype(np.uint64)
    np.testing.assert_array_equal(right, ot.codes >> shift)
    G.compare_structure(t, ot)
    return ot


# (width, sigma, n, kind, l2_bits, sample_rate)
CASES = [
    (1, 256, 1 << 20, "zipf", 512, 4096),
    (1, 256, 300001, "uniform", 512, 4096),
    (1, 2, 100003, "uniform", 512, 512),
    (1, 3, 65537, "zipf", 512, 4096),
    (1, 6, 16385, "alternate", 512, 512),   # two occurring symbols: one level
    (1, 200, 250000, "zipf", 256, 1024),
    (1, 255, 99999, "skew15", 1024, 2048),
    (1, 40, 1 << 20, "geometric", 512, 4096),  # the length limit binds (ceil(lg 40) + 8 = 14 bits)
    (1, 256, 200000, "equal", 2048, 512),      # one occurring symbol: no level
    (1, 11, 63, "zipf", 512, 4096),
    (1, 11, 65, "zipf", 512, 4096),
    (1, 13, 513, "zipf", 512, 4096),
    (1, 4, 0, "uniform", 512, 4096),
    (2, 65536, 400000, "zipf", 512, 4096),
    (2, 1000, 300000, "skew15", 512, 2048),
    (2, 60001, 100000, "sparse", 512, 4096),   # seven symbols of a large alphabet
    (4, 4096, 1 << 22, "skew15", 512, 4096),   # codes of up to 20 bits (4-byte carried codes)
    (4, 12345, 200000, "uniform", 256, 4096),
    (4, 1000003, 300000, "sparse", 512, 4096),
]


def _seq(kind, n, sigma, w, seed):
    if kind == "skew15":
        return skewed(seed, n, sigma, w, 1.5)
    if kind == "geometric":
        return geometric(seed, n, sigma, w)
    return make_seq(kind, n, sigma, w, seed)


@pytest.mark.parametrize("width,sigma,n,kind,l2,s", CASES)
def test_huffman_structure_and_queries(width, sigma, n, kind, l2, s):
    G.log("huffman: width=%d sigma=%d n=%d %s l2=%d s=%d" % (width, sigma, n, kind, l2, s))
    S = _seq(kind, n, sigma, width, 0x4A10 + n + sigma)
    t = G.gpu_build(S, sigma, l2_bits=l2, sample_rate=s, huffman=True)
    try:
        ot = compare_huffman(t, S, sigma, l2, s)
        if kind == "geometric":
            assert ot.L == oracle.huffman_limit(sigma) == 14
        G.compare_queries(t, S, sigma, *G.edge_queries(S, sigma))
        G.compare_queries(t, S, sigma, *G.random_queries(S, sigma, 4096, 0x4A11 + n))
    finally:
        t.free()


def test_huffman_more_than_1024_tiles():
    """2^24 + 123 u8 Zipf symbols (2-byte codes: 2049 tiles at level 0): every part, the binned
    answers of each kind on a sample, and whole-batch properties."""
    n, sigma = (1 << 24) + 123, 256
    G.log("huffman: n=%d u8 sigma=%d (more than 1024 tiles per level)" % (n, sigma))
    S = make_seq("zipf", n, sigma, 1, 0x4A12)
    t = G.gpu_build(S, sigma, huffman=True)
    try:
        ot = compare_huffman(t, S, sigma)
        assert ot.L > 8  # codes wider than a byte
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, 1 << 18, 0x4A13)
        smp = workloads.uniform(0x4A14, 8192, 1 << 18).astype(np.int64)
        acc = G.host(t.access(G.dev(pos)))
        rk = G.host(t.rank(G.dev(rc), G.dev(ri)))
        sl = G.host(t.select(G.dev(sc), G.dev(sk)))
        np.testing.assert_array_equal(acc[smp], oracle.access(S, pos[smp]))
        np.testing.assert_array_equal(rk[smp], oracle.rank(S, sigma, rc[smp], ri[smp]))
        np.testing.assert_array_equal(sl[smp], oracle.select(S, sigma, sc[smp], sk[smp]))
        np.testing.assert_array_equal(acc, S[pos.astype(np.int64)])
        np.testing.assert_array_equal(G.host(t.access(G.dev(sl))), sc)
        np.testing.assert_array_equal(G.host(t.rank(G.dev(sc), G.dev(sl))), sk - 1)
    finally:
        t.free()


@pytest.mark.parametrize("width,sigma,n,kind", [(1, 256, (1 << 21) + 777, "zipf"), (2, 1000, 1 << 20, "skew15"),
                                                (4, 4096, 1 << 21, "skew15")])
def test_huffman_binned_and_narrow_equal_wide(width, sigma, n, kind):
    """Narrow and full-width carried codes build the same tree; binned batches of 2^17 queries on the
    Huffman-shaped tree and on the balanced tree of the same sequence give the same answers; select
    also through wt_select_noalloc and from host memory."""
    import torch
    import paper_2505_03372_amd as wt
    G.log("huffman binned / narrow vs wide: width=%d sigma=%d n=%d %s" % (width, sigma, n, kind))
    S = _seq(kind, n, sigma, width, 0x4A15 + sigma)
    th = G.gpu_build(S, sigma, huffman=True, narrow=True)
    tw = G.gpu_build(S, sigma, huffman=True, wide=True)
    tt = G.gpu_build(S, sigma)
    try:
        assert th.info["level_n"] == tw.info["level_n"]
        for l in range(th.info["levels"]):
            for part in (wt.PART_BITS, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START):
                np.testing.assert_array_equal(th.export(part, l), tw.export(part, l))
        q = 1 << 17
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, q, 0x4A16 + sigma)
        dpos, drc, dri, dsc, dsk = (G.dev(a) for a in (pos, rc, ri, sc, sk))
        for name, f in (("access", lambda t: t.access(dpos)), ("rank", lambda t: t.rank(drc, dri)),
                        ("select", lambda t: t.select(dsc, dsk))):
            got, exp = G.host(f(th)), G.host(f(tt))
            assert np.array_equal(got, exp), "%s: Huffman-shaped and balanced trees differ at %d places" % (
                name, int(np.count_nonzero(got != exp)))
        out = torch.empty(q, dtype=torch.uint64, device="cuda")
        th.select_noalloc(dsc, dsk, out)
        np.testing.assert_array_equal(G.host(out), G.host(tt.select(dsc, dsk)))
        got, _ = th.query_host(wt.OP_SELECT, sk, sc, chunk=40000)
        np.testing.assert_array_equal(got, G.host(tt.select(dsc, dsk)))
        smp = workloads.uniform(0x4A17, 2048, q).astype(np.int64)
        np.testing.assert_array_equal(G.host(out)[smp], oracle.select(S, sigma, sc[smp], sk[smp]))
    finally:
        th.free()
        tw.free()
        tt.free()
        wt.lib().wt_query_host_release()


def test_huffman_extracted_alphabet():
    import paper_2505_03372_amd as wt
    n, d = 300000, 300
    G.log("huffman: extracted alphabet of %d u32 values" % d)
    vals = np.sort(np.unique(workloads.raw(0x4A18, 0, 4 * d) % np.uint64(1 << 31)))[:d].astype(np.uint32)
    idx = workloads.zipf(0x4A19, n, vals.size, 1.0, 4, workloads.permutation(0x4A1A, vals.size))
    S = vals[idx.astype(np.int64)].astype(np.uint32)
    t = wt.build(G.dev(S), 0, huffman=True)
    try:
        assert t.info["huffman"] and t.info["alphabet_extracted"] and t.info["sigma"] == vals.size
        codes = np.searchsorted(vals, S).astype(np.uint32)
        compare_huffman(t, codes, int(vals.size))
        pos, rc, ri, sc, sk = G.random_queries(codes, int(vals.size), 4096, 0x4A1B)
        np.testing.assert_array_equal(G.host(t.access(G.dev(pos))), vals[oracle.access(codes, pos).astype(np.int64)])
        np.testing.assert_array_equal(G.host(t.rank(G.dev(vals[rc.astype(np.int64)]), G.dev(ri))),
                                      oracle.rank(codes, int(vals.size), rc, ri))
        np.testing.assert_array_equal(G.host(t.select(G.dev(vals[sc.astype(np.int64)]), G.dev(sk))),
                                      oracle.select(codes, int(vals.size), sc, sk))
    finally:
        t.free()


def test_huffman_refusals():
    import paper_2505_03372_amd as wt
    S = workloads.uniform(0x4A1C, 5000, 10, 1)
    with pytest.raises(wt.WTError):
        G.gpu_build(S, 10, huffman=True, matrix=True)
    t = G.gpu_build(S, 10, huffman=True)
    try:
        with pytest.raises(wt.WTError):
            t.learn_select()
    finally:
        t.free()
    t2 = G.gpu_build(S, 10)
    try:
        with pytest.raises(wt.WTError):
            t2.export(wt.PART_HUFF_CODES)
    finally:
        t2.free()
    # a symbol out of range is reported by the histogram pass that comes first
    bad = S.copy()
    bad[77] = 12
    with pytest.raises(wt.WTError):
        G.gpu_build(bad, 10, huffman=True)

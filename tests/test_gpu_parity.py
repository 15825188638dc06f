"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Small and medium cases compare the whole structure (level bits, L1/L2, samples, node tables,
cumulative histogram) and the answers to random and boundary queries. The workloads of the
benchmark run at full size in the launch configuration bench.py times, with the answers of a
sample of the queries checked against the oracle's sweep.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_03372_amd as wt
    wt.lib()  # fails loudly when the HIP library is missing


def make_seq(kind, n, sigma, width, seed):
    dt = workloads.dtype_for(width)
    if kind == "uniform":
        return workloads.uniform(seed, n, sigma, width)
    if kind == "zipf":
        return workloads.zipf(seed, n, sigma, 1.0, width, workloads.permutation(seed + 1, sigma))
    if kind == "zipf12":
        return workloads.zipf(seed, n, sigma, 1.2, width, workloads.permutation(seed + 1, sigma))
    if kind == "equal":
        return np.full(n, sigma - 1, dtype=dt)
    if kind == "alternate":
        return ((np.arange(n) % 2) * (sigma - 1)).astype(dt)
    if kind == "runs":
        return np.sort(workloads.uniform(seed, n, sigma, width))
    if kind == "sparse":  # few distinct symbols spread over a large alphabet
        vals = workloads.uniform(seed + 2, 7, sigma, 8).astype(np.uint64)
        return vals[workloads.uniform(seed, n, 7, 8)].astype(dt)
    raise ValueError(kind)


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
    (1, 4, 2, "uniform", 512, 4096),
    (1, 11, 63, "uniform", 512, 4096),
    (1, 11, 64, "uniform", 512, 4096),
    (1, 11, 65, "uniform", 512, 4096),
    (1, 13, 511, "zipf", 512, 4096),
    (1, 13, 512, "zipf", 512, 4096),
    (1, 13, 513, "zipf", 512, 4096),
    (1, 16, 16383, "uniform", 512, 4096),
    (1, 16, 16384, "uniform", 512, 4096),
    (1, 9, 65536, "uniform", 512, 512),
    (1, 1, 1000, "equal", 512, 4096),
    (1, 4, 0, "uniform", 512, 4096),
    (2, 65536, 400000, "zipf", 512, 4096),
    (2, 25, 200000, "zipf", 512, 4096),
    (2, 40000, 300000, "uniform", 512, 2048),
    (2, 4, 8193, "uniform", 512, 512),
    (2, 1000, 150000, "runs", 512, 4096),
    (2, 60001, 100000, "sparse", 512, 4096),
    (4, 1 << 20, 1 << 21, "zipf12", 512, 4096),
    (4, 12345, 200000, "uniform", 256, 4096),
    (4, 3, 100001, "alternate", 512, 512),
    (4, 1 << 20, 300000, "sparse", 512, 4096),
    (4, 70001, 4097, "uniform", 512, 4096),
    (4, 1 << 24, 200000, "uniform", 512, 4096),   # 512 histogram windows of 2^15 symbols
    (4, 1000003, 500000, "zipf12", 512, 4096),    # last window partly used
]


@pytest.mark.parametrize("width,sigma,n,kind,l2,srate", CASES,
                         ids=["w%d-s%d-n%d-%s-l2_%d-s%d" % c for c in CASES])
def test_structure_and_answers(width, sigma, n, kind, l2, srate):
    seed = 0xC0FFEE + 31 * n + sigma + width
    S = make_seq(kind, n, sigma, width, seed)
    G.log("case w=%d sigma=%d n=%d kind=%s l2=%d s=%d seed=%#x: build" % (width, sigma, n, kind, l2, srate, seed))
    t = G.gpu_build(S, sigma, l2_bits=l2, sample_rate=srate)
    ot = oracle.OracleTree(S, sigma, l2_bits=l2, sample_rate=srate)
    G.compare_structure(t, ot)
    G.log("  queries")
    G.compare_queries(t, S, sigma, *G.random_queries(S, sigma, 4096, seed))
    G.compare_queries(t, S, sigma, *G.edge_queries(S, sigma))
    t.free()


# More than 1024 tiles per level (the tile prefix then runs in chunks of 1024 tiles): the whole
# structure against the oracle, with a ragged last tile.
BIG_CASES = [
    (1, 256, (1 << 25) + 12345, "zipf", 512, 4096),   # 2049 tiles of 16384 u8 symbols
    (4, 70001, 5_000_003, "zipf12", 512, 4096),       # 1221 tiles of 4096 u32 symbols, reduced codes
]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("width,sigma,n,kind,l2,srate", BIG_CASES,
                         ids=["w%d-s%d-n%d-%s-l2_%d-s%d" % c for c in BIG_CASES])
def test_structure_above_1024_tiles(width, sigma, n, kind, l2, srate):
    seed = 0xB16 + width
    S = make_seq(kind, n, sigma, width, seed)
    G.log("big case w=%d sigma=%d n=%d kind=%s: build" % (width, sigma, n, kind))
    t = G.gpu_build(S, sigma, l2_bits=l2, sample_rate=srate)
    G.log("  oracle tree")
    ot = oracle.OracleTree(S, sigma, l2_bits=l2, sample_rate=srate)
    G.compare_structure(t, ot)
    G.log("  queries")
    G.compare_queries(t, S, sigma, *G.random_queries(S, sigma, 1 << 14, seed))
    G.compare_queries(t, S, sigma, *G.edge_queries(S, sigma))
    t.free()


def test_plain_small_config_exact():
    wl = workloads.make("plain_small")
    G.log("plain_small: n=%d sigma=%d build" % (wl.n, wl.sigma))
    t = G.gpu_build(wl.S, wl.sigma)
    G.compare_structure(t, oracle.OracleTree(wl.S, wl.sigma))
    G.log("plain_small: 2^16 queries of each kind")
    G.compare_queries(t, wl.S, wl.sigma, wl.acc_pos, wl.rank_c, wl.rank_i, wl.sel_c, wl.sel_k)
    t.free()


def test_symbol_out_of_range_is_reported():
    import paper_2505_03372_amd as wt
    S = workloads.uniform(5, 50000, 10, 1)
    S[12345] = 200
    G.log("out-of-range build")
    with pytest.raises(wt.WTError) as ei:
        G.gpu_build(S, 10)
    assert ei.value.status == wt.WT_ERR_SYMBOL_RANGE
    # the library stays usable
    t = G.gpu_build(S[:12345].copy(), 10)
    G.compare_queries(t, S[:12345], 10, *G.random_queries(S[:12345], 10, 512, 9))
    t.free()


@pytest.mark.parametrize("width,sigma", [(1, 10), (2, 40000), (4, 1 << 20)])
def test_symbol_out_of_range_is_reported_every_histogram(width, sigma):
    """Each histogram variant (replicated LDS counters, LDS windows, the windowed radix step for
    alphabets above 2^16) flags a symbol >= sigma, and builds nothing."""
    import paper_2505_03372_amd as wt
    S = workloads.uniform(6, 300000, sigma, width)
    S[299999] = sigma
    G.log("out-of-range build w=%d sigma=%d" % (width, sigma))
    with pytest.raises(wt.WTError) as ei:
        G.gpu_build(S, sigma)
    assert ei.value.status == wt.WT_ERR_SYMBOL_RANGE


@pytest.mark.parametrize("width,sigma,shift", [(1, 7, 1), (1, 200, 13), (1, 200, 5), (1, 256, 3), (2, 1000, 1),
                                               (2, 40000, 5), (2, 7, 7), (2, 300, 3), (2, 1 << 16, 3), (4, 3000, 1),
                                               (4, 3000, 3), (4, 1 << 20, 2)])
def test_unaligned_input_pointer(width, sigma, shift):
    """Symbols starting `shift` elements past a 16-byte boundary: every vector of the histogram and of
    level 0 is read across two aligned blocks (each funnel shift, whole tiles and the ragged last
    one; alphabets covering the whole symbol type take the histogram's full-range count;
    non-power-of-two alphabets take the reduced codes of level 0)."""
    import torch
    import paper_2505_03372_amd as wt
    n = 70001
    S = workloads.uniform(77 + shift, n, sigma, width)
    d = torch.from_numpy(np.concatenate([np.zeros(shift, dtype=S.dtype), S])).cuda()[shift:]
    assert d.data_ptr() % 16 == (shift * width) % 16 != 0
    G.log("unaligned input build w=%d sigma=%d shift=%d" % (width, sigma, shift))
    t = wt.build(d, sigma)
    G.compare_structure(t, oracle.OracleTree(S, sigma))
    t.free()


def test_build_profile_entries():
    S = workloads.uniform(3, 1 << 18, 256, 1)
    t = G.gpu_build(S, 256, profile=True)
    prof = t.profile()
    levels = [p for p in prof if p["kernel"] == "level"]
    assert [p["level"] for p in levels] == list(range(8))
    assert all(p["ms"] > 0 for p in levels)
    t.free()


def _sampled_check(t, S, sigma, acc_pos, rank_c, rank_i, sel_c, sel_k, stride):
    import torch
    if acc_pos is not None:
        G.log("  access batch of %d" % acc_pos.size)
        got = G.host(t.access(G.dev(acc_pos)))
        idx = np.arange(0, acc_pos.size, stride)
        G._assert_eq("access", got[idx], oracle.access(S, acc_pos[idx]), acc_pos[idx])
    if rank_c is not None:
        G.log("  rank batch of %d" % rank_c.size)
        got = G.host(t.rank(G.dev(rank_c), G.dev(rank_i)))
        idx = np.arange(0, rank_c.size, stride)
        G._assert_eq("rank", got[idx], oracle.rank(S, sigma, rank_c[idx], rank_i[idx]), rank_i[idx])
    if sel_c is not None:
        G.log("  select batch of %d" % sel_c.size)
        got = G.host(t.select(G.dev(sel_c), G.dev(sel_k)))
        idx = np.arange(0, sel_c.size, stride)
        G._assert_eq("select", got[idx], oracle.select(S, sigma, sel_c[idx], sel_k[idx]), sel_k[idx])
    torch.cuda.synchronize()


def _level_properties(t, S, sigma):
    code, ln = oracle.codes(sigma)
    hist = np.bincount(S, minlength=sigma).astype(np.int64)
    L = t.info["levels"]
    for l in range(L):
        live = ln > l
        bit = ((code.astype(np.int64) >> (L - 1 - l)) & 1).astype(bool)
        assert t.info["level_n"][l] == int(hist[live].sum())
        assert t.info["level_ones"][l] == int(hist[live & bit].sum())


def test_full_size_text_zipf():
    """n = 2^30 u8, Zipf(1.0) over 256 symbols; 2^26 queries of each kind (sampled check)."""
    G.log("text_zipf: generating 2^30 symbols")
    wl = workloads.make("text_zipf")
    G.log("text_zipf: build")
    t = G.gpu_build(wl.S, wl.sigma)
    _level_properties(t, wl.S, wl.sigma)
    _sampled_check(t, wl.S, wl.sigma, wl.acc_pos, wl.rank_c, wl.rank_i, wl.sel_c, wl.sel_k, stride=1024)
    t.free()


def test_full_size_large_alphabet():
    """n = 2^28 u32, sigma = 2^20 (half uniform, half Zipf(1.2)); 2^24 rank and select (sampled check)."""
    G.log("large_alpha: generating 2^28 symbols")
    wl = workloads.make("large_alpha", kinds=("rank", "select"))
    G.log("large_alpha: build")
    t = G.gpu_build(wl.S, wl.sigma)
    _level_properties(t, wl.S, wl.sigma)
    _sampled_check(t, wl.S, wl.sigma, None, wl.rank_c, wl.rank_i, wl.sel_c, wl.sel_k, stride=256)
    t.free()


@pytest.mark.parametrize("order", ["random", "sorted", "reversed", "one_position"])
def test_binned_batches_equal_unbinned(order):
    """Batches of at least 2^16 queries are binned by where their answers lie before the traversal;
    their answers must equal those of the same queries asked in batches below the binning size."""
    import paper_2505_03372_amd as wt
    n, sigma = 3_000_017, 300
    S = make_seq("zipf", n, sigma, 2, 0x5151)
    t = G.gpu_build(S, sigma)
    q = (1 << 17) + 33
    pos, rc, ri, sc, sk = G.random_queries(S, sigma, q, 0x77)
    if order == "sorted":
        o = np.argsort(pos, kind="stable"); pos = pos[o]; o = np.lexsort((ri, rc)); rc, ri = rc[o], ri[o]
        o = np.lexsort((sk, sc)); sc, sk = sc[o], sk[o]
    elif order == "reversed":
        pos, rc, ri, sc, sk = pos[::-1].copy(), rc[::-1].copy(), ri[::-1].copy(), sc[::-1].copy(), sk[::-1].copy()
    elif order == "one_position":
        pos[:] = n // 2; ri[:] = n // 2; sc[:] = sc[0]; sk[:] = 1
    # out-of-domain arguments mixed in
    pos[::97] = n + 5; ri[::89] = n + 1; rc[::83] = sigma + 3; sk[::79] = 0; sc[::73] = sigma
    G.log("binned vs unbinned, order %s, q=%d" % (order, q))
    def pieces(fn, *arrs):
        step = (1 << 16) - 1
        return np.concatenate([G.host(fn(*[G.dev(np.ascontiguousarray(a[i:i + step])) for a in arrs]))
                               for i in range(0, q, step)])
    got = G.host(t.access(G.dev(pos)))
    G._assert_eq("access binned", got, pieces(t.access, pos), pos)
    got = G.host(t.rank(G.dev(rc), G.dev(ri)))
    G._assert_eq("rank binned", got, pieces(t.rank, rc, ri), ri)
    got = G.host(t.select(G.dev(sc), G.dev(sk)))
    G._assert_eq("select binned", got, pieces(t.select, sc, sk), sk)
    t.learn_select()
    got = G.host(t.select_learned(G.dev(sc), G.dev(sk)))
    G._assert_eq("learned select binned", got, pieces(t.select, sc, sk), sk)
    idx = np.arange(0, q, 61)
    G._assert_eq("select vs oracle", got[idx], oracle.select(S, sigma, sc[idx], sk[idx]), sk[idx])
    t.free()


@pytest.mark.parametrize("order", ["random", "one_position", "two_values"])
def test_two_pass_binning_equals_one_pass(order):
    """Batches of 2^24 queries and more are binned in two passes (coarse bucket groups, then buckets);
    their answers equal those of the same queries asked in batches binned in one pass, and the oracle's
    on a sample. one_position / two_values put the whole batch into one or two buckets."""
    n, sigma = 3_000_017, 300
    S = make_seq("zipf", n, sigma, 2, 0x5152)
    t = G.gpu_build(S, sigma)
    q = (1 << 24) + 77
    pos, rc, ri, sc, sk = G.random_queries(S, sigma, q, 0x78)
    if order == "one_position":
        pos[:] = n // 3; ri[:] = n // 3; sc[:] = sc[0]; sk[:] = 2
    elif order == "two_values":
        pos[::2] = 5; ri[::2] = n; sk[1::2] = 1
    pos[::97] = n + 5; ri[::89] = n + 1; rc[::83] = sigma + 3; sk[::79] = 0; sc[::73] = sigma
    G.log("two-pass binning, order %s, q=%d" % (order, q))

    def pieces(fn, *arrs):
        step = 1 << 22
        return np.concatenate([G.host(fn(*[G.dev(np.ascontiguousarray(a[i:i + step])) for a in arrs]))
                               for i in range(0, q, step)])
    got = G.host(t.access(G.dev(pos)))
    G._assert_eq("access two-pass", got, pieces(t.access, pos), pos)
    idx = np.arange(0, q, 4099)
    G._assert_eq("access vs oracle", got[idx], oracle.access(S, pos[idx]), pos[idx])
    got = G.host(t.rank(G.dev(rc), G.dev(ri)))
    G._assert_eq("rank two-pass", got, pieces(t.rank, rc, ri), ri)
    G._assert_eq("rank vs oracle", got[idx], oracle.rank(S, sigma, rc[idx], ri[idx]), ri[idx])
    got = G.host(t.select(G.dev(sc), G.dev(sk)))
    G._assert_eq("select two-pass", got, pieces(t.select, sc, sk), sk)
    G._assert_eq("select vs oracle", got[idx], oracle.select(S, sigma, sc[idx], sk[idx]), sk[idx])
    t.learn_select()
    got = G.host(t.select_learned(G.dev(sc), G.dev(sk)))
    G._assert_eq("learned select two-pass", got, pieces(t.select, sc, sk), sk)
    t.free()


# (width, sigma, n, kind): trees whose level sequence narrows (u32 -> u16 -> u8, u16 -> u8) and whose
# later levels find nodes by position, including tiles with more nodes than the per-tile list holds
NARROW_CASES = [
    (4, 1 << 20, (1 << 21) + 333, "zipf12"),
    (4, 1 << 17, 1 << 20, "uniform"),
    (4, 70001, 500000, "zipf"),
    (4, 300, 100000, "uniform"),
    (2, 65536, (1 << 20) + 5, "uniform"),
    (2, 40000, 300000, "zipf"),
    (2, 1000, 1 << 20, "runs"),
    (2, 60001, 100000, "sparse"),
    (4, 1 << 20, 300000, "sparse"),
]


@pytest.mark.parametrize("width,sigma,n,kind", NARROW_CASES)
def test_narrow_codes_build_the_same_tree(width, sigma, n, kind):
    """The narrowing build (forced at these sizes: nodes by position after the prefix is dropped) equals
    the full-width build part by part, and both equal the oracle."""
    import paper_2505_03372_amd as wt
    G.log("narrow vs wide: width=%d sigma=%d n=%d %s" % (width, sigma, n, kind))
    S = make_seq(kind, n, sigma, width, 0x7A00 + sigma + n)
    tn = G.gpu_build(S, sigma, narrow=True)
    tw = G.gpu_build(S, sigma, wide=True)
    try:
        G.compare_structure(tn, oracle.OracleTree(S, sigma))
        for l in range(tn.info["levels"]):
            for part in (wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0):
                np.testing.assert_array_equal(tn.export(part, l), tw.export(part, l))
        G.compare_queries(tn, S, sigma, *G.random_queries(S, sigma, 4096, 0x7A01 + n))
    finally:
        tn.free()
        tw.free()

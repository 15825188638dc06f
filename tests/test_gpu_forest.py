"""GPU tests of the batched forest build and the mixed queries over a forest.

* every tree of a forest (edge shapes: empty, one symbol, sigma = 1 and 2, alphabets just below and
  above the histogram's LDS limit, sequences spanning two tile chunks; per-tree |L2| and s) has the
  oracle's bits, directory, samples, node tables and histogram, and answers like the oracle;
* a tree of a forest is identical (every exported part) to the tree wt_build makes alone;
* mixed queries equal the per-tree query calls (and the oracle), with the sentinels for unknown trees
  and ops;
* an out-of-range symbol in one sequence fails the whole build and names the sequence;
* the full batched configuration (1024 u16 sequences, 2^24 mixed queries): sampled trees equal single
  builds, sampled queries equal the oracle.
"""
import ctypes

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


# (n, sigma, kind, l2_bits, sample_rate); 0 = default
SHAPES = [
    (0, 5, "uniform", 0, 0),
    (1, 1, "equal", 0, 0),
    (1, 2, "uniform", 0, 0),
    (17, 3, "uniform", 256, 512),
    (1000, 4, "zipf", 0, 0),
    (8191, 7, "runs", 1024, 1024),
    (8192, 256, "uniform", 0, 0),
    (8193, 300, "zipf", 2048, 8192),
    (70000, 65536, "uniform", 0, 0),
    (300000, 2, "alternate", 256, 512),
    (196613, 1000, "zipf12", 0, 0),
    (123457, 16384, "zipf", 512, 4096),
    (123457, 16385, "uniform", 1024, 2048),
    (50000, 65535, "sparse", 0, 0),
    (2000000, 25, "zipf", 0, 0),
    (9000000, 40000, "zipf", 0, 0),  # more than 1024 tiles: two tile chunks per level
]
ORACLE_MAX_N = 10_000_000  # every shape, including the two-chunk tree


def _seqs():
    return [make_seq(kind, n, sigma, 2, 0xF0 + i) for i, (n, sigma, kind, _, _) in enumerate(SHAPES)]


@pytest.fixture(scope="module")
def small_forest():
    import paper_2505_03372_amd as wt
    seqs = _seqs()
    G.log("forest of %d edge shapes" % len(seqs))
    dev = [G.dev(S) for S in seqs]
    f = wt.build_forest(dev, [s[1] for s in SHAPES], l2_bits=[s[3] for s in SHAPES],
                        sample_rates=[s[4] for s in SHAPES])
    yield f, seqs
    f.free()


@pytest.mark.timeout(600)
def test_forest_trees_match_oracle(small_forest):
    f, seqs = small_forest
    assert len(f) == len(SHAPES)
    assert f.info["trees"] == len(SHAPES) and f.info["graph_kernels"] > 0
    for j, ((n, sigma, kind, l2, s), S) in enumerate(zip(SHAPES, seqs)):
        t = f[j]
        assert t.info["l2_bits"] == (l2 or 512) and t.info["sample_rate"] == (s or 4096)
        assert t.n == n and t.sigma == sigma
        G.log("  tree %d n=%d sigma=%d %s" % (j, n, sigma, kind))
        if n <= ORACLE_MAX_N:
            ot = oracle.OracleTree(S, sigma, l2_bits=l2 or 512, sample_rate=s or 4096)
            G.compare_structure(t, ot)
        pos, rc, ri, sc, sk = G.random_queries(S, sigma, 3000, 0xAB + j)
        G.compare_queries(t, S, sigma, pos, rc, ri, sc, sk)
        G.compare_queries(t, S, sigma, *G.edge_queries(S, sigma))


def test_forest_trees_equal_single_builds(small_forest):
    import paper_2505_03372_amd as wt
    f, seqs = small_forest
    parts = [wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START,
             wt.PART_NODE_R0]
    for j, ((n, sigma, kind, l2, s), S) in enumerate(zip(SHAPES, seqs)):
        t1 = G.gpu_build(S, sigma, l2_bits=l2 or 512, sample_rate=s or 4096)
        tf = f[j]
        assert tf.info["level_n"] == t1.info["level_n"] and tf.info["level_ones"] == t1.info["level_ones"]
        np.testing.assert_array_equal(tf.export(wt.PART_CUM_HIST), t1.export(wt.PART_CUM_HIST))
        for l in range(t1.info["levels"]):
            for part in parts:
                a, b = tf.export(part, l), t1.export(part, l)
                assert a.shape == b.shape and np.array_equal(a, b), (j, l, part)
        t1.free()


def _same_forests(fa, fb, count):
    import paper_2505_03372_amd as wt
    parts = [wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START,
             wt.PART_NODE_R0]
    for j in range(count):
        ta, tb = fa[j], fb[j]
        assert ta.info["level_n"] == tb.info["level_n"] and ta.info["level_ones"] == tb.info["level_ones"], j
        for l in range(ta.info["levels"]):
            for part in parts:
                a, b = ta.export(part, l), tb.export(part, l)
                assert a.shape == b.shape and np.array_equal(a, b), (j, l, part)


def test_forest_narrow_codes_equal_wide(small_forest):
    """The default forest carries codes that narrow level by level (nodes by position once prefix bits are
    dropped); the same forest with full-width codes is identical part by part."""
    import paper_2505_03372_amd as wt
    f, seqs = small_forest
    G.log("forest: full-width codes against the default")
    fw = wt.build_forest([G.dev(S) for S in seqs], [s[1] for s in SHAPES], l2_bits=[s[3] for s in SHAPES],
                         sample_rates=[s[4] for s in SHAPES], wide=True)
    try:
        assert fw.info["graph_kernels"] < f.info["graph_kernels"]  # one level launch per level when wide
        _same_forests(f, fw, len(SHAPES))
    finally:
        fw.free()


# u32 sequences: codes narrow from 4 to 2 to 1 byte (alphabets up to 2^20, 20 levels)
SHAPES32 = [
    (300001, 1 << 20, "zipf12"),
    (100000, 70000, "uniform"),
    (65537, 1000003, "sparse"),
    (200000, 300, "zipf"),
    (9000, 1 << 17, "uniform"),
    (50000, 2, "alternate"),
    (1, 5, "uniform"),
    (0, 9, "uniform"),
]


def test_forest_u32_narrow_codes():
    import paper_2505_03372_amd as wt
    seqs = [make_seq(kind, n, sigma, 4, 0x3A0 + i) for i, (n, sigma, kind) in enumerate(SHAPES32)]
    sig = [s[1] for s in SHAPES32]
    G.log("u32 forest of %d shapes, narrow and wide codes" % len(seqs))
    dev = [G.dev(S) for S in seqs]
    fn = wt.build_forest(dev, sig)
    fw = wt.build_forest(dev, sig, wide=True)
    try:
        _same_forests(fn, fw, len(seqs))
        for j, (S, sigma) in enumerate(zip(seqs, sig)):
            if S.size == 0:
                continue
            G.compare_structure(fn[j], oracle.OracleTree(S, sigma))
            G.compare_queries(fn[j], S, sigma, *G.random_queries(S, sigma, 2048, 0x3B0 + j))
    finally:
        fn.free()
        fw.free()


def _mixed_reference(f, seqs, tree, op, sym, arg):
    """Per-tree query calls for every query (grouped by tree and op)."""
    out = np.full(tree.size, np.iinfo(np.uint64).max, dtype=np.uint64)
    for j in range(len(f)):
        for o in range(3):
            idx = np.nonzero((tree == j) & ((op == o) | ((op == 3) & (o == 2))))[0]
            if idx.size == 0:
                continue
            t = f[j]
            if o == 0:
                r = G.host(t.access(G.dev(arg[idx]))).astype(np.uint64)
            elif o == 1:
                r = G.host(t.rank(G.dev(sym[idx]), G.dev(arg[idx])))
            else:
                r = G.host(t.select(G.dev(sym[idx]), G.dev(arg[idx])))
            out[idx] = r
    return out


@pytest.mark.parametrize("q", [3001, 30001, 200003])  # one kernel up to 16384, class-sorted below 2^16, sorted by (class, position) above
def test_mixed_queries_match_per_tree_calls(small_forest, q):
    f, seqs = small_forest
    T = len(seqs)
    r = workloads.raw(0x3151, 0, 4 * q)
    tree = (r[:q] % np.uint64(T + 2)).astype(np.uint32)  # two unknown tree ids
    op = (r[q:2 * q] % np.uint64(5)).astype(np.uint8)     # op 3: learned select (plain here), op 4 unknown
    op[:6] = [0, 1, 2, 3, 255, 7]
    sym = np.zeros(q, dtype=np.uint32)
    arg = np.zeros(q, dtype=np.uint64)
    for j in range(T):
        idx = np.nonzero(tree == j)[0]
        S = seqs[j]
        n, sigma = S.size, SHAPES[j][1]
        a = r[2 * q + idx]
        b = r[3 * q + idx]
        arg[idx] = a % np.uint64(n + 2)                  # some positions past the end
        sym[idx] = (b % np.uint64(sigma + 1)).astype(np.uint32)  # some symbols past the alphabet
        is_sel = (op[idx] == 2) | (op[idx] == 3)
        selj = idx[is_sel]
        if n:
            cnt = np.bincount(S, minlength=sigma + 1).astype(np.uint64)
            arg[selj] = a[is_sel] % (cnt[sym[selj]] + np.uint64(2))  # k = 0 and k > count included
    G.log("mixed queries q=%d over %d trees" % (q, T))
    got = G.host(f.query_mixed(G.dev(tree), G.dev(op), G.dev(sym), G.dev(arg)))
    exp = _mixed_reference(f, seqs, tree, op, sym, arg)
    bad = (tree >= T) | (op > 3)
    assert np.all(got[bad] == np.iinfo(np.uint64).max)
    G._assert_eq("mixed vs per-tree", got, exp, np.stack([tree.astype(np.uint64), op.astype(np.uint64), arg], 1))
    # and the oracle on a sample
    idx = np.arange(0, q, 97)
    for j in range(T):
        sub = idx[(tree[idx] == j)]
        S = seqs[j]
        for o, fn in ((0, None), (1, oracle.rank), (2, oracle.select)):
            s2 = sub[(op[sub] == o) | ((op[sub] == 3) & (o == 2))]
            if s2.size == 0:
                continue
            if o == 0:
                e = oracle.access(S, arg[s2]).astype(np.uint64)
            else:
                e = fn(S, SHAPES[j][1], sym[s2], arg[s2])
            G._assert_eq("mixed vs oracle tree %d op %d" % (j, o), got[s2], e, arg[s2])


def test_forest_symbol_range_error():
    import paper_2505_03372_amd as wt
    seqs = [make_seq("uniform", 5000, 10, 2, 1), make_seq("uniform", 7000, 20, 2, 2), make_seq("uniform", 3000, 30, 2, 3)]
    seqs[2][1234] = 30
    with pytest.raises(wt.WTError) as ei:
        wt.build_forest([G.dev(S) for S in seqs], [10, 20, 30])
    assert ei.value.status == wt.WT_ERR_SYMBOL_RANGE and "sequence 2" in str(ei.value)


def test_forest_tree_is_borrowed(small_forest):
    import paper_2505_03372_amd as wt
    f, _ = small_forest
    assert wt.lib().wt_free(f[3].handle) == wt.WT_ERR_STATE


def test_forest_full_size_batched_config():
    """1024 u16 sequences (n log-uniform in [2^10, 2^24], sigma log-uniform in [4, 2^16], Zipf 1.0) and
    2^24 mixed queries (tree and op uniform)."""
    import torch
    import paper_2505_03372_amd as wt
    G.log("batched config: generating")
    fw = workloads.make_forest()
    G.log("batched config: %d symbols, upload" % fw.S.size)
    dS = G.dev(fw.S)
    views = [dS[int(fw.offsets[j]):int(fw.offsets[j + 1])] for j in range(fw.trees)]
    G.log("batched config: build")
    f = wt.build_forest(views, [int(s) for s in fw.sigmas])
    G.log("  %s" % f.info)
    assert f.info["symbols"] == fw.S.size
    # sampled trees equal single builds: the largest, the one with most levels, and a spread
    ns = np.diff(fw.offsets)
    pick = sorted({int(np.argmax(ns)), int(np.argmax(fw.sigmas)), *range(0, fw.trees, 128)})
    for j in pick:
        S = fw.seq(j)
        t1 = G.gpu_build(S, int(fw.sigmas[j]))
        tf = f[j]
        assert tf.info["level_n"] == t1.info["level_n"] and tf.info["level_ones"] == t1.info["level_ones"], j
        for l in range(t1.info["levels"]):
            for part in (wt.PART_BITS, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_R0):
                assert np.array_equal(tf.export(part, l), t1.export(part, l)), (j, l, part)
        t1.free()
    G.log("batched config: 2^24 mixed queries")
    got = G.host(f.query_mixed(G.dev(fw.tree), G.dev(fw.op), G.dev(fw.sym), G.dev(fw.arg)))
    idx = np.arange(0, got.size, 256)
    for j in range(fw.trees):
        sub = idx[fw.tree[idx] == j]
        if sub.size == 0:
            continue
        S, sigma = fw.seq(j), int(fw.sigmas[j])
        for o in range(3):
            s2 = sub[fw.op[sub] == o]
            if s2.size == 0:
                continue
            if o == 0:
                e = oracle.access(S, fw.arg[s2]).astype(np.uint64)
            elif o == 1:
                e = oracle.rank(S, sigma, fw.sym[s2], fw.arg[s2])
            else:
                e = oracle.select(S, sigma, fw.sym[s2], fw.arg[s2])
            G._assert_eq("batched mixed tree %d op %d" % (j, o), got[s2], e, fw.arg[s2])
    f.free()
    del dS
    torch.cuda.empty_cache()


def test_autotune_and_tuned_forest(tmp_path):
    import paper_2505_03372_amd as wt
    shapes = [(5000, 10), (300000, 100), (300000, 5000), (2_000_000, 60000), (40000, 3), (0, 7)]
    seqs = [make_seq("zipf", n, sg, 2, 0x70 + i) for i, (n, sg) in enumerate(shapes)]
    sigmas = [sg for _, sg in shapes]
    dev = [G.dev(S) for S in seqs]
    G.log("autotune over %d sequences" % len(seqs))
    tt, rep = wt.autotune(dev, sigmas, max_probe_n=1 << 20, queries=1 << 14)
    G.log("  %s" % rep)
    buckets = {wt.tune_bucket(n, sg) for n, sg in shapes if n > 0}
    assert set(rep["choice"]) == buckets and rep["buckets"] == len(buckets)
    for l2, s in rep["choice"].values():
        assert l2 in (256, 512, 1024) and s in (1024, 4096, 16384)
        assert 16 / l2 + 64 / s + 64 / 65536 <= 0.10
    path = str(tmp_path / "tune.json")
    wt.save_tune(tt, path)
    tt2 = wt.load_tune(path)
    assert bytes(tt2) == bytes(tt)
    f = wt.build_forest(dev, sigmas, tune=tt2)
    for j, ((n, sg), S) in enumerate(zip(shapes, seqs)):
        t = f[j]
        l2, s = rep["choice"].get(wt.tune_bucket(n, sg), (512, 4096))
        assert (t.info["l2_bits"], t.info["sample_rate"]) == (l2, s), j
        G.compare_structure(t, oracle.OracleTree(S, sg, l2_bits=l2, sample_rate=s))
        G.compare_queries(t, S, sg, *G.random_queries(S, sg, 3000, 0xCD + j))
    f.free()

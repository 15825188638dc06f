"""Pins of the CPU oracle against facts the thesis and the mathematics fix (no GPU).

Each test names what it pins:
* the thesis's worked example (golden fixture, printed values);
* brute force on tiny inputs, exhaustively over positions, symbols and k;
* invariants of rank/select that hold at any size;
* the code table's shape (prefix-free, order-preserving, two children everywhere,
  non-increasing lengths, natural binary for powers of two);
* level bits reproduced by the thesis's query walks with naive counting;
* the directory against naive counts and the printed overhead percentages;
* node-start ranks against the histogram formula (an independent route).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import walker

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _example():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        g = json.load(f)
    sym = {ch: i for i, ch in enumerate(g["alphabet"])}
    S = np.array([sym[ch] for ch in g["text"]], dtype=np.uint8)
    return g, sym, S


def test_worked_example_answers():
    g, sym, S = _example()
    sigma = len(g["alphabet"])
    acc = oracle.access(S, np.array([g["access"]["i"]], np.uint64))
    assert acc[0] == sym[g["access"]["result"]]
    rk = oracle.rank(S, sigma, np.array([sym[g["rank"]["symbol"]]], np.uint32), np.array([g["rank"]["i"]], np.uint64))
    assert rk[0] == g["rank"]["result"]
    # the select position is the 4th one of level 0 (checked through the tree below); here the
    # answer must be the position of the 2nd c by definition
    sl = oracle.select(S, sigma, np.array([sym[g["select"]["symbol"]]], np.uint32),
                       np.array([g["select"]["k"]], np.uint64))
    assert sl[0] == oracle.brute_select(list(S), sigma, sym["c"], 2)


def test_worked_example_intermediates():
    g, sym, S = _example()
    t = oracle.OracleTree(S, len(g["alphabet"]))
    a = g["access"]
    res, trace = walker.walk_access(t, a["i"])
    assert res == sym[a["result"]]
    assert trace[0][0] == "step" and trace[0][2] == a["level0_bit"] and trace[0][3] == a["position_in_right_child"]
    assert trace[1][0] == "leaf" and trace[1][2] == a["level1_bit"]
    r = g["rank"]
    res, trace = walker.walk_rank(t, sym[r["symbol"]], r["i"])
    assert res == r["result"]
    assert trace[0][1] == r["bits_considered_at_level1"]
    s = g["select"]
    res, trace = walker.walk_select(t, sym[s["symbol"]], s["k"])
    # deepest level first: select0 with argument 2 lands at node position 3, then the 4th one of level 0
    assert trace[0][0] == 1 and trace[0][1] == 0 and trace[0][2] == s["level1_select0_arg"]
    assert trace[0][3] == s["position_in_level1_node"]
    assert trace[1][0] == 0 and trace[1][1] == 1 and trace[1][2] == s["level0_select1_arg"]
    assert res == oracle.brute_select(list(S), 4, sym["c"], 2)


TINY_SIGMAS = [1, 2, 3, 4, 5, 6, 7, 8, 11, 13, 16, 255, 256]


def _tiny_seq(n, sigma, seed, kind="uniform"):
    if kind == "uniform":
        return workloads.uniform(seed, n, sigma, 1 if sigma <= 256 else 2)
    if kind == "equal":
        return np.full(n, sigma - 1, dtype=np.uint8 if sigma <= 256 else np.uint16)
    if kind == "alternate":
        return (np.arange(n) % min(sigma, 2) * (sigma - 1)).astype(np.uint8 if sigma <= 256 else np.uint16)
    raise ValueError(kind)


@pytest.mark.parametrize("sigma", TINY_SIGMAS)
@pytest.mark.parametrize("kind", ["uniform", "equal", "alternate"])
def test_answers_match_brute_force_exhaustively(sigma, kind):
    for n in (0, 1, 2, 7, 40):
        S = _tiny_seq(n, sigma, 1000 + n + sigma, kind)
        Sl = [int(x) for x in S]
        pos = np.arange(0, n + 2, dtype=np.uint64)
        acc = oracle.access(S, pos)
        assert [int(x) for x in acc] == [oracle.brute_access(Sl, int(i)) for i in pos]
        cs = [c for c in range(min(sigma + 1, 20))] + [sigma + 3]
        cc, ii = np.meshgrid(np.array(cs, np.uint32), np.arange(0, n + 2, dtype=np.uint64))
        rk = oracle.rank(S, sigma, cc.ravel(), ii.ravel())
        exp = [oracle.brute_rank(Sl, sigma, int(c), int(i)) for c, i in zip(cc.ravel(), ii.ravel())]
        assert [int(x) for x in rk] == exp
        cc, kk = np.meshgrid(np.array(cs, np.uint32), np.arange(0, n + 2, dtype=np.uint64))
        sl = oracle.select(S, sigma, cc.ravel(), kk.ravel())
        exp = [oracle.brute_select(Sl, sigma, int(c), int(k)) for c, k in zip(cc.ravel(), kk.ravel())]
        assert [int(x) for x in sl] == exp


def test_answers_match_brute_force_random_medium():
    S, sigma = workloads.make_text("plain_small", n=3000)
    Sl = [int(x) for x in S]
    q = workloads.make_queries("plain_small", S, sigma, q=300)
    acc = oracle.access(S, q["acc_pos"])
    assert all(int(a) == oracle.brute_access(Sl, int(i)) for a, i in zip(acc, q["acc_pos"]))
    rk = oracle.rank(S, sigma, q["rank_c"], q["rank_i"])
    assert all(int(r) == oracle.brute_rank(Sl, sigma, int(c), int(i))
               for r, c, i in zip(rk, q["rank_c"], q["rank_i"]))
    sl = oracle.select(S, sigma, q["sel_c"], q["sel_k"])
    assert all(int(s) == oracle.brute_select(Sl, sigma, int(c), int(k))
               for s, c, k in zip(sl, q["sel_c"], q["sel_k"]))


def test_rank_select_invariants():
    S, sigma = workloads.make_text("text_zipf", n=50000)
    n = S.size
    cnt = np.bincount(S, minlength=sigma)
    pos = np.arange(0, n, 37, dtype=np.uint64)
    for c in [int(S[0]), int(S[1]), int(np.argmax(cnt)), int(np.argmin(cnt))]:
        cs = np.full(pos.size, c, np.uint32)
        # rank(c, n) = count(c)
        assert oracle.rank(S, sigma, np.array([c], np.uint32), np.array([n], np.uint64))[0] == cnt[c]
        # with r = rank(c, i+1): select(c, r) <= i < select(c, r+1) (select(c,0) := -1, select(c,count+1) := n)
        r = oracle.rank(S, sigma, cs, pos + 1).astype(np.int64)
        lo = oracle.select(S, sigma, cs, r.astype(np.uint64)).astype(np.int64)
        lo[r == 0] = -1
        hi = oracle.select(S, sigma, cs, (r + 1).astype(np.uint64)).astype(np.int64)
        assert np.all(lo <= pos.astype(np.int64)) and np.all(pos.astype(np.int64) < hi)
        # rank(c, select(c,k)) = k-1, access(select(c,k)) = c
        ks = np.arange(1, cnt[c] + 1, max(1, cnt[c] // 50), dtype=np.uint64)
        sp = oracle.select(S, sigma, np.full(ks.size, c, np.uint32), ks)
        assert np.all(oracle.rank(S, sigma, np.full(ks.size, c, np.uint32), sp) == ks - 1)
        assert np.all(oracle.access(S, sp) == c)
    # sum over symbols of rank(c, i) = i
    for i in [0, 1, 999, n // 2, n]:
        cs = np.arange(sigma, dtype=np.uint32)
        assert int(oracle.rank(S, sigma, cs, np.full(sigma, i, np.uint64)).sum()) == i


def _code_bits(code, ln, L):
    return format(int(code), "0%db" % L)[: int(ln)] if L else ""


@pytest.mark.parametrize("sigma", list(range(1, 300)) + [1000, 1023, 1025, 4096, 5000, 65535, 65536, 70001])
def test_code_table_shape(sigma):
    code, ln = oracle.codes(sigma)
    L = oracle.num_levels(sigma)
    assert (1 << L) >= sigma and (L == 0 or (1 << (L - 1)) < sigma)
    words = [_code_bits(code[c], ln[c], L) for c in range(sigma)]
    # order-preserving (lexicographic on the bit strings) and non-increasing lengths
    assert all(words[i] < words[i + 1] for i in range(sigma - 1))
    assert all(ln[i] >= ln[i + 1] for i in range(sigma - 1))
    # complete prefix code: every internal node has two children (Kraft sum exactly 1)
    if sigma > 1:
        from fractions import Fraction
        assert sum(Fraction(1, 1 << int(x)) for x in ln) == 1
        assert max(ln) == L
    # the split of each node is the largest power of two strictly below its width
    if sigma <= 300:
        def check(prefix, s, e):
            if e - s == 1:
                return
            p = walker.pow2_below(e - s)
            left = [c for c in range(s, e) if words[c].startswith(prefix + "0")]
            right = [c for c in range(s, e) if words[c].startswith(prefix + "1")]
            assert left == list(range(s, s + p)) and right == list(range(s + p, e))
            check(prefix + "0", s, s + p)
            check(prefix + "1", s + p, e)
        check("", 0, sigma)
    # powers of two: natural binary codes of full length
    if sigma & (sigma - 1) == 0:
        assert all(int(code[c]) == c for c in range(sigma)) and all(int(x) == L for x in ln)
    # symbols at or above the previous power of two are the only ones that may be shorter
    if sigma > 1 and sigma & (sigma - 1):
        P = 1 << (L - 1)
        assert all(int(ln[c]) == L for c in range(P))


@pytest.mark.parametrize("sigma,kind,n", [(4, "uniform", 500), (5, "uniform", 700), (6, "alternate", 300),
                                          (7, "uniform", 1000), (13, "uniform", 800), (2, "equal", 65),
                                          (256, "uniform", 3000), (11, "equal", 100), (1, "equal", 10)])
def test_levels_reproduce_sequence_through_query_walks(sigma, kind, n):
    S = _tiny_seq(n, sigma, 77 + sigma, kind)
    t = oracle.OracleTree(S, sigma)
    Sl = [int(x) for x in S]
    code, ln = oracle.codes(sigma)
    hist = np.bincount(S, minlength=sigma)
    for l in range(t.L):
        # level size: symbols whose code is longer than l; ones: those with bit l set
        exp_n = sum(int(hist[c]) for c in range(sigma) if ln[c] > l)
        exp_ones = sum(int(hist[c]) for c in range(sigma) if ln[c] > l and (int(code[c]) >> (t.L - 1 - l)) & 1)
        assert t.level_n[l] == exp_n and t.ones[l] == exp_ones
    for i in range(0, n, max(1, n // 60)):
        assert walker.walk_access(t, i)[0] == Sl[i]
    for c in range(min(sigma, 9)):
        for i in range(0, n + 1, max(1, n // 25)):
            assert walker.walk_rank(t, c, i)[0] == oracle.brute_rank(Sl, sigma, c, i)
        for k in range(1, int(hist[c]) + 1, max(1, int(hist[c]) // 10)):
            assert walker.walk_select(t, c, k)[0] == oracle.brute_select(Sl, sigma, c, k)


@pytest.mark.parametrize("l2", [256, 512, 1024])
@pytest.mark.parametrize("n", [1, 511, 512, 513, 65536, 65537, 200000])
def test_directory_against_naive_counts(l2, n):
    # a single level (sigma = 2) whose bits are the symbols themselves
    S = workloads.uniform(5000 + n, n, 2, 1)
    t = oracle.OracleTree(S, 2, l2_bits=l2, sample_rate=512)
    assert t.bit_string(0) == "".join(str(int(x)) for x in S)
    row = S.astype(np.int64)
    ones_before = np.concatenate([[0], np.cumsum(row)])
    L1, L2 = t.L1[0], t.L2[0]
    assert L1.size == (n + 65535) // 65536 + 1 and L2.size == (n + l2 - 1) // l2 + 1
    # the thesis's binary rank: L1 of the block + L2 of the sub-block + popcount of the rest
    xs = np.unique(np.concatenate([np.arange(0, n + 1, 97), [0, n], np.arange(0, n + 1, l2)]))
    for x in xs:
        x = int(x)
        b, j = x // 65536, x // l2
        r = int(L1[b]) + int(L2[j]) + int(row[j * l2: x].sum())
        assert r == ones_before[x]
    # L2 restarts at every L1 boundary; last L1 entry is the total
    assert all(int(L2[j]) == 0 for j in range(L2.size) if (j * l2) % 65536 == 0)
    assert int(L1[-1]) == int(row.sum())
    # samples: position of every (k s)-th one / zero
    s = 512
    for k, p in enumerate(t.samples1[0], start=1):
        assert row[p] == 1 and ones_before[p] == k * s - 1
    zeros_before = np.arange(n + 1) - ones_before
    for k, p in enumerate(t.samples0[0], start=1):
        assert row[p] == 0 and zeros_before[p] == k * s - 1
    assert len(t.samples1[0]) == int(row.sum()) // s and len(t.samples0[0]) == (n - int(row.sum())) // s


def test_directory_overhead_matches_printed_percentages():
    with open(os.path.join(GOLDEN, "overhead.json")) as f:
        g = json.load(f)
    n = 1 << 22
    S = workloads.uniform(4242, n, 2, 1)
    for case in g["cases"]:
        s = case["sample_rate"] or 4096
        t = oracle.OracleTree(S, 2, l2_bits=case["l2_bits"], sample_rate=s)
        bits = (t.L1[0].size - 1) * 64 + (t.L2[0].size - 1) * 16  # without the sentinels
        if case["sample_rate"]:
            bits += (n // s) * 64  # the thesis's upper bound on samples of ones and zeros together
            assert len(t.samples1[0]) + len(t.samples0[0]) <= n // s
        pct = 100.0 * bits / n
        assert round(pct, case["printed_digits"]) == case["percent"]


@pytest.mark.parametrize("sigma,n", [(4, 2000), (6, 3000), (7, 999), (13, 4000), (100, 5000), (256, 6000), (300, 7000)])
def test_node_ranks_match_histogram_formula(sigma, n):
    S = workloads.zipf(99 + sigma, n, sigma, 1.0, 2, workloads.permutation(7, sigma))
    t = oracle.OracleTree(S, sigma)
    code, ln = oracle.codes(sigma)
    hist = np.bincount(S, minlength=sigma)
    L = t.L
    for l in range(L):
        for p in range(1 << l):
            syms = [c for c in range(sigma) if ln[c] > l and (int(code[c]) >> (L - l) if l else 0) == p]
            if not syms:
                assert t.node_start[l][p] == oracle.U64_MAX
                continue
            s0 = syms[0]
            # start = occurrences of all smaller symbols (they all reach level l)
            assert int(t.node_start[l][p]) == int(t.cum_hist[s0])
            # rank0 at the start = occurrences of smaller symbols that reach level l with bit 0
            exp = sum(int(hist[c]) for c in range(s0)
                      if ln[c] > l and ((int(code[c]) >> (L - 1 - l)) & 1) == 0)
            assert int(t.node_r0[l][p]) == exp


def test_mlp_reference_gradients_match_finite_differences():
    rng = workloads.raw(0xABC, 0, 2000).astype(np.float64) / 2.0**64
    u = rng[:500]
    v = np.sqrt(u) + 0.01 * (rng[500:1000] - 0.5)  # a monotone target with noise
    th = oracle.mlp_init() + 0.1 * (rng[1000:1049] - 0.5)
    loss, g = oracle.mlp_loss_grad(th, u, v)
    # the loss is the mean squared error of the forward pass
    assert abs(loss - np.mean((oracle.mlp_forward(th, u) - v) ** 2)) < 1e-12
    h = 1e-6
    for j in range(oracle.MLP_PARAMS):
        tp = th.copy(); tp[j] += h
        tm = th.copy(); tm[j] -= h
        fd = (oracle.mlp_loss_grad(tp, u, v)[0] - oracle.mlp_loss_grad(tm, u, v)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_mlp_init_is_identity_on_unit_interval():
    u = np.linspace(0, 1, 101)
    assert np.allclose(oracle.mlp_forward(oracle.mlp_init(), u), u, atol=1e-15)


def _mlp_clamp_theta():
    """A network whose units are negative on part of [0, 1] (and two of them everywhere):
    unit 0: h = 2u - 0.5 (on for u > 1/4), weight 3; unit 1: h = 0.25 - u (on for u < 1/4), weight -2;
    units 2..15: h = -1 (never on), weight 1; output bias 0.1."""
    th = np.zeros(oracle.MLP_PARAMS)
    th[0], th[16], th[32] = 2.0, -0.5, 3.0
    th[1], th[17], th[33] = -1.0, 0.25, -2.0
    for k in range(2, 16):
        th[k], th[16 + k], th[32 + k] = 0.0, -1.0, 1.0
    th[48] = 0.1
    return th


def test_mlp_forward_hand_values_where_relu_clamps():
    # y(u) = 0.1 + 3 max(2u - 0.5, 0) - 2 max(0.25 - u, 0) + 14 max(-1, 0), worked by hand:
    #   u = 0:    0.1 + 0   - 0.5 = -0.4      u = 0.1: 0.1 + 0 - 0.3 = -0.2
    #   u = 0.25: 0.1 + 0   - 0   =  0.1      u = 0.5: 0.1 + 1.5 - 0 = 1.6
    #   u = 1:    0.1 + 4.5 - 0   =  4.6
    # Dropping the clamp would add 14 * (-1) plus the negative parts of units 0 and 1.
    th = _mlp_clamp_theta()
    u = np.array([0.0, 0.1, 0.25, 0.5, 1.0])
    exp = np.array([-0.4, -0.2, 0.1, 1.6, 4.6])
    np.testing.assert_allclose(oracle.mlp_forward(th, u), exp, rtol=0, atol=1e-12)


def test_mlp_gradient_hand_values_where_relu_clamps():
    # One point (u, v) = (0.5, 1.0): y = 1.6, r = 0.6, loss = 0.36, dL/dy = 2 r = 1.2.
    # Unit 0 is on (h0 = 0.5): dL/dw2_0 = 1.2 * 0.5 = 0.6, dL/db1_0 = 1.2 * 3 = 3.6, dL/dw1_0 = 3.6 * 0.5 = 1.8.
    # Unit 1 (h1 = -0.25) and units 2..15 (h = -1) are off: every derivative of theirs is 0.
    # dL/db2 = 1.2.
    th = _mlp_clamp_theta()
    loss, g = oracle.mlp_loss_grad(th, np.array([0.5]), np.array([1.0]))
    assert abs(loss - 0.36) < 1e-12
    exp = np.zeros(oracle.MLP_PARAMS)
    exp[32], exp[16], exp[0], exp[48] = 0.6, 3.6, 1.8, 1.2
    np.testing.assert_allclose(g, exp, rtol=0, atol=1e-12)


def test_alphabet_hand_example_and_library_routine():
    # hand example: the distinct values of (7, 3, 7, 100, 3, 0) in increasing order are (0, 3, 7, 100)
    S = np.array([7, 3, 7, 100, 3, 0], dtype=np.uint32)
    assert oracle.alphabet(S).tolist() == [0, 3, 7, 100]
    assert oracle.alphabet(np.zeros(0, np.uint8)).size == 0
    assert oracle.alphabet(np.full(9, 200, np.uint8)).tolist() == [200]
    # against numpy's unique on random inputs of every width
    for w, hi in ((1, 256), (2, 60000), (4, 1 << 31)):
        S = (workloads.raw(0xA1 + w, 0, 20000) % np.uint64(hi)).astype(workloads.dtype_for(w))
        np.testing.assert_array_equal(oracle.alphabet(S), np.unique(S).astype(np.uint64))

"""Pins of the oracle's Huffman-shaped tree (wt_oracle.c: oracle_huffman_lengths, oracle_huffman_codes,
oracle_level_bits_codes, oracle_nodes_codes), against facts that do not come from the oracle itself:

* code lengths: a textbook example with a unique optimum, exhaustive search over every length vector
  on tiny alphabets (with and without a binding length limit), the cost of the classical two-smallest
  merging (heapq) when the limit does not bind, Kraft's equality, and the tie rule on equal counts;
* canonical codes: prefix-free, lengths non-increasing and values increasing in rank order, every
  depth's internal prefixes on the left, code values multiples of their leaf width;
* levels: total bits = sum of count x length, node starts = counts of the symbols ordered before the
  node, and top-down / bottom-up walks over the levels with naive bit counting that reproduce access,
  rank and select of the raw sequence.
"""
import heapq
import itertools

import numpy as np
import pytest

import oracle
import workloads


def _cost(h, ln):
    return int(sum(int(a) * int(b) for a, b in zip(h, ln)))


def _kraft_full(ln):
    ln = [int(x) for x in ln if x > 0]
    L = max(ln)
    return sum(1 << (L - x) for x in ln) == (1 << L)


def test_textbook_examples():
    # counts 45, 13, 12, 16, 9, 5: the classical example whose optimal code costs 224 bits with
    # lengths 1, 3, 3, 3, 4, 4 (the two rarest symbols share the deepest level)
    h = np.array([45, 13, 12, 16, 9, 5], dtype=np.uint64)
    ln = oracle.huffman_lengths(h)
    assert list(ln) == [1, 3, 3, 3, 4, 4]
    assert _cost(h, ln) == 224
    # powers of two: the unique optimum is a spine (1, 2, 3, 4, 4)
    h = np.array([8, 4, 2, 1, 1], dtype=np.uint64)
    assert list(oracle.huffman_lengths(h)) == [1, 2, 3, 4, 4]


def test_tie_rule_on_equal_counts():
    # equal counts: symbols are taken in (count, symbol) order, so the later symbol gets the shorter code
    assert list(oracle.huffman_lengths(np.array([3, 3, 3], dtype=np.uint64))) == [2, 2, 1]
    assert list(oracle.huffman_lengths(np.array([5, 5, 5, 5], dtype=np.uint64))) == [2, 2, 2, 2]
    assert list(oracle.huffman_lengths(np.array([2, 2, 2, 2, 2], dtype=np.uint64))) == [3, 3, 2, 2, 2]


def test_degenerate_alphabets():
    assert list(oracle.huffman_lengths(np.array([0, 0, 0], dtype=np.uint64))) == [0, 0, 0]
    assert list(oracle.huffman_lengths(np.array([0, 9, 0], dtype=np.uint64))) == [0, 0, 0]
    assert list(oracle.huffman_lengths(np.array([0, 9, 0, 1], dtype=np.uint64))) == [0, 1, 0, 1]
    with pytest.raises(ValueError):
        oracle.huffman_lengths(np.ones(5, dtype=np.uint64), 2)


def _brute_min_cost(h, limit):
    best = None
    for ln in itertools.product(range(1, limit + 1), repeat=len(h)):
        if sum(2.0 ** -x for x in ln) <= 1.0 + 1e-12:
            c = _cost(h, ln)
            best = c if best is None or c < best else best
    return best


@pytest.mark.parametrize("seed", range(12))
def test_lengths_optimal_by_exhaustive_search(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 7))
    h = rng.integers(1, 50, size=m).astype(np.uint64)
    if seed % 3 == 0:
        h = np.array([1, 1, 2, 3, 5, 8][:m], dtype=np.uint64)  # skewed: the limit binds
    for limit in range(max(1, (m - 1).bit_length()), 6):
        ln = oracle.huffman_lengths(h, limit)
        assert int(ln.max()) <= limit
        assert _kraft_full(ln)
        assert _cost(h, ln) == _brute_min_cost(h, limit), (h, limit, ln)


def _heap_huffman_cost(h):
    """Classical Huffman: merge the two lightest weights until one is left; the cost is the sum of
    the merged weights."""
    q = [int(x) for x in h if x > 0]
    heapq.heapify(q)
    cost = 0
    while len(q) > 1:
        a = heapq.heappop(q)
        b = heapq.heappop(q)
        cost += a + b
        heapq.heappush(q, a + b)
    return cost


@pytest.mark.parametrize("seed,m", [(1, 2), (2, 17), (3, 256), (4, 300), (5, 1000)])
def test_lengths_match_classical_huffman_cost(seed, m):
    rng = np.random.default_rng(100 + seed)
    h = (rng.zipf(1.3, size=m) % 100000).astype(np.uint64) + 1
    ln = oracle.huffman_lengths(h, 24)
    assert _kraft_full(ln)
    assert _cost(h, ln) == _heap_huffman_cost(h)


def test_zero_counts_get_no_code():
    h = np.array([0, 4, 0, 0, 7, 1, 0, 2], dtype=np.uint64)
    ln = oracle.huffman_lengths(h)
    assert all(ln[h == 0] == 0) and all(ln[h > 0] > 0)
    assert _cost(h, ln) == _heap_huffman_cost(h)


@pytest.mark.parametrize("seed", range(6))
def test_canonical_codes(seed):
    rng = np.random.default_rng(200 + seed)
    sigma = int(rng.integers(2, 300))
    h = (rng.zipf(1.2, size=sigma) % 5000).astype(np.uint64)
    h[rng.random(sigma) < 0.2] = 0
    h[:2] += 1
    ln = oracle.huffman_lengths(h)
    code, rk, L = oracle.huffman_codes(ln)
    assert L == int(ln.max())
    present = [c for c in range(sigma) if ln[c] > 0]
    assert sorted(int(rk[c]) for c in present) == list(range(len(present)))
    assert all(rk[c] == 0xFFFFFFFF for c in range(sigma) if ln[c] == 0)
    by_rank = sorted(present, key=lambda c: int(rk[c]))
    # lengths non-increasing, symbols increasing among equal lengths, values increasing in rank order
    for a, b in zip(by_rank, by_rank[1:]):
        assert ln[a] > ln[b] or (ln[a] == ln[b] and a < b)
        assert code[a] < code[b]
    words = {}
    for c in present:
        w = int(ln[c])
        v = int(code[c])
        assert v % (1 << (L - w)) == 0  # a multiple of its leaf width
        words[c] = format(v >> (L - w), "0%db" % w)
    # prefix-free
    ws = sorted(words.values())
    for a, b in zip(ws, ws[1:]):
        assert not b.startswith(a)
    # at every depth d the prefixes of longer codes (internal nodes) come before the codes of length d
    for d in range(1, L + 1):
        internal = {int(code[c]) >> (L - d) for c in present if ln[c] > d}
        leaves = {int(code[c]) >> (L - d) for c in present if ln[c] == d}
        if internal:
            assert internal == set(range(len(internal)))
            assert not leaves or min(leaves) >= len(internal)


def _walk_tables(t):
    by_rank = sorted((c for c in range(t.sigma) if t.lens[c] > 0), key=lambda c: int(t.rank[c]))
    cumr = [0]
    for c in by_rank:
        cumr.append(cumr[-1] + int(t.hist[c]))
    return by_rank, cumr


def _node_range(t, by_rank, l, p):
    """Ranks [s, e) whose code has prefix p at level l (contiguous in rank order)."""
    rs = [r for r, c in enumerate(by_rank) if (int(t.codes[c]) >> (t.L - l) if l else 0) == p]
    return (rs[0], rs[-1] + 1) if rs else (0, 0)


def _naive_rank(t, l, b, x):
    return sum(1 for j in range(x) if t.bit(l, j) == b)


def walk_access(t, by_rank, cumr, i):
    if t.L == 0:
        return int(np.nonzero(t.hist)[0][0])  # the one occurring symbol
    p, x = 0, i
    for l in range(t.L):
        s, e = _node_range(t, by_rank, l, p)
        base = cumr[s]
        b = t.bit(l, base + x)
        x = _naive_rank(t, l, b, base + x) - _naive_rank(t, l, b, base)
        p = 2 * p + b
        cs, ce = _node_range(t, by_rank, l + 1, p)
        c = by_rank[cs]
        if ce - cs == 1 and int(t.lens[c]) == l + 1:
            return c
    return None


def walk_rank(t, c, i):
    by_rank, cumr = _walk_tables(t)
    if t.lens[c] == 0:
        return i if (t.L == 0 and t.hist[c] > 0) else 0
    p, x = 0, i
    for l in range(int(t.lens[c])):
        s, _ = _node_range(t, by_rank, l, p)
        base = cumr[s]
        b = (int(t.codes[c]) >> (t.L - 1 - l)) & 1
        x = _naive_rank(t, l, b, base + x) - _naive_rank(t, l, b, base)
        p = 2 * p + b
    return x


def walk_select(t, c, k):
    by_rank, cumr = _walk_tables(t)
    if k == 0:
        return oracle.U64_MAX
    if k > int(t.hist[c]):
        return t.n
    if t.L == 0:
        return k - 1
    r = k
    for l in range(int(t.lens[c]) - 1, -1, -1):
        p = int(t.codes[c]) >> (t.L - l) if l else 0
        s, _ = _node_range(t, by_rank, l, p)
        base = cumr[s]
        b = (int(t.codes[c]) >> (t.L - 1 - l)) & 1
        target = _naive_rank(t, l, b, base) + r
        seen = 0
        for j in range(t.level_n[l]):
            if t.bit(l, j) == b:
                seen += 1
                if seen == target:
                    break
        r = j - base + 1
    return r - 1


CASES = [
    ("zipf", 600, 40, 1),
    ("zipf", 500, 256, 1),
    ("uniform", 300, 7, 1),
    ("sparse", 400, 50, 2),  # most symbols absent
    ("two", 200, 9, 1),      # two occurring symbols: one level
    ("one", 50, 5, 1),       # one occurring symbol: no level
    ("fib", 800, 14, 2),     # very skewed counts: long codes
]


def _seq(kind, n, sigma, w, seed):
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[w]
    if kind == "zipf":
        return workloads.zipf(seed, n, sigma, 1.0, w, workloads.permutation(seed + 1, sigma))
    if kind == "uniform":
        return workloads.uniform(seed, n, sigma, w)
    if kind == "sparse":
        return (workloads.uniform(seed, n, 6, w).astype(np.int64) * 7 + 3).astype(dt)
    if kind == "two":
        return np.where(workloads.uniform(seed, n, 3, w) == 0, 2, 6).astype(dt)
    if kind == "one":
        return np.full(n, 4, dtype=dt)
    fib = [1, 1]
    while len(fib) < sigma:
        fib.append(fib[-1] + fib[-2])
    S = np.repeat(np.arange(sigma), fib[:sigma])[:n]
    return S[workloads.permutation(seed, S.size)].astype(dt)


@pytest.mark.parametrize("kind,n,sigma,w", CASES)
def test_huffman_levels_by_walks(kind, n, sigma, w):
    S = _seq(kind, n, sigma, w, 0x4F10 + n)
    t = oracle.OracleTree(S, sigma, huffman=True)
    m = int(np.count_nonzero(t.hist))
    assert t.L == (0 if m <= 1 else int(t.lens.max()))
    # every element is carried down to its code's end: sum of level sizes = sum of count x length
    assert sum(t.level_n) == _cost(t.hist, t.lens)
    by_rank, cumr = _walk_tables(t)
    # node starts: the elements of the symbols ordered before the node's first symbol
    for l in range(t.L):
        for p in range(1 << l):
            s, e = _node_range(t, by_rank, l, p)
            inner = e - s >= 2 or (e - s == 1 and int(t.lens[by_rank[s]]) > l)
            if inner and l < int(t.lens[by_rank[s]]):
                assert int(t.node_start[l][p]) == cumr[s], (l, p)
            else:
                assert int(t.node_start[l][p]) == oracle.U64_MAX, (l, p)
    Sl = [int(x) for x in S]
    for i in range(0, n, max(1, n // 60)):
        assert walk_access(t, by_rank, cumr, i) == Sl[i]
    rng = np.random.default_rng(n)
    for _ in range(40):
        c = int(rng.integers(0, sigma))
        i = int(rng.integers(0, n + 1))
        assert walk_rank(t, c, i) == oracle.brute_rank(Sl, sigma, c, i)
        cnt = int(t.hist[c])
        for k in (1, cnt, cnt + 1, (cnt + 1) // 2):
            assert walk_select(t, c, k) == oracle.brute_select(Sl, sigma, c, k)

"""Pins of the wavelet-matrix oracle (OracleMatrix; no GPU).

* a twelve-symbol matrix worked by hand (golden fixture): level bits, zeros, starts below the last level;
* an independent route: the matrix rebuilt in pure Python by repeated stable zeros-then-ones
  partitions (the oracle instead sorts once per level by the reversed top bits);
* the matrix answers access / rank / select exactly as the definitions do, through the matrix's own
  walks with naive bit counting (top-down access and rank, bottom-up select);
* closed forms: ones of level l = sum over symbols of count(c) times bit L-1-l of c; the starts
  below the last level are the exclusive prefix sums of the counts in reversed-bit order;
* the rank directory and samples of each level equal those of the same bit row counted naively.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rev(x, l):
    return int(format(x, "0%db" % l)[::-1], 2) if l else 0


def test_hand_example():
    with open(os.path.join(GOLDEN, "wm_hand_example.json")) as f:
        g = json.load(f)
    S = np.array(g["text"], dtype=np.uint8)
    m = oracle.OracleMatrix(S, g["sigma"])
    assert m.L == len(g["levels"])
    for l, lev in enumerate(g["levels"]):
        assert m.bit_string(l) == lev["bits"], l
        assert m.zeros[l] == lev["zeros"], l
    for c, st in g["starts"].items():
        assert int(m.starts[int(c)]) == st, c


def _partition_levels(S, sigma):
    """The matrix by its construction rule: level bits, then a stable zeros-then-ones partition."""
    L = oracle.num_levels(sigma)
    seq = [int(x) for x in S]
    rows, zeros = [], []
    for l in range(L):
        sh = L - 1 - l
        bits = [(x >> sh) & 1 for x in seq]
        rows.append("".join(str(b) for b in bits))
        zeros.append(bits.count(0))
        seq = [x for x, b in zip(seq, bits) if b == 0] + [x for x, b in zip(seq, bits) if b == 1]
    starts = {}
    for p, x in enumerate(seq):
        starts.setdefault(x, p)
    return rows, zeros, seq, starts


@pytest.mark.parametrize("sigma,n,w", [(2, 97, 1), (3, 50, 1), (5, 200, 1), (8, 333, 1), (13, 257, 2),
                                       (256, 1500, 1), (1000, 3000, 2), (1, 20, 1)])
def test_matches_repeated_partitions(sigma, n, w):
    S = (workloads.raw(0xA100 + sigma, 0, n) % np.uint64(sigma)).astype(np.uint8 if w == 1 else np.uint16)
    m = oracle.OracleMatrix(S, sigma)
    rows, zeros, last, starts = _partition_levels(S, sigma)
    assert m.L == len(rows)
    for l in range(m.L):
        assert m.bit_string(l) == rows[l], l
        assert m.zeros[l] == zeros[l]
        assert m.ones[l] == n - zeros[l]
    for c, p in starts.items():
        assert int(m.starts[c]) == p


def _rank_bit(m, l, b, x):
    return sum(1 for j in range(x) if m.bit(l, j) == b)


def _select_bit(m, l, b, k):
    seen = 0
    for j in range(m.n):
        if m.bit(l, j) == b:
            seen += 1
            if seen == k:
                return j
    raise ValueError("select beyond count")


def _wm_access(m, i):
    c = 0
    for l in range(m.L):
        b = m.bit(l, i)
        c |= b << (m.L - 1 - l)
        i = m.zeros[l] + _rank_bit(m, l, 1, i) if b else _rank_bit(m, l, 0, i)
    return c


def _wm_rank(m, c, i):
    for l in range(m.L):
        b = (c >> (m.L - 1 - l)) & 1
        i = m.zeros[l] + _rank_bit(m, l, 1, i) if b else _rank_bit(m, l, 0, i)
    return i - int(m.starts[c])


def _wm_select(m, c, k):
    p = int(m.starts[c]) + k - 1
    for l in range(m.L - 1, -1, -1):
        b = (c >> (m.L - 1 - l)) & 1
        p = _select_bit(m, l, 1, p - m.zeros[l] + 1) if b else _select_bit(m, l, 0, p + 1)
    return p


@pytest.mark.parametrize("sigma,n", [(2, 40), (6, 60), (8, 64), (11, 45), (32, 90)])
def test_matrix_walks_reproduce_the_definitions(sigma, n):
    S = (workloads.raw(0xA200 + sigma, 0, n) % np.uint64(sigma)).astype(np.uint8)
    m = oracle.OracleMatrix(S, sigma)
    cnt = np.bincount(S, minlength=sigma)
    for i in range(n):
        assert _wm_access(m, i) == S[i]
    for c in range(sigma):
        for i in range(0, n + 1, 3):
            assert _wm_rank(m, c, i) == int(np.count_nonzero(S[:i] == c))
        for k in range(1, int(cnt[c]) + 1):
            assert _wm_select(m, c, k) == int(np.nonzero(S == c)[0][k - 1])


@pytest.mark.parametrize("sigma", [4, 7, 256, 300, 4099])
def test_closed_forms(sigma):
    n = 20000
    S = workloads.zipf(0xA300 + sigma, n, sigma, 1.0, 2 if sigma > 256 else 1,
                       workloads.permutation(0xA301, sigma))
    m = oracle.OracleMatrix(S, sigma)
    cnt = np.bincount(S, minlength=sigma).astype(np.int64)
    L = m.L
    for l in range(L):
        sh = L - 1 - l
        assert m.ones[l] == int(sum(int(cnt[c]) for c in range(sigma) if (c >> sh) & 1))
    order = sorted(range(sigma), key=lambda c: _rev(c, L))
    acc = 0
    for c in order:
        assert int(m.starts[c]) == acc
        acc += int(cnt[c])


def test_directory_and_samples_of_a_level():
    n, sigma = 150000, 64
    S = (workloads.raw(0xA401, 0, n) % np.uint64(sigma)).astype(np.uint8)
    m = oracle.OracleMatrix(S, sigma, l2_bits=512, sample_rate=4096)
    for l in (0, m.L - 1):
        bits = np.array([m.bit(l, j) for j in range(n)], dtype=np.int64)
        pre = np.concatenate([[0], np.cumsum(bits)])
        L1 = pre[np.minimum(np.arange(0, (n + 65535) // 65536 + 1) * 65536, n)]
        np.testing.assert_array_equal(m.L1[l], L1)
        x = np.minimum(np.arange(0, (n + 511) // 512 + 1) * 512, n)
        np.testing.assert_array_equal(m.L2[l], (pre[x] - pre[np.minimum((x // 65536) * 65536, n)]).astype(np.uint16))
        ones = np.nonzero(bits)[0]
        zeros_ = np.nonzero(bits == 0)[0]
        np.testing.assert_array_equal(m.samples1[l], ones[4095::4096])
        np.testing.assert_array_equal(m.samples0[l], zeros_[4095::4096])

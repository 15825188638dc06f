"""Pins of the all-core form of the CPU oracle (wt_oracle_par.c, used by the bench's all-core CPU
baseline): its answers and tree parts equal those of the serial oracle (itself pinned in
test_oracle.py) and brute force, for thread counts that cut the sequence into uneven chunks, on
tiny inputs exhaustively, on medium random inputs, and at the edges (empty sequence, i = n,
k = 0, k > count, absent and out-of-alphabet symbols)."""
import numpy as np
import pytest

import oracle
import workloads


def _queries(seed, S, sigma, q):
    n = S.size
    r = [workloads.raw(seed + j, 0, q) for j in range(4)]
    c = (r[0] % np.uint64(sigma + 2)).astype(np.uint32)  # includes absent and >= sigma symbols
    i = r[1] % np.uint64(n + 2)                          # includes n and n + 1
    cnt = np.bincount(S, minlength=sigma + 2).astype(np.uint64)
    k = r[2] % (cnt[c] + np.uint64(2))                   # includes 0, count and count + 1
    pos = r[3] % np.uint64(n + 2)
    return c, i, k, pos


@pytest.mark.parametrize("nthreads", [1, 3, 8])
def test_par_queries_equal_brute_force_on_tiny_inputs(nthreads):
    for n, sigma, seed in ((0, 3, 1), (1, 1, 2), (7, 3, 3), (37, 5, 4), (64, 2, 5), (101, 17, 6)):
        S = (workloads.raw(seed, 0, n) % np.uint64(sigma)).astype(np.uint8)
        Sl = list(S)
        # exhaustive over symbols (plus one absent and one out of range), positions and k
        cs = np.repeat(np.arange(sigma + 2, dtype=np.uint32), n + 2)
        xs = np.tile(np.arange(n + 2, dtype=np.uint64), sigma + 2)
        rk = oracle.par_rank(S, sigma, cs, xs, nthreads)
        sl = oracle.par_select(S, sigma, cs, xs, nthreads)
        ac = oracle.par_access(S, np.arange(n + 2, dtype=np.uint64), nthreads)
        for j in range(cs.size):
            assert int(rk[j]) == oracle.brute_rank(Sl, sigma, int(cs[j]), int(xs[j])), (n, sigma, j)
            assert int(sl[j]) == oracle.brute_select(Sl, sigma, int(cs[j]), int(xs[j])), (n, sigma, j)
        for i in range(n + 2):
            assert int(ac[i]) == oracle.brute_access(Sl, i)


@pytest.mark.parametrize("nthreads", [2, 5, 8])
@pytest.mark.parametrize("width,sigma", [(1, 256), (2, 1000), (4, 70000)])
def test_par_queries_equal_serial_oracle(nthreads, width, sigma):
    n = 200_003
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[width]
    S = workloads.zipf(0x51 + width, n, sigma, 1.0, width, workloads.permutation(0x52 + width, sigma)).astype(dt)
    c, i, k, pos = _queries(0x900 + width, S, sigma, 50_000)
    np.testing.assert_array_equal(oracle.par_rank(S, sigma, c, i, nthreads), oracle.rank(S, sigma, c, i))
    np.testing.assert_array_equal(oracle.par_select(S, sigma, c, k, nthreads), oracle.select(S, sigma, c, k))
    np.testing.assert_array_equal(oracle.par_access(S, pos, nthreads), oracle.access(S, pos))


@pytest.mark.parametrize("nthreads", [1, 4, 8])
@pytest.mark.parametrize("n,sigma,width", [(0, 5, 1), (1, 2, 1), (70_001, 256, 1), (100_000, 77, 1),
                                           (65_537, 1000, 2), (40_000, 70_000, 4), (5000, 1, 1)])
def test_par_tree_equals_serial_oracle(nthreads, n, sigma, width):
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[width]
    S = (workloads.raw(0x77 + n, 0, n) % np.uint64(sigma)).astype(dt)
    t = oracle.OracleTree(S, sigma, l2_bits=512, sample_rate=1024, with_nodes=False)
    p = oracle.par_tree(S, sigma, l2_bits=512, sample_rate=1024, nthreads=nthreads)
    assert p["L"] == t.L and p["level_n"] == t.level_n
    for l in range(t.L):
        np.testing.assert_array_equal(p["bits"][l], t.bits[l])
        np.testing.assert_array_equal(p["L1"][l], t.L1[l])
        np.testing.assert_array_equal(p["L2"][l], t.L2[l])
        np.testing.assert_array_equal(p["samples1"][l], t.samples1[l])
        np.testing.assert_array_equal(p["samples0"][l], t.samples0[l])


def test_par_tree_rejects_out_of_range_symbols():
    S = np.array([0, 1, 2, 9], dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.par_tree(S, 5)

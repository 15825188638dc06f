"""GPU parity of alphabet extraction (wt_build with sigma = 0; Section 5.1's minimal alphabet, Section
6.3.1's build with the alphabet extracted).

* the tree's alphabet (WT_PART_ALPHABET) equals the oracle's distinct values of S, sigma their number;
* every part of the tree equals the oracle tree of S rewritten as codes (the index of each value in the
  alphabet) with that sigma, and the declared-alphabet build of the same codes;
* answers, asked and returned in the caller's values (absent values and values beyond the largest
  included), equal the oracle's, from 4 to 2^16 distinct u32 values over small and huge value ranges
  (both presence-map paths), for u8 and u16, one distinct value, and the empty sequence.
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
    wt.lib()


def _seq(width, n, d, hi, seed):
    """n >= d symbols over exactly d distinct values drawn from [0, hi): every value once, in a seeded
    order, then Zipf(1.0) over a seeded permutation."""
    vals = np.unique(workloads.raw(workloads.subseed(seed, 1), 0, 4 * d) % np.uint64(hi))
    vals = vals[workloads.permutation(workloads.subseed(seed, 2), vals.size)][:d]
    assert vals.size == d and n >= d
    idx = workloads.zipf(workloads.subseed(seed, 3), n - d, d, 1.0, 4,
                         workloads.permutation(workloads.subseed(seed, 4), d))
    S = np.concatenate([vals, vals[idx.astype(np.int64)]]).astype(workloads.dtype_for(width))
    return S, np.sort(vals)


def _codes(alpha, x):
    """Values as codes (their index in the alphabet); values not in it become len(alpha) (absent)."""
    x = x.astype(np.uint64)
    i = np.searchsorted(alpha, x)
    ok = (i < alpha.size) & (alpha[np.minimum(i, max(alpha.size - 1, 0))] == x) if alpha.size else np.zeros(x.size, bool)
    return np.where(ok, i, alpha.size).astype(np.uint32)


# (width, n, distinct values, value range)
CASES = [
    (4, 300_001, 4, 1 << 24),        # global presence words (2^18 of them)
    (4, 250_000, 300, 1 << 18),      # LDS presence words
    (4, 400_000, 1 << 16, 1 << 31),  # 2^25 presence words, 16 levels
    (4, 100_000, 1000, 1 << 19),     # exactly the LDS limit (8192 words)
    (1, 200_003, 200, 256),
    (2, 150_000, 5000, 1 << 16),
    (2, 70_000, 1, 1 << 16),         # one distinct value: no levels
]


@pytest.mark.parametrize("width,n,d,hi", CASES, ids=["w%d-n%d-d%d-hi%d" % c for c in CASES])
def test_extracted_alphabet_structure_and_answers(width, n, d, hi):
    import paper_2505_03372_amd as wt
    seed = 0xA1FA + 13 * d + width
    S, vals = _seq(width, n, d, hi, seed)
    G.log("alphabet case w=%d n=%d d=%d hi=%d: build with sigma = 0" % (width, n, d, hi))
    t = wt.build(G.dev(S), 0)
    alpha = oracle.alphabet(S)
    np.testing.assert_array_equal(alpha, vals.astype(np.uint64))
    info = t.info
    assert info["sigma"] == d and info["alphabet_extracted"] and info["max_symbol"] == int(alpha[-1])
    np.testing.assert_array_equal(t.export(wt.PART_ALPHABET).astype(np.uint64), alpha)
    codes = _codes(alpha, S).astype(workloads.dtype_for(width))
    G.log("  structure against the oracle tree of the codes")
    G.compare_structure(t, oracle.OracleTree(codes, d))
    G.log("  structure against the declared-alphabet build of the codes")
    t2 = G.gpu_build(codes, d)
    parts = [wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START,
             wt.PART_NODE_R0]
    for l in range(t2.info["levels"]):
        for part in parts:
            np.testing.assert_array_equal(t.export(part, l), t2.export(part, l))
    t2.free()
    G.log("  answers in the caller's values")
    if hi <= (1 << 24):
        pos, rc, ri, sc, sk = G.random_queries(S, hi, 8192, seed)
    else:  # value range too large for count arrays indexed by value: draw k through the codes
        pos = workloads.uniform(workloads.subseed(seed, 11), 8192, n)
        rc = workloads.draw_from_seq(workloads.subseed(seed, 12), S, 8192)
        ri = workloads.uniform(workloads.subseed(seed, 13), 8192, n + 1)
        sc = workloads.draw_from_seq(workloads.subseed(seed, 14), S, 8192)
        cnt = np.bincount(_codes(alpha, S), minlength=d).astype(np.uint64)
        sk = workloads.draw_k(workloads.subseed(seed, 15), _codes(alpha, sc), cnt, 8192)
    # absent values, values past the largest, k = 0 and k past the count mixed in
    absent = np.setdiff1d(np.arange(min(hi, 2048), dtype=np.uint64), alpha)[:5].astype(np.uint32)
    extra_c = np.concatenate([absent, np.array([alpha[-1] + 1, 0xFFFFFFFF], np.uint64).astype(np.uint32),
                              alpha[:3].astype(np.uint32)])
    rc = np.concatenate([rc, extra_c]); ri = np.concatenate([ri, np.full(extra_c.size, n // 2, np.uint64)])
    sc = np.concatenate([sc, extra_c]); sk = np.concatenate([sk, np.ones(extra_c.size, np.uint64)])
    sk[::97] = 0
    sk[1::89] += np.uint64(1 << 40)
    pos = np.concatenate([pos, np.array([n - 1, n, n + 5], np.uint64)])
    got = G.host(t.access(G.dev(pos)))
    G._assert_eq("access", got, oracle.access(S, pos), pos)
    # the oracle answers on the codes; values map to codes (absent ones to d, outside the alphabet)
    got = G.host(t.rank(G.dev(rc), G.dev(ri)))
    G._assert_eq("rank", got, oracle.rank(codes, d, _codes(alpha, rc), ri), ri)
    got = G.host(t.select(G.dev(sc), G.dev(sk)))
    G._assert_eq("select", got, oracle.select(codes, d, _codes(alpha, sc), sk), sk)
    if hi <= (1 << 24):  # the oracle straight on the values (its count arrays span the value range)
        G._assert_eq("rank on values", G.host(t.rank(G.dev(rc), G.dev(ri))), oracle.rank(S, hi, rc, ri), ri)
        G._assert_eq("select on values", G.host(t.select(G.dev(sc), G.dev(sk))), oracle.select(S, hi, sc, sk), sk)
    if d > 1:
        t.learn_select()
        G._assert_eq("learned select", G.host(t.select_learned(G.dev(sc), G.dev(sk))),
                     oracle.select(codes, d, _codes(alpha, sc), sk), sk)
    t.free()


def test_extracted_alphabet_empty_sequence():
    import paper_2505_03372_amd as wt
    import torch
    t = wt.build(torch.zeros(0, dtype=torch.uint32, device="cuda"), 0)
    assert t.info["sigma"] == 1 and t.info["levels"] == 0 and t.n == 0
    pos = np.array([0, 1, 5], np.uint64)
    assert (G.host(t.access(G.dev(pos))) == 0xFFFFFFFF).all()
    c = np.array([0, 7, 0xFFFFFFFF], np.uint32)
    assert G.host(t.rank(G.dev(c), G.dev(np.zeros(3, np.uint64)))).tolist() == [0, 0, 0]
    assert G.host(t.select(G.dev(c), G.dev(np.array([0, 1, 2], np.uint64)))).tolist() == [2 ** 64 - 1, 0, 0]
    t.free()


def test_extracted_alphabet_binned_batches():
    """Batches above the binning size map their symbols before the binning."""
    import paper_2505_03372_amd as wt
    n, d = 2_000_003, 3000
    S, vals = _seq(4, n, d, 1 << 22, 0xB1B1)
    t = wt.build(G.dev(S), 0)
    alpha = oracle.alphabet(S)
    codes = _codes(alpha, S)
    q = (1 << 17) + 5
    pos, rc, ri, sc, sk = G.random_queries(S, 1 << 22, q, 0x321)
    idx = np.arange(0, q, 37)
    G._assert_eq("access", G.host(t.access(G.dev(pos)))[idx], oracle.access(S, pos[idx]), pos[idx])
    G._assert_eq("rank", G.host(t.rank(G.dev(rc), G.dev(ri)))[idx],
                 oracle.rank(codes, d, _codes(alpha, rc[idx]), ri[idx]), ri[idx])
    G._assert_eq("select", G.host(t.select(G.dev(sc), G.dev(sk)))[idx],
                 oracle.select(codes, d, _codes(alpha, sc[idx]), sk[idx]), sk[idx])
    t.free()

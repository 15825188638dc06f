"""Helpers of the GPU parity tests: run the HIP path through the C ABI and compare with the oracle.

Every comparison is exact (integer work): level bits, L1/L2 directory, select samples, node
tables and cumulative histogram element by element, and the answers of access/rank/select.
"""
from __future__ import annotations

import numpy as np

import oracle
import workloads

PARTS = ("bits", "L1", "L2", "samples1", "samples0", "node_start", "node_r0")


def log(msg: str):
    print(msg, flush=True)


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t) -> np.ndarray:
    return t.cpu().numpy()


def gpu_build(S: np.ndarray, sigma: int, **kw):
    import paper_2505_03372_amd as wt
    return wt.build(dev(S), sigma, **kw)


def compare_structure(t, ot: "oracle.OracleTree"):
    import paper_2505_03372_amd as wt
    info = t.info
    assert info["levels"] == ot.L
    assert info["level_n"] == ot.level_n, (info["level_n"], ot.level_n)
    assert info["level_ones"] == ot.ones, (info["level_ones"], ot.ones)
    np.testing.assert_array_equal(t.export(wt.PART_CUM_HIST), ot.cum_hist)
    parts = {
        "bits": (wt.PART_BITS, ot.bits),
        "L1": (wt.PART_L1, ot.L1),
        "L2": (wt.PART_L2, ot.L2),
        "samples1": (wt.PART_SAMPLES1, ot.samples1),
        "samples0": (wt.PART_SAMPLES0, ot.samples0),
        "node_start": (wt.PART_NODE_START, ot.node_start),
        "node_r0": (wt.PART_NODE_R0, ot.node_r0),
    }
    for l in range(ot.L):
        for name, (part, ref) in parts.items():
            got = t.export(part, l)
            exp = ref[l]
            assert got.shape == exp.shape, (name, l, got.shape, exp.shape)
            if not np.array_equal(got, exp):
                bad = np.nonzero(got != exp)[0]
                raise AssertionError("%s level %d differs at %d places, first %d: got %d expected %d"
                                     % (name, l, bad.size, bad[0], got[bad[0]], exp[bad[0]]))


def edge_queries(S: np.ndarray, sigma: int, rng_seed: int = 1):
    """Boundary arguments of every query kind: ends of the sequence, absent and invalid symbols,
    k = 0, k = count, k = count + 1."""
    n = S.size
    cnt = np.bincount(S, minlength=sigma) if n else np.zeros(sigma, np.int64)
    syms = sorted(set([0, sigma - 1, min(sigma, 255), sigma, sigma + 7]
                      + ([int(S[0]), int(S[-1])] if n else [])
                      + [int(np.argmax(cnt)), int(np.argmin(cnt))]))
    pos = np.array(sorted(set([0, 1, max(n - 1, 0), n, n + 1, n + 1000])), dtype=np.uint64)
    acc = pos
    rc, ri, sc, sk = [], [], [], []
    for c in syms:
        for i in pos:
            rc.append(c)
            ri.append(int(i))
        count = int(cnt[c]) if c < sigma else 0
        for k in sorted(set([0, 1, 2, max(count - 1, 0), count, count + 1])):
            sc.append(c)
            sk.append(k)
    return (acc, np.array(rc, np.uint32), np.array(ri, np.uint64), np.array(sc, np.uint32),
            np.array(sk, np.uint64))


def compare_queries(t, S, sigma, acc_pos=None, rank_c=None, rank_i=None, sel_c=None, sel_k=None):
    if acc_pos is not None and acc_pos.size:
        got = host(t.access(dev(acc_pos.astype(np.uint64))))
        exp = oracle.access(S, acc_pos)
        _assert_eq("access", got, exp, acc_pos)
    if rank_c is not None and rank_c.size:
        got = host(t.rank(dev(rank_c.astype(np.uint32)), dev(rank_i.astype(np.uint64))))
        exp = oracle.rank(S, sigma, rank_c, rank_i)
        _assert_eq("rank", got, exp, np.stack([rank_c.astype(np.uint64), rank_i], 1))
    if sel_c is not None and sel_c.size:
        got = host(t.select(dev(sel_c.astype(np.uint32)), dev(sel_k.astype(np.uint64))))
        exp = oracle.select(S, sigma, sel_c, sel_k)
        _assert_eq("select", got, exp, np.stack([sel_c.astype(np.uint64), sel_k], 1))


def _assert_eq(kind, got, exp, args):
    if not np.array_equal(got, exp):
        bad = np.nonzero(got != exp)[0]
        raise AssertionError("%s differs at %d of %d queries; first: args %s got %d expected %d"
                             % (kind, bad.size, got.size, args[bad[0]], got[bad[0]], exp[bad[0]]))


def random_queries(S, sigma, q, seed):
    n = S.size
    pos = workloads.uniform(workloads.subseed(seed, 1), q, max(n, 1))
    rc = workloads.draw_from_seq(workloads.subseed(seed, 2), S, q) if n else np.zeros(q, np.uint32)
    ri = workloads.uniform(workloads.subseed(seed, 3), q, n + 1)
    sc = workloads.draw_from_seq(workloads.subseed(seed, 4), S, q) if n else np.zeros(q, np.uint32)
    cnt = np.bincount(S, minlength=sigma).astype(np.uint64) if n else np.zeros(sigma, np.uint64)
    sk = workloads.draw_k(workloads.subseed(seed, 5), sc, cnt, q)
    return pos, rc, ri, sc, sk

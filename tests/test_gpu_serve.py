"""GPU tests of the serving loop (continuous batching over a resident forest).

* every request's answers are the same alone (one slot, one request at a time) and in the mix (eight
  slots, overlapping requests: page-locked host buffers, so the copies are asynchronous, and the
  completion records must show requests in different slots on the device at the same time), equal
  to one wt_query_mixed call per request, and equal to the oracle
  on a sample (learned selects inside mixed batches are switched off: answered by the plain select);
* the in-flight device memory never exceeds the budget, and requests still complete exactly.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu

TREES, N = 8, 1 << 20


@pytest.fixture(scope="module")
def served():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_03372_amd as wt
    seqs = []
    for j in range(TREES):
        sj = workloads.subseed(0x5E4E, j)
        seqs.append(workloads.zipf(sj, N, 256, 1.0, 1, workloads.permutation(sj + 1, 256)))
    G.log("serving: forest of %d x 2^20 u8" % TREES)
    f = wt.build_forest([G.dev(S) for S in seqs], [256] * TREES)
    for t in f.trees:
        t.learn_select()
    yield f, seqs
    f.free()


def _trace(seqs, nreq, qmax, seed, gap_s):
    """Poisson arrivals, sizes log-uniform in [1, qmax], 70 % select / 20 % rank / 10 % access."""
    sizes = workloads.loguniform(workloads.subseed(seed, 1), nreq, 1, qmax).astype(np.int64)
    u = workloads.raw(workloads.subseed(seed, 2), 0, nreq).astype(np.float64) / 2.0 ** 64
    arr = np.cumsum(-np.log1p(-u) * gap_s)
    reqs = []
    off = 0
    base = workloads.subseed(seed, 3)
    for i in range(nreq):
        q = int(sizes[i])
        r = workloads.raw(base, off, off + 4 * q)
        off += 4 * q
        tree = (r[:q] % np.uint64(TREES)).astype(np.uint32)
        pick = r[q:2 * q] % np.uint64(10)
        op = np.where(pick < 7, 2, np.where(pick < 9, 1, 0)).astype(np.uint8)
        pos = (r[2 * q:3 * q] % np.uint64(N)).astype(np.uint64)
        sym = np.array([seqs[t][p] for t, p in zip(tree, pos)], dtype=np.uint32)
        arg = pos.copy()
        sel = op == 2
        for t in range(TREES):
            m = sel & (tree == t)
            if m.any():
                cnt = np.bincount(seqs[t], minlength=256).astype(np.uint64)
                arg[m] = 1 + r[3 * q:4 * q][m] % cnt[sym[m]]
        reqs.append(dict(tree=tree, op=op, sym=sym, arg=arg, out=np.zeros(q, np.uint64), arrival_s=float(arr[i])))
    return reqs


def _pinned(a: np.ndarray):
    """Page-locked host copy (asynchronous copies, as the server's callers use)."""
    import torch
    t = torch.empty(a.size, dtype=getattr(torch, str(a.dtype)), pin_memory=True)
    t.numpy()[:] = a
    return t


def _run(f, reqs, slots, budget=0, learned=False, coalesce=0):
    import paper_2505_03372_amd as wt
    rq = []
    for r in reqs:
        op = r["op"].copy()
        if learned:
            op[op == 2] = 3
        rq.append(dict(arrival_s=r["arrival_s"], tree=_pinned(r["tree"]), op=_pinned(op), sym=_pinned(r["sym"]),
                       arg=_pinned(r["arg"]), out=_pinned(np.zeros_like(r["out"]))))
    s = wt.Server(f, slots=slots, mem_budget=budget, coalesce=coalesce)
    comps, st = s.run(rq)
    s.close()
    assert all(c["status"] == wt.WT_OK for c in comps)
    return [r["out"].numpy().copy() for r in rq], comps, st


def _overlapping_pairs(comps) -> int:
    """Pairs of requests in different slots that were on the device at the same time (each admitted
    before the other completed)."""
    n = 0
    for i, a in enumerate(comps):
        for b in comps[i + 1:]:
            if a["slot"] != b["slot"] and a["admit_s"] < b["done_s"] and b["admit_s"] < a["done_s"]:
                n += 1
    return n


def test_results_alone_equal_results_in_the_mix(served):
    f, seqs = served
    reqs = _trace(seqs, 120, 1 << 15, 0x77, 20e-6)
    G.log("serving: mix (8 slots)")
    mix, comps_mix, st_mix = _run(f, reqs, 8)
    G.log("  %s" % st_mix)
    assert st_mix["peak_in_flight"] > 1
    ov = _overlapping_pairs(comps_mix)
    G.log("  overlapping request pairs: %d" % ov)
    assert ov > 0, "no two requests were in flight at the same time"
    G.log("serving: alone (1 slot, one request per batch)")
    alone_reqs = [dict(r, arrival_s=0.0) for r in reqs]
    alone, _, st_alone = _run(f, alone_reqs, 1, coalesce=1)
    assert st_alone["peak_in_flight"] == 1 and st_alone["batches"] == len(reqs)
    for i, r in enumerate(reqs):
        ref = G.host(f.query_mixed(G.dev(r["tree"]), G.dev(r["op"]), G.dev(r["sym"]), G.dev(r["arg"])))
        np.testing.assert_array_equal(mix[i], ref, err_msg="request %d in the mix" % i)
        np.testing.assert_array_equal(alone[i], ref, err_msg="request %d alone" % i)
    # oracle on a sample of every request
    for i in range(0, len(reqs), 7):
        r = reqs[i]
        for t in range(TREES):
            for o in range(3):
                m = np.nonzero((r["tree"] == t) & (r["op"] == o))[0][:50]
                if m.size == 0:
                    continue
                S = seqs[t]
                if o == 0:
                    e = oracle.access(S, r["arg"][m]).astype(np.uint64)
                elif o == 1:
                    e = oracle.rank(S, 256, r["sym"][m], r["arg"][m])
                else:
                    e = oracle.select(S, 256, r["sym"][m], r["arg"][m])
                np.testing.assert_array_equal(mix[i][m], e)


def test_memory_budget_bounds_in_flight_bytes(served):
    f, seqs = served
    reqs = _trace(seqs, 60, 1 << 16, 0x99, 5e-6)
    biggest = max(len(r["arg"]) for r in reqs)
    budget = 3 * (60 * biggest + (1 << 16))
    G.log("serving: budget %d bytes" % budget)
    out, comps, st = _run(f, reqs, 8, budget=budget)
    G.log("  %s" % st)
    assert 0 < st["peak_bytes"] <= budget
    for i, r in enumerate(reqs):
        ref = G.host(f.query_mixed(G.dev(r["tree"]), G.dev(r["op"]), G.dev(r["sym"]), G.dev(r["arg"])))
        np.testing.assert_array_equal(out[i], ref)


def test_coalesced_small_requests(served):
    """Small requests waiting together are answered as coalesced batches (fewer batches than requests)
    with the answers of one wt_query_mixed call per request, including requests of one query and
    all-access requests without symbols."""
    f, seqs = served
    reqs = _trace(seqs, 200, 1 << 12, 0x7A, 0.0)
    for r in reqs[::9]:  # all-access requests, passed without symbols
        r["op"][:] = 0
    G.log("serving: coalesced small requests")
    import paper_2505_03372_amd as wt
    rq = []
    for i, r in enumerate(reqs):
        acc = i % 9 == 0
        rq.append(dict(arrival_s=0.0, tree=_pinned(r["tree"]), op=_pinned(r["op"]),
                       sym=None if acc else _pinned(r["sym"]), arg=_pinned(r["arg"]),
                       out=_pinned(np.zeros_like(r["out"]))))
    s = wt.Server(f, slots=2, coalesce=16384)
    comps, st = s.run(rq)
    s.close()
    G.log("  %s" % st)
    assert all(c["status"] == wt.WT_OK for c in comps)
    assert st["batches"] < len(reqs) // 4
    for i, r in enumerate(reqs):
        ref = G.host(f.query_mixed(G.dev(r["tree"]), G.dev(r["op"]), G.dev(r["sym"]), G.dev(r["arg"])))
        np.testing.assert_array_equal(rq[i]["out"].numpy(), ref, err_msg="request %d" % i)


@pytest.mark.skip(reason="learned selects inside mixed batches are switched off: that traversal (tree arguments per "
                         "lane) faulted once on 64 trees of 2^26 symbols and no cause was found; op 3 is answered by "
                         "the plain select, and the single-tree learned select is tested in test_gpu_learned.py")
def test_learned_selects_in_mixed_batches(served):
    f, seqs = served
    reqs = _trace(seqs, 120, 1 << 15, 0x78, 20e-6)
    lmix, _, _ = _run(f, reqs, 8, learned=True)
    for i, r in enumerate(reqs):
        ref = G.host(f.query_mixed(G.dev(r["tree"]), G.dev(r["op"]), G.dev(r["sym"]), G.dev(r["arg"])))
        np.testing.assert_array_equal(lmix[i], ref, err_msg="request %d learned" % i)


C4_TREES, C4_N = 64, 1 << 26


@pytest.mark.timeout(900)
def test_serving_at_full_shape_plain_ops():
    """The serving workload's shape: 64 resident trees of 2^26 u8 Zipf(1.0) symbols (one forest build).
    A trace of requests of log-uniform size in [1, 2^18] (70 % select, 20 % rank, 10 % access, tree
    uniform per query) answered by the server with 8 slots equals one wt_query_mixed call per request,
    and the oracle on a sample of eight trees."""
    import paper_2505_03372_amd as wt
    import torch
    G.log("c4 shape: generating %d x 2^26 u8 Zipf(1.0)" % C4_TREES)
    fw = workloads.make_forest(trees=C4_TREES, n_range=(C4_N, C4_N), sigma_range=(256, 256), queries=0, width=1,
                               index=4)
    dS = torch.from_numpy(fw.S).cuda()
    G.log("c4 shape: forest build")
    f = wt.build_forest([dS[int(fw.offsets[j]):int(fw.offsets[j + 1])] for j in range(C4_TREES)],
                        [256] * C4_TREES)
    del dS
    nreq = 30
    base = workloads.subseed(0xC4C4, 1)
    sizes = workloads.loguniform(workloads.subseed(base, 1), nreq, 1, 1 << 18).astype(np.int64)
    counts = {}
    reqs = []
    off = 0
    for i in range(nreq):
        q = int(sizes[i])
        r = workloads.raw(workloads.subseed(base, 2), off, off + 4 * q)
        off += 4 * q
        tree = (r[:q] % np.uint64(C4_TREES)).astype(np.uint32)
        pick = r[q:2 * q] % np.uint64(10)
        op = np.where(pick < 7, 2, np.where(pick < 9, 1, 0)).astype(np.uint8)
        pos = r[2 * q:3 * q] % np.uint64(C4_N)
        sym = fw.S[(fw.offsets[tree] + pos).astype(np.int64)].astype(np.uint32)
        arg = pos.copy()
        sel = op == 2
        for t in np.unique(tree[sel]):
            if t not in counts:
                counts[t] = np.bincount(fw.seq(int(t)), minlength=256).astype(np.uint64)
            m = sel & (tree == t)
            arg[m] = 1 + r[3 * q:4 * q][m] % counts[t][sym[m]]
        reqs.append(dict(tree=tree, op=op, sym=sym, arg=arg, out=np.zeros(q, np.uint64), arrival_s=2e-5 * i))
    G.log("c4 shape: serving %d requests, %d queries" % (nreq, int(sizes.sum())))
    out, comps, st = _run(f, reqs, 8)
    G.log("  %s" % st)
    for i, r in enumerate(reqs):
        ref = G.host(f.query_mixed(G.dev(r["tree"]), G.dev(r["op"]), G.dev(r["sym"]), G.dev(r["arg"])))
        np.testing.assert_array_equal(out[i], ref, err_msg="request %d" % i)
    G.log("c4 shape: oracle sample")
    tree_all = np.concatenate([r["tree"] for r in reqs])
    op_all = np.concatenate([r["op"] for r in reqs])
    sym_all = np.concatenate([r["sym"] for r in reqs])
    arg_all = np.concatenate([r["arg"] for r in reqs])
    got_all = np.concatenate(out)
    for t in range(0, C4_TREES, 8):
        S = fw.seq(t)
        for o in range(3):
            m = np.nonzero((tree_all == t) & (op_all == o))[0][:300]
            if m.size == 0:
                continue
            if o == 0:
                e = oracle.access(S, arg_all[m]).astype(np.uint64)
            elif o == 1:
                e = oracle.rank(S, 256, sym_all[m], arg_all[m])
            else:
                e = oracle.select(S, 256, sym_all[m], arg_all[m])
            np.testing.assert_array_equal(got_all[m], e, err_msg="tree %d op %d" % (t, o))
    f.free()

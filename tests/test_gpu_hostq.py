"""GPU tests of queries from host memory (wt_query_host; Section 5.2.1's chunked copy pipeline).

For access, rank and select over page-locked and pageable host arrays, with one chunk, many small
chunks (a ragged last one), chunks large enough to be binned and an exact multiple of the chunk size,
the answers equal those of the device-resident calls on the same queries (which the parity tests pin to
the oracle) and the oracle on a sample. The captured graph of the page-locked path is replayed several
times with other device work and synchronisations between the replays, every replay checked. Also: a
wavelet matrix, an extracted alphabet, the graph-less stream pipeline, q = 0.
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
    yield
    wt.lib().wt_query_host_release()


def _pinned(a):
    import torch
    t = torch.empty(a.size, dtype=getattr(torch, str(a.dtype)), pin_memory=True)
    t.numpy()[:] = a
    return t.numpy(), t  # the tensor keeps the page-locked memory alive


def _device_answers(t, op, sym, arg):
    import paper_2505_03372_amd as wt
    if op == wt.OP_ACCESS:
        return G.host(t.access(G.dev(arg)))
    if op == wt.OP_RANK:
        return G.host(t.rank(G.dev(sym), G.dev(arg)))
    return G.host(t.select(G.dev(sym), G.dev(arg)))


def _oracle(S, sigma, op, sym, arg):
    import paper_2505_03372_amd as wt
    if op == wt.OP_ACCESS:
        return oracle.access(S, arg)
    if op == wt.OP_RANK:
        return oracle.rank(S, sigma, sym, arg)
    return oracle.select(S, sigma, sym, arg)


def _args(S, sigma, op, q, seed):
    import paper_2505_03372_amd as wt
    pos, rc, ri, sc, sk = G.random_queries(S, sigma, q, seed)
    if op == wt.OP_ACCESS:
        return None, pos
    if op == wt.OP_RANK:
        return rc, ri
    return sc, sk


@pytest.fixture(scope="module")
def tree():
    n, sigma = (1 << 21) + 777, 200
    S = workloads.zipf(0x4051, n, sigma, 1.0, 1, workloads.permutation(0x4052, sigma))
    t = G.gpu_build(S, sigma)
    yield t, S, sigma
    t.free()


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("q,chunk", [(1000, 0), (100003, 3000), (300000, 70000), (262144, 65536)])
@pytest.mark.parametrize("opname", ["access", "rank", "select"])
def test_host_queries_equal_device_queries(tree, opname, q, chunk, pinned):
    import paper_2505_03372_amd as wt
    t, S, sigma = tree
    op = {"access": wt.OP_ACCESS, "rank": wt.OP_RANK, "select": wt.OP_SELECT}[opname]
    G.log("host queries: %s q=%d chunk=%d pinned=%s" % (opname, q, chunk, pinned))
    sym, arg = _args(S, sigma, op, q, 0x4053 + q)
    exp = _device_answers(t, op, sym, arg)
    keep = []
    if pinned:
        arg_h, ka = _pinned(arg)
        keep.append(ka)
        sym_h = None
        if sym is not None:
            sym_h, ks = _pinned(sym)
            keep.append(ks)
        out_h, ko = _pinned(np.zeros(q, dtype=exp.dtype))
        keep.append(ko)
    else:
        arg_h, sym_h, out_h = arg.copy(), None if sym is None else sym.copy(), np.zeros(q, dtype=exp.dtype)
    replays = 3 if pinned else 1
    for r in range(replays):
        out_h[:] = 0
        got, st = t.query_host(op, arg_h, sym_h, out=out_h, chunk=chunk)
        assert st["pinned"] == int(pinned)
        assert st["chunks"] == (-(-q // chunk) if chunk else 1)
        assert st["graph"] == int(pinned and st["chunks"] > 1)
        if not np.array_equal(got, exp):
            bad = np.nonzero(got != exp)[0]
            raise AssertionError("replay %d: %d answers differ from the device path, in chunks %s" % (
                r, bad.size, sorted(set((bad // max(chunk, 1)).tolist()))[:20]))
        # other device work and a synchronisation between the replays
        _device_answers(t, op, sym, arg)
    smp = workloads.uniform(0x4054, 1024, q).astype(np.int64)
    np.testing.assert_array_equal(out_h[smp], _oracle(S, sigma, op, None if sym is None else sym[smp], arg[smp]))


def test_host_queries_stream_pipeline_and_empty(tree):
    import paper_2505_03372_amd as wt
    t, S, sigma = tree
    sym, arg = _args(S, sigma, wt.OP_SELECT, 50000, 0x4055)
    sym_h, ks = _pinned(sym)
    arg_h, ka = _pinned(arg)
    out_h, ko = _pinned(np.zeros(sym.size, dtype=np.uint64))
    got, st = t.query_host(wt.OP_SELECT, arg_h, sym_h, out=out_h, chunk=4096, graph=False)
    assert st["graph"] == 0 and st["chunks"] == 13
    np.testing.assert_array_equal(got, _device_answers(t, wt.OP_SELECT, sym, arg))
    got, st = t.query_host(wt.OP_RANK, np.zeros(0, np.uint64), np.zeros(0, np.uint32))
    assert got.size == 0


@pytest.mark.parametrize("kind", ["matrix", "extracted"])
def test_host_queries_other_trees(kind):
    import paper_2505_03372_amd as wt
    n = 500000
    G.log("host queries on a %s tree" % kind)
    if kind == "matrix":
        sigma = 1000
        S = workloads.zipf(0x4056, n, sigma, 1.0, 2, workloads.permutation(0x4057, sigma))
        t = G.gpu_build(S, sigma, matrix=True)
        codes, vals = S, None
    else:
        vals = np.sort(np.unique(workloads.raw(0x4058, 0, 400) % np.uint64(1 << 30)))[:300].astype(np.uint32)
        idx = workloads.zipf(0x4059, n, vals.size, 1.0, 4, workloads.permutation(0x405A, vals.size))
        S = vals[idx.astype(np.int64)]
        t = wt.build(G.dev(S), 0)
        sigma = int(vals.size)
        codes = np.searchsorted(vals, S).astype(np.uint32)
    try:
        for op in (wt.OP_ACCESS, wt.OP_RANK, wt.OP_SELECT):
            sym, arg = _args(codes, sigma, op, 80000, 0x405B + op)
            if vals is not None and sym is not None:
                sym = vals[sym.astype(np.int64)]
            exp = _device_answers(t, op, sym, arg)
            for pinned in (True, False):
                if pinned:
                    arg_h, ka = _pinned(arg)
                    sym_h, ks = _pinned(sym) if sym is not None else (None, None)
                    out_h, ko = _pinned(np.zeros(arg.size, dtype=exp.dtype))
                else:
                    arg_h, sym_h, out_h = arg, sym, np.zeros(arg.size, dtype=exp.dtype)
                got, _ = t.query_host(op, arg_h, sym_h, out=out_h, chunk=20000)
                assert np.array_equal(got, exp), "op %d pinned=%s differs" % (op, pinned)
    finally:
        t.free()
        wt.lib().wt_query_host_release()

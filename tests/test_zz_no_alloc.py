"""GPU test of wt_select_noalloc (select with its buffers in the library's static device array).

Two calls in a row through the C ABI, the second with a smaller batch, each compared element by
element with wt_select on the same queries and with the oracle on a sample: binned batches (at least
2^16 queries) and an unbinned one, a tree with a declared alphabet and one with an extracted alphabet
(the mapped symbols also live in the static array), plus the size limit.
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


def _queries(S, sigma, q, seed, cnt):
    c = workloads.draw_from_seq(seed, S, q)
    k = workloads.draw_k(seed + 1, c, cnt, q)
    # edge arguments: k = 0, k = count + 1, an absent value
    k[:3] = 0
    k[3:6] = cnt[c[3:6].astype(np.int64)] + 1
    c[6] = sigma + 5
    return c, k


def _check_pair(t, S, sigma, c, k, sample, c_oracle=None):
    """wt_select_noalloc against wt_select on every query and against the oracle on a sample (symbols
    given to the oracle as c_oracle when the tree maps values to codes)."""
    import torch
    dc, dk = G.dev(c), G.dev(k)
    ref = t.select(dc, dk)
    out = torch.full((k.size,), 0xDEAD, dtype=torch.uint64, device="cuda")
    t.select_noalloc(dc, dk, out)
    torch.cuda.synchronize()
    got, exp = G.host(out), G.host(ref)
    assert np.array_equal(got, exp), "wt_select_noalloc differs from wt_select at %d places" % int(
        np.count_nonzero(got != exp))
    idx = sample[sample < k.size]
    co = c if c_oracle is None else c_oracle
    assert np.array_equal(got[idx], oracle.select(S, sigma, co[idx], k[idx]))


@pytest.mark.parametrize("first,second", [(1 << 20, 100003), (300000, 1 << 16), (70000, 5000)])
def test_noalloc_select_declared_alphabet(first, second):
    import paper_2505_03372_amd as wt
    n, sigma = (1 << 21) + 777, 256
    G.log("noalloc select: n=%d sigma=%d batches %d then %d" % (n, sigma, first, second))
    S = workloads.zipf(0x50A1, n, sigma, 1.0, 1, workloads.permutation(0x50A2, sigma))
    cnt = np.bincount(S, minlength=sigma + 8).astype(np.uint64)
    t = G.gpu_build(S, sigma)
    try:
        sample = workloads.uniform(0x50A3, 4096, first).astype(np.int64)
        c1, k1 = _queries(S, sigma, first, 0x50A4, cnt)
        _check_pair(t, S, sigma, c1, k1, sample)
        c2, k2 = _queries(S, sigma, second, 0x50A5, cnt)
        _check_pair(t, S, sigma, c2, k2, sample)
    finally:
        t.free()


def test_noalloc_select_extracted_alphabet():
    import paper_2505_03372_amd as wt
    n, d = 1 << 20, 300
    G.log("noalloc select: extracted alphabet, n=%d, %d distinct u32 values" % (n, d))
    vals = np.sort(np.unique(workloads.raw(0x50B1, 0, 4 * d) % np.uint64(1 << 30)))[:d].astype(np.uint32)
    idx = workloads.zipf(0x50B2, n, vals.size, 1.0, 4, workloads.permutation(0x50B3, vals.size))
    S = vals[idx.astype(np.int64)].astype(np.uint32)
    t = wt.build(G.dev(S), 0)
    try:
        d = int(vals.size)
        codes = np.searchsorted(vals, S).astype(np.uint32)  # the oracle answers over the codes 0 .. d-1
        cnt = np.bincount(codes, minlength=d).astype(np.uint64)
        absent = np.uint32(int(vals.max()) + 2)
        for q, seed in ((1 << 19, 0x50B4), (20000, 0x50B5)):
            cc = workloads.draw_from_seq(seed, codes, q)
            k = 1 + workloads.raw(seed + 1, 0, q) % cnt[cc.astype(np.int64)]
            k[:2] = 0
            c = vals[cc.astype(np.int64)]
            c[2], cc[2] = absent, d  # a value that does not occur: code d is past the alphabet
            sample = workloads.uniform(seed + 2, 2048, q).astype(np.int64)
            _check_pair(t, codes, d, c, k, sample, c_oracle=cc)
    finally:
        t.free()


def test_noalloc_select_rejects_oversized_batch():
    import torch
    import paper_2505_03372_amd as wt
    S = workloads.uniform(0x50C1, 4096, 16).astype(np.uint8)
    t = G.gpu_build(S, 16)
    try:
        q = (1 << 20) + 1
        c = torch.zeros(q, dtype=torch.uint32, device="cuda")
        k = torch.ones(q, dtype=torch.uint64, device="cuda")
        out = torch.empty(q, dtype=torch.uint64, device="cuda")
        with pytest.raises(wt.WTError):
            t.select_noalloc(c, k, out)
    finally:
        t.free()

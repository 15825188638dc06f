"""GPU parity of the rank/select support of a plain bit array (wt_bv_build; thesis Section 4 and the
rank/select benchmark of Section 6.1/6.2).

* the structure (bits, L1, L2, select samples, level totals) equals the oracle's definitions applied to
  the bits as a binary sequence (oracle tree with sigma = 2), and the tree wt_build makes of that
  sequence, for lengths around every word, L2, tile and L1 boundary, fill rates 10/50/90 % with the
  uniform and the adversarial placement, several |L2| and s;
* access / rank_b / select_b answers equal the oracle's, with the out-of-domain sentinels;
* a 2^30-bit array at the benchmark's |L2| = 512 and s = 16384: sampled answers against the oracle.
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


def _check(t, bits_u8, l2, s):
    import paper_2505_03372_amd as wt
    n = bits_u8.size
    ot = oracle.OracleTree(bits_u8, 2, l2_bits=l2, sample_rate=s)
    assert t.info["sigma"] == 2 and t.info["levels"] == 1 and t.n == n
    G.compare_structure(t, ot)
    # the same tree as the general build over the binary sequence
    t2 = G.gpu_build(bits_u8, 2, l2_bits=l2, sample_rate=s)
    for part in (wt.PART_BITS, wt.PART_L1, wt.PART_L2, wt.PART_SAMPLES1, wt.PART_SAMPLES0, wt.PART_NODE_START,
                 wt.PART_NODE_R0):
        np.testing.assert_array_equal(t.export(part, 0), t2.export(part, 0))
    np.testing.assert_array_equal(t.export(wt.PART_CUM_HIST), t2.export(wt.PART_CUM_HIST))
    t2.free()
    # answers: random and boundary arguments
    G.compare_queries(t, bits_u8, 2, *G.random_queries(bits_u8, 2, 4096, 0x77 + n))
    G.compare_queries(t, bits_u8, 2, *G.edge_queries(bits_u8, 2))


SIZES = [0, 1, 63, 64, 65, 511, 512, 513, 16383, 16384, 16385, 65535, 65536, 65537, 3 * 65536 + 4097,
         (1 << 20) + 7]


@pytest.mark.parametrize("n", SIZES)
def test_bitvec_sizes(n):
    import paper_2505_03372_amd as wt
    words = workloads.bit_words(0xB1 + n, n, 0.5, False) if n else np.zeros(1, np.uint64)
    bits = workloads.unpack_bits(words, n)
    G.log("bit array n=%d" % n)
    t = wt.build_bitvector(G.dev(words), n, l2_bits=512, sample_rate=512)
    _check(t, bits, 512, 512)
    t.free()


@pytest.mark.parametrize("fill", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("adversarial", [False, True])
@pytest.mark.parametrize("l2,s", [(512, 16384), (256, 1024), (1024, 4096), (2048, 512)])
def test_bitvec_fills(fill, adversarial, l2, s):
    import paper_2505_03372_amd as wt
    n = (1 << 21) + 333
    words = workloads.bit_words(0xF111 + int(fill * 10) + adversarial, n, fill, adversarial)
    bits = workloads.unpack_bits(words, n)
    G.log("bit array fill %.1f %s l2=%d s=%d" % (fill, "adversarial" if adversarial else "uniform", l2, s))
    t = wt.build_bitvector(G.dev(words), n, l2_bits=l2, sample_rate=s)
    _check(t, bits, l2, s)
    t.free()


def test_bitvec_ignores_bits_past_n_and_keeps_no_reference():
    import paper_2505_03372_amd as wt
    n = 1000
    words = np.full(16, np.uint64(0xFFFFFFFFFFFFFFFF))
    d = G.dev(words)
    t = wt.build_bitvector(d, n)
    d.zero_()  # the build copied the bits
    assert t.info["level_ones"] == [n]
    assert G.host(t.rank(G.dev(np.array([1, 1, 0], np.uint32)), G.dev(np.array([n, n + 1, n], np.uint64)))).tolist() \
        == [n, 2 ** 64 - 1, 0]
    t.free()


@pytest.mark.timeout(600)
def test_bitvec_full_size_sampled():
    """2^30 bits, 50 % uniform, |L2| = 512, s = 16384; 2^22 queries of every kind, sampled oracle check."""
    import paper_2505_03372_amd as wt
    n = 1 << 30
    words = workloads.bit_words(0xFA11, n, 0.5, False)
    G.log("bit array 2^30: build")
    t = wt.build_bitvector(G.dev(words), n, l2_bits=512, sample_rate=16384)
    bits = workloads.unpack_bits(words, n)
    ones = int(t.info["level_ones"][0])
    assert ones == int(np.unpackbits(words.view(np.uint8)).sum())
    qs = workloads.make_bitvec_queries(0x5151, n, ones, 1 << 22)
    idx = np.arange(0, 1 << 22, 1024)
    G.log("  access / rank / select")
    got = G.host(t.access(G.dev(qs["pos"])))
    G._assert_eq("access", got[idx], oracle.access(bits, qs["pos"][idx]), qs["pos"][idx])
    for b in (0, 1):
        c = np.full(1 << 22, b, np.uint32)
        got = G.host(t.rank(G.dev(c), G.dev(qs["rank_i"])))
        G._assert_eq("rank%d" % b, got[idx], oracle.rank(bits, 2, c[idx], qs["rank_i"][idx]), qs["rank_i"][idx])
        k = qs["k%d" % b]
        got = G.host(t.select(G.dev(c), G.dev(k)))
        G._assert_eq("select%d" % b, got[idx], oracle.select(bits, 2, c[idx], k[idx]), k[idx])
    t.free()

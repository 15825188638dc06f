"""GPU tests of the learned select index.

* the device loss and gradient (the training kernel's own code) against the FP64 oracle of the
  network, within a relative 1e-4 (FP32 accumulation);
* learned select answers equal to the oracle's and to the plain select's on many trees
  (exactness does not depend on the FP32 model: the prediction is corrected exactly);
* what training gains: the trained networks' mean prediction error (in L2 blocks, over every L2
  boundary of every node) is below that of the untrained starting point (the linear map);
* the piecewise-linear form queries evaluate equals the trained network (FP64 forward pass of the
  exported parameters), and every model sits in the slot of its child node.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import gpu_cases as G
from tests.test_gpu_parity import make_seq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_03372_amd as wt
    wt.lib()


@pytest.mark.parametrize("P,seed", [(1, 1), (7, 2), (300, 3), (2048, 4)])
def test_device_gradient_matches_fp64_reference(P, seed):
    import paper_2505_03372_amd as wt
    r = workloads.raw(0xD00 + seed, 0, P * 2 + 49).astype(np.float64) / 2.0**64
    u = r[:P]
    v = np.sqrt(u) + 0.05 * (r[P:2 * P] - 0.5)
    th = oracle.mlp_init() + 0.2 * (r[2 * P:] - 0.5)
    th32, u32, v32 = th.astype(np.float32), u.astype(np.float32), v.astype(np.float32)
    G.log("mlp grad P=%d" % P)
    out = G.host(wt.mlp_loss_grad(G.dev(th32), G.dev(u32), G.dev(v32)))
    # reference on the same FP32-rounded inputs, in FP64
    loss, grad = oracle.mlp_loss_grad(th32.astype(np.float64), u32.astype(np.float64), v32.astype(np.float64))
    assert abs(out[0] - loss) <= 1e-4 * abs(loss) + 1e-9
    scale = max(1e-6, float(np.abs(grad).max()))
    np.testing.assert_allclose(out[1:], grad, rtol=1e-4, atol=1e-4 * scale)


LEARN_CASES = [
    (1, 256, 1 << 20, "zipf"),
    (1, 256, 1 << 20, "uniform"),
    (1, 77, 300001, "zipf"),
    (1, 5, 100000, "alternate"),
    (1, 2, 70001, "uniform"),
    (1, 7, 131073, "runs"),
    (2, 25, 500000, "zipf"),
    (2, 40000, 300000, "uniform"),
    (4, 1 << 20, 1 << 21, "zipf12"),
    (4, 3, 100001, "uniform"),
    (1, 1, 1000, "equal"),
    (1, 11, 65, "uniform"),
]


@pytest.mark.parametrize("width,sigma,n,kind", LEARN_CASES, ids=["w%d-s%d-n%d-%s" % c for c in LEARN_CASES])
def test_learned_select_is_exact(width, sigma, n, kind):
    seed = 0xBEEF + n + sigma
    S = make_seq(kind, n, sigma, width, seed)
    G.log("learned case w=%d sigma=%d n=%d kind=%s" % (width, sigma, n, kind))
    t = G.gpu_build(S, sigma)
    info = t.learn_select()
    assert info["params_per_model"] == 49
    _, _, _, sc, sk = G.random_queries(S, sigma, 8192, seed)
    got = G.host(t.select_learned(G.dev(sc), G.dev(sk)))
    plain = G.host(t.select(G.dev(sc), G.dev(sk)))
    exp = oracle.select(S, sigma, sc, sk)
    G._assert_eq("learned select vs oracle", got, exp, np.stack([sc.astype(np.uint64), sk], 1))
    G._assert_eq("learned select vs plain", got, plain, np.stack([sc.astype(np.uint64), sk], 1))
    _, _, _, ec, ek = G.edge_queries(S, sigma)
    got = G.host(t.select_learned(G.dev(ec), G.dev(ek)))
    G._assert_eq("learned select edges", got, oracle.select(S, sigma, ec, ek), np.stack([ec.astype(np.uint64), ek], 1))
    t.free()


def test_training_reduces_prediction_error():
    S, sigma = workloads.make_text("text_zipf", n=1 << 24)
    G.log("training gain on text_zipf prefix 2^24")
    t = G.gpu_build(S, sigma)
    info = t.learn_select()
    G.log("  %s" % info)
    assert info["models"] > 0
    assert info["mean_err_blocks"] < 0.8 * info["mean_err_init_blocks"]
    assert info["max_err_blocks"] <= info["max_err_init_blocks"] + 2
    t.free()


def test_learned_search_window_against_sampled_select():
    """What the model saves over the plain select, on the same tree: the plain select searches the L2
    blocks between the two samples around its target (every level and side, weighted by the targets an
    interval holds); the learned select starts at the model's prediction and searches around it. The
    trained models' mean error is well below the plain search range (both in L2 blocks)."""
    import paper_2505_03372_amd as wt
    S, sigma = workloads.make_text("text_zipf", n=1 << 24)
    G.log("learned window vs sampled range on text_zipf prefix 2^24")
    t = G.gpu_build(S, sigma)
    try:
        info = t.learn_select()
        inf = t.info
        s, l2 = inf["sample_rate"], inf["l2_bits"]
        spans, weights = [], []
        for l in range(inf["levels"]):
            nl, ones = inf["level_n"][l], inf["level_ones"][l]
            for part, cnt in ((wt.PART_SAMPLES1, ones), (wt.PART_SAMPLES0, nl - ones)):
                smp = t.export(part, l).astype(np.int64)
                bounds = np.concatenate([[0], smp, [max(nl - 1, 0)]])
                spans.append((bounds[1:] // l2) - (bounds[:-1] // l2) + 1)
                w = np.full(smp.size + 1, s, dtype=np.float64)
                w[-1] = cnt - s * smp.size
                weights.append(w)
        plain = float(np.average(np.concatenate(spans), weights=np.concatenate(weights)))
        G.log("  plain search range %.2f L2 blocks, learned mean error %.2f blocks (training %.2f ms)"
              % (plain, info["mean_err_blocks"], info["train_ms"]))
        assert 2.0 * info["mean_err_blocks"] < plain
    finally:
        t.free()


def test_compiled_models_equal_networks_and_slots():
    sigma, n = 77, 300001
    S = make_seq("zipf", n, sigma, 1, 0xC0DE)
    G.log("compiled models sigma=%d n=%d" % (sigma, n))
    t = G.gpu_build(S, sigma)
    t.learn_select()
    ref = oracle.OracleTree(S, sigma)
    L = ref.L
    u = np.concatenate([(np.arange(1, 200) - 0.5) / 199.0, [1e-6, 1 - 1e-6]])
    trained = 0
    for l in range(L):
        bits = np.unpackbits(np.asarray(ref.bits[l]).view(np.uint8), bitorder="little")[: ref.level_n[l]]
        for p in range(1 << l):
            for b in (0, 1):
                slot = (1 << (l + 1)) - 2 + 2 * p + b
                M = t.learned_model(slot)
                st = int(ref.node_start[l][p])
                if M["eps"] < 0:
                    continue
                trained += 1
                assert (M["level"], M["side"]) == (l, b), slot
                assert M["start"] == st, slot
                seg = bits[st: st + M["len"]]
                assert M["count"] == int((seg == b).sum()), slot
                r0 = int(ref.node_r0[l][p])
                assert M["rank0"] == (st - r0 if b else r0), slot
                kn = M["knots"]
                m = M["pieces"] - 1
                assert 0 <= m <= 16 and np.all(np.diff(kn[:m]) >= 0) and np.all(kn[m:] == 2.0), slot
                th = M["params"].astype(np.float64)
                w1, b1 = th[:16], th[16:32]
                inside = [x for x in (-b1[w1 != 0] / w1[w1 != 0]) if 0 < x < 1]
                assert len(inside) == m, slot
                s_idx = np.searchsorted(kn[:m].astype(np.float64), u, side="right")
                got = M["slope"][s_idx].astype(np.float64) * u + M["intercept"][s_idx].astype(np.float64)
                exp = oracle.mlp_forward(th, u)
                scale = 1.0 + np.abs(th[32:48]).sum() * (np.abs(w1).max() + np.abs(b1).max())
                np.testing.assert_allclose(got, exp, rtol=0, atol=2e-6 * scale, err_msg="slot %d" % slot)
    assert trained > 50
    t.free()


def test_learned_select_full_size_text_zipf():
    """n = 2^30 u8 Zipf(1.0): 2^26 learned selects, sampled check against the oracle."""
    G.log("text_zipf learned: generating")
    wl = workloads.make("text_zipf", kinds=("select",))
    t = G.gpu_build(wl.S, wl.sigma)
    G.log("text_zipf learned: training")
    t.learn_select()
    G.log("text_zipf learned: 2^26 selects")
    got = G.host(t.select_learned(G.dev(wl.sel_c), G.dev(wl.sel_k)))
    idx = np.arange(0, got.size, 1024)
    G._assert_eq("learned select", got[idx], oracle.select(wl.S, wl.sigma, wl.sel_c[idx], wl.sel_k[idx]), wl.sel_k[idx])
    t.free()


@pytest.mark.parametrize("width,sigma,n,kind", [(1, 40, (1 << 21) + 777, "zipf"), (2, 1000, (1 << 20) + 13, "uniform")])
def test_learned_select_every_occurrence_binned(width, sigma, n, kind):
    """Every occurrence of every symbol asked at once, in shuffled order (one binned batch): every
    position of the sequence is the answer of one query, including those just past an L1 block
    boundary, where the learned correction's group crosses into the next L1 block. The answers are
    the positions of each symbol in increasing order (a stable sort of S by symbol)."""
    seed = 0xE0CC + n
    S = make_seq(kind, n, sigma, width, seed)
    G.log("every occurrence, w=%d sigma=%d n=%d kind=%s" % (width, sigma, n, kind))
    t = G.gpu_build(S, sigma)
    t.learn_select()
    cnt = np.bincount(S, minlength=sigma)
    sc = np.repeat(np.arange(sigma, dtype=np.uint32), cnt)
    sk = (np.arange(n, dtype=np.uint64) - np.repeat(np.cumsum(cnt) - cnt, cnt).astype(np.uint64) + 1)
    exp = np.argsort(S, kind="stable").astype(np.uint64)
    perm = np.random.default_rng(seed).permutation(n)
    sc, sk, exp = sc[perm], sk[perm], exp[perm]
    args = np.stack([sc.astype(np.uint64), sk], 1)
    got = G.host(t.select_learned(G.dev(sc), G.dev(sk)))
    G._assert_eq("learned select, every occurrence", got, exp, args)
    G._assert_eq("plain select, every occurrence", G.host(t.select(G.dev(sc), G.dev(sk))), exp, args)
    idx = np.arange(0, n, 997)
    G._assert_eq("oracle sample", exp[idx], oracle.select(S, sigma, sc[idx], sk[idx]), args[idx])
    t.free()

"""GPU checks of the learned area factor: the HIP feature, forward, backward
and Adam kernels against the float64 oracle (and finite differences), the
batched solve started at the predicted factor against the oracle run from
the same start factors, and the autotuner's result invariance."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

KEYS = ("status", "iters", "final_alpha", "applied", "iter_cap", "flow_value", "cut_before",
        "cut_after", "weight_a", "weight_b", "region_vertices", "region_edges")


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def _case(seed=71, n=1 << 15, k=16):
    g = gen.rgg(n, 2, 8.0, seed=seed, wlo=1, whi=10)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.02, seed)
    return g, part, k


def test_pair_features_match_oracle(gpu_lib, ctx):
    g, part, k = _case()
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    f = gpu_lib.fr_pair_features(ctx, g, part.copy(), k, pairs, 30000)
    for i, (a, b) in enumerate(pairs):
        ref = oracle.pair_features(g, part, k, a, b, 30000)
        # computed in float64 on the device and rounded once to float32
        assert np.allclose(f[i], ref.astype(np.float32), rtol=2e-7, atol=1e-7), (i, f[i], ref)


def _oracle_params(fr, w):
    return {k: v.astype(np.float64) for k, v in fr.mlp_unpack(w).items()}


def test_forward_and_gradient_match_oracle(gpu_lib, ctx):
    gpu_lib.fr_mlp_init(ctx, 123)
    w = gpu_lib.fr_mlp_get_weights(ctx)
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1.5, (301, 8)).astype(np.float32)  # several blocks and a ragged tail
    y = rng.integers(0, 5, 301).astype(np.int32)
    P = _oracle_params(gpu_lib, w)
    p_ref, _ = oracle.mlp_forward(P, x.astype(np.float64))
    p_gpu = gpu_lib.fr_mlp_forward(ctx, x)
    assert np.allclose(p_gpu, p_ref, rtol=1e-5, atol=1e-6)
    loss, grad = gpu_lib.fr_mlp_loss_grad(ctx, x, y)
    l_ref, g_ref = oracle.mlp_loss_grad(P, x.astype(np.float64), y)
    assert abs(loss - l_ref) <= 1e-5 * abs(l_ref) + 1e-6
    g_ref_flat = np.concatenate([g_ref[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    scale = np.abs(g_ref_flat).max()
    assert np.allclose(grad, g_ref_flat, rtol=1e-3, atol=1e-5 * scale)


def test_cost_loss_and_gradient_match_oracle(gpu_lib, ctx):
    """The expected-cost loss (per-sample class costs) and its gradient on the
    device against the fp64 reference, over several blocks and a ragged tail."""
    gpu_lib.fr_mlp_init(ctx, 124)
    w = gpu_lib.fr_mlp_get_weights(ctx)
    rng = np.random.default_rng(15)
    x = rng.normal(0, 1.5, (301, 8)).astype(np.float32)
    costs = rng.uniform(0, 2, (301, 5)).astype(np.float32)
    P = _oracle_params(gpu_lib, w)
    loss, grad = gpu_lib.fr_mlp_loss_grad_cost(ctx, x, costs)
    l_ref, g_ref = oracle.mlp_loss_grad_cost(P, x.astype(np.float64), costs.astype(np.float64))
    assert abs(loss - l_ref) <= 1e-5 * abs(l_ref) + 1e-6
    g_ref_flat = np.concatenate([g_ref[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    scale = np.abs(g_ref_flat).max()
    assert np.allclose(grad, g_ref_flat, rtol=1e-3, atol=1e-5 * scale)
    with pytest.raises(gpu_lib.FlowRefineError):
        bad = costs.copy()
        bad[3, 2] = np.nan
        gpu_lib.fr_mlp_loss_grad_cost(ctx, x, bad)


def test_cost_training_learns_the_cheap_class(gpu_lib, ctx):
    """Training on costs 1 - [class = rule(x)]: the expected cost falls and
    the argmax follows the rule."""
    gpu_lib.fr_mlp_init(ctx, 17)
    rng = np.random.default_rng(18)
    x = rng.normal(0, 1.0, (2000, 8)).astype(np.float32)
    y = np.argmax(x[:, :5] + 0.3 * x[:, 5:6], axis=1)
    costs = 1.0 - np.eye(5, dtype=np.float32)[y]
    losses = gpu_lib.fr_mlp_train_cost(ctx, x, costs, epochs=15, batch=128, lr=3e-3, seed=2)
    assert losses[-1] < 0.5 * losses[0]
    acc = np.mean(np.argmax(gpu_lib.fr_mlp_forward(ctx, x), axis=1) == y)
    assert acc > 0.8


def test_predict_is_the_most_probable_factor(gpu_lib, ctx):
    """fr_mlp_predict: 2^c for the most probable class c of the forward pass
    (first on ties), where the fp64 reference is clear of a near-tie."""
    gpu_lib.fr_mlp_init(ctx, 321)
    w = gpu_lib.fr_mlp_get_weights(ctx)
    x = np.random.default_rng(9).normal(0, 2.0, (517, 8)).astype(np.float32)
    p_ref, _ = oracle.mlp_forward(_oracle_params(gpu_lib, w), x.astype(np.float64))
    top2 = np.sort(p_ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-4
    a = gpu_lib.fr_mlp_predict(ctx, x)
    assert set(np.unique(a)) <= {1, 2, 4, 8, 16}
    assert np.array_equal(a[clear], (1 << np.argmax(p_ref, axis=1))[clear])
    assert clear.sum() > 400


def test_gradient_finite_differences(gpu_lib, ctx):
    gpu_lib.fr_mlp_init(ctx, 7)
    w = gpu_lib.fr_mlp_get_weights(ctx).astype(np.float64)
    rng = np.random.default_rng(6)
    x = rng.normal(0, 1.0, (64, 8)).astype(np.float32)
    y = rng.integers(0, 5, 64).astype(np.int32)
    _, grad = gpu_lib.fr_mlp_loss_grad(ctx, x, y)
    h = 2e-3
    for idx in np.argsort(-np.abs(grad))[:12]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        gpu_lib.fr_mlp_set_weights(ctx, wp)
        lp, _ = gpu_lib.fr_mlp_loss_grad(ctx, x, y)
        gpu_lib.fr_mlp_set_weights(ctx, wm)
        lm, _ = gpu_lib.fr_mlp_loss_grad(ctx, x, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[idx]) <= 5e-2 * abs(grad[idx]) + 2e-4, (idx, fd, grad[idx])
    gpu_lib.fr_mlp_set_weights(ctx, w)


def test_adam_step_matches_numpy(gpu_lib, ctx):
    gpu_lib.fr_mlp_init(ctx, 9)
    w0 = gpu_lib.fr_mlp_get_weights(ctx)
    rng = np.random.default_rng(8)
    x = rng.normal(0, 1.0, (32, 8)).astype(np.float32)
    y = rng.integers(0, 5, 32).astype(np.int32)
    _, g = gpu_lib.fr_mlp_loss_grad(ctx, x, y)
    lr = 1e-3
    gpu_lib.fr_mlp_train(ctx, x, y, epochs=1, batch=32, lr=lr, seed=0)  # one full-batch step
    w1 = gpu_lib.fr_mlp_get_weights(ctx)
    # Adam step 1: m = 0.1 g, v = 0.001 g^2, bias-corrected m_hat = g, v_hat = g^2
    step = lr * g / (np.abs(g) + 1e-8)
    ok = np.abs(g) > 1e-5  # sign-stable entries
    assert np.allclose((w0 - w1)[ok], step[ok], rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(w0 - w1) <= lr * 1.0001 + 1e-9)


def test_training_reduces_loss(gpu_lib, ctx):
    gpu_lib.fr_mlp_init(ctx, 11)
    rng = np.random.default_rng(12)
    x = rng.normal(0, 1.0, (2000, 8)).astype(np.float32)
    y = (np.argmax(x[:, :5] + 0.3 * x[:, 5:6], axis=1)).astype(np.int32)  # learnable rule
    losses = gpu_lib.fr_mlp_train(ctx, x, y, epochs=15, batch=128, lr=3e-3, seed=1)
    assert losses[-1] < 0.5 * losses[0]
    acc = np.mean(np.argmax(gpu_lib.fr_mlp_forward(ctx, x), axis=1) == y)
    assert acc > 0.8


def test_batch_with_learned_factor_matches_oracle(gpu_lib, ctx):
    """Flows stay exact under the learned start factor: the oracle, started at
    the factor the device chose for each pair (with the one restart from the
    plain start, rule R6b), gives the same results."""
    import torch

    gpu_lib.fr_mlp_init(ctx, 21)
    g, part, k = _case(seed=73)
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000)
    dg = gpu_lib.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    prm = gpu_lib.params(**p, use_mlp=1)
    res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, prm)
    # the start factors are the argmax of the network on the pairs' features
    feats = gpu_lib.fr_pair_features(ctx, g, part.copy(), k, pairs, 30000)
    probs = gpu_lib.fr_mlp_forward(ctx, feats)
    for i in range(len(pairs)):
        assert res[i]["start_alpha"] == gpu_lib.ALPHAS[int(np.argmax(probs[i]))]
    cur = part.copy()
    for i, (a, b) in enumerate(pairs):
        o = oracle.refine_pair(g, cur, k, a, b,
                               dict(p, alpha=res[i]["start_alpha"], restart_alpha=p["alpha"]),
                               want_side=False)
        for key in KEYS:
            assert res[i][key] == o.result[key], (i, key)
        assert trace[i] == o.trace
        cur = o.part
    assert np.array_equal(dpart.cpu().numpy(), cur)


def test_autotune_keeps_results(gpu_lib, ctx):
    import torch

    g, part, k = _case(seed=75, n=1 << 14, k=8)
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    dg = gpu_lib.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    cands = [dict(block_threads=1024, blocks_per_cu=2, tpv=4, relabel_period=200),
             dict(block_threads=512, blocks_per_cu=4, tpv=8, relabel_period=50),
             dict(block_threads=256, blocks_per_cu=8, tpv=2, relabel_period=400)]
    prm = gpu_lib.params()
    best, ms = gpu_lib.fr_autotune(ctx, dg, dpart, k, pairs, prm, cands, reps=1)
    assert 0 <= best < 3 and all(m > 0 for m in ms)
    assert ctx.get_tuning() == dict(cands[best], mb_lds=1, slice_us=8000)
    assert np.array_equal(dpart.cpu().numpy(), part)  # the partition is not modified
    ctx.set_tuning()


def test_trained_factor_gain(gpu_lib, ctx):
    """What the trained network gains on held-out graphs of the training
    family (one sweep over the colour classes), against the plain adaptive
    search (start at alpha' = 16) and against constant starts at 8 and 4:
    at least 20 % fewer corridor edges than the plain search with the total
    cut at most 1 % above it, and fewer corridor edges than the best constant
    start (8) with the total cut at most 0.1 % above it.  All runs are exact
    flow solves; only the start factor differs."""
    import torch

    gpu_lib.load_trained_mlp(ctx)
    base = dict(alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    runs = {"plain": dict(alpha=16), "constant_8": dict(alpha=8), "constant_4": dict(alpha=4),
            "learned": dict(alpha=16, use_mlp=1)}
    tot = {name: [0, 0, 0] for name in runs}  # solves, region edges, final cut
    for seed in (5001, 5002, 5003):
        g = gen.rgg(1 << 18, 2, 8.0, seed=seed, wlo=1, whi=10)
        part = gen.rcb(g, 64)
        gen.global_noise(g, part, 0.02, seed)
        dg = gpu_lib.DeviceGraph.from_host(g)
        part0 = torch.as_tensor(part).cuda()
        edges, colour = gpu_lib.fr_quotient_matchings(ctx, dg, part0, 64)
        for name, extra in runs.items():
            dpart = part0.clone()
            for c in sorted(set(colour.tolist())):
                pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour.tolist()) if cc == c]
                res, _ = gpu_lib.flow_refine_batch(ctx, dg, dpart, 64, pairs,
                                                   gpu_lib.params(**base, **extra))
                tot[name][0] += sum(r["iters"] for r in res)
                tot[name][1] += sum(r["region_edges"] for r in res)
            tot[name][2] += oracle.total_cut(g, dpart.cpu().numpy())
    print(" | ".join(f"{n}: solves {v[0]} edges {v[1]} cut {v[2]}" for n, v in tot.items()),
          flush=True)
    assert tot["learned"][1] <= 0.8 * tot["plain"][1]
    assert tot["learned"][2] <= 1.01 * tot["plain"][2]
    assert tot["learned"][1] < tot["constant_8"][1]
    assert tot["learned"][2] <= 1.001 * tot["constant_8"][2]


@pytest.mark.parametrize("fused", [False, True])
def test_learned_start_restart_matches_oracle(gpu_lib, fused):
    """The restart of a learned start (R6b) on the device: a network whose
    output is always class 0 starts every pair at factor 1; on the wavy and
    swapped 2-block cases that search stops without improvement, the pair
    restarts from 16 and reaches a lower cut, exactly as the oracle's
    restarted search does (records, result, partition), with the launch
    chains (speculative slots after the restart) and with fused rounds."""
    import torch
    from tests.test_oracle import _swapped, _wavy

    c = gpu_lib.Context()
    try:
        c.set_fused(fused)
        w = np.zeros(gpu_lib.fr_mlp_num_params(), dtype=np.float32)
        w[-5] = 10.0  # b3: class 0 (factor 1) wins on every input
        gpu_lib.fr_mlp_set_weights(c, w)
        p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
                 eps_ppm=30000)
        for g, part in (_wavy(902, 0.2, 1), _wavy(911, 0.2, 1), _swapped(715)):
            print(f"restart case n={g.n} fused={fused}", flush=True)
            o = oracle.refine_pair(g, part, 2, 0, 1, dict(p, alpha=1, restart_alpha=16),
                                   want_side=False)
            plain1 = oracle.refine_pair(g, part, 2, 0, 1, dict(p, alpha=1), want_side=False)
            assert o.result["cut_after"] < plain1.result["cut_after"]
            dpart = torch.as_tensor(part.copy()).cuda()
            res, tr = gpu_lib.flow_refine_batch(c, gpu_lib.DeviceGraph.from_host(g), dpart, 2,
                                                [(0, 1)], gpu_lib.params(**p, use_mlp=1))
            assert res[0]["start_alpha"] == 1
            for key in KEYS:
                assert res[0][key] == o.result[key], key
            assert tr[0] == o.trace
            assert np.array_equal(dpart.cpu().numpy(), o.part)
            assert gpu_lib.stats_dict(c)["restarts"] == 1
    finally:
        c.close()

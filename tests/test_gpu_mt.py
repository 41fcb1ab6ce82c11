"""Multi-try FM (Sec. 4.2) on the GPU against the oracle: batches and single
pairs (result records including the kept multi-try moves, traces,
partition), sweeps with and without active blocks, the closed form of a move
into a third block, the parameter check, and the largest rounds of C3 and C5
at full size (the multi-try phase checked on its own: the GPU batch with it
against the oracle's phase run on the GPU batch without it)."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import csr_from_edges

pytestmark = pytest.mark.gpu

KEYS = ("status", "iters", "final_alpha", "applied", "iter_cap", "flow_value", "cut_before",
        "cut_after", "weight_a", "weight_b", "region_vertices", "region_edges", "mt_kept")


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def _prm(fr, p):
    return fr.params(**{k: v for k, v in p.items() if k in dict(fr.FrParams._fields_)})


def _case(seed, n, k, noise=0.05, wmax=1, deg=6.0):
    g = gen.rgg(n, 2, deg, seed, 1, wmax)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, noise, seed)
    return g, part


def _batch_vs_oracle(fr, ctx, g, part, k, pairs, p):
    import torch

    print(f"mt batch n={g.n} k={k} pairs={len(pairs)} {p}", flush=True)
    rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
    assert rc == 0
    dg = fr.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr = fr.flow_refine_batch(ctx, dg, dpart, k, pairs, _prm(fr, p))
    for i in range(len(pairs)):
        for key in KEYS:
            assert res[i][key] == ores[i][key], (pairs[i], key, res[i][key], ores[i][key])
        assert tr[i] == otr[i]
    assert np.array_equal(dpart.cpu().numpy(), opart)
    return res, fr.stats_dict(ctx)


@pytest.mark.parametrize("seed", range(10))
def test_batch_random(gpu_lib, ctx, seed):
    k = (4, 6, 8)[seed % 3]
    g, part = _case(40 + seed, n=2000 + 500 * seed, k=k, noise=0.04, wmax=1 + seed % 4)
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == seed % 2]
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6,
             eps_ppm=30000 if seed % 4 else 0, mt_alpha=(1, 4, 10)[seed % 3], mt_seed=seed)
    if seed % 5 == 3:
        p.update(fm_limit=20, fm_seed=seed)
    res, st = _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)
    assert st["mt_searches"] > 0


def test_pair_with_multitry(gpu_lib, ctx):
    import torch

    g, part = _case(7, n=6000, k=4, noise=0.05)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=30000, mt_alpha=10, mt_seed=11)
    o = oracle.refine_pair(g, part, 4, 1, 2, p)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr, side = gpu_lib.flow_refine_pair(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 4, 1, 2,
                                             _prm(gpu_lib, p), want_side=True)
    for key in KEYS:
        assert res[key] == o.result[key], key
    assert tr == o.trace and np.array_equal(side, o.side)
    assert np.array_equal(dpart.cpu().numpy(), o.part)
    assert res["mt_kept"] > 0


def test_third_block_move(gpu_lib, ctx):
    """Vertex 0 (block 0) has its three neighbours in block 2: the pair
    (0, 1) refinement's multi-try round moves it there."""
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (4, 5), (5, 6), (1, 7), (7, 8), (4, 8)]
    g = csr_from_edges(9, edges)
    part = np.array([0, 2, 2, 2, 1, 1, 1, 2, 2], dtype=np.int32)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=1_000_000, mt_alpha=10, mt_seed=3)
    res, _ = _batch_vs_oracle(gpu_lib, ctx, g, part, 3, [(0, 1)], p)
    assert res[0]["mt_kept"] >= 1


@pytest.mark.parametrize("active", [0, 1])
def test_sweep(gpu_lib, ctx, active):
    import torch

    k = 8
    g, part = _case(61 + active, n=6000, k=k, noise=0.04, wmax=3)
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6,
             eps_ppm=30000, mt_alpha=10, mt_seed=5, active_blocks=active)
    rc, tc, stats, opart = oracle.sweep(g, part, k, p, max_sweeps=5)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    cut, st = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, k,
                                        _prm(gpu_lib, p), 5)
    assert cut == tc and st.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


def test_rejects_negative_alpha(gpu_lib, ctx):
    import torch

    g, part = _case(3, n=500, k=2)
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, gpu_lib.DeviceGraph.from_host(g),
                                 torch.as_tensor(part).cuda(), 2, 0, 1,
                                 gpu_lib.params(mt_alpha=-1))
    assert e.value.code == -8


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_largest_round_multitry_phase(gpu_lib, cid):
    """The largest round of C3 / C5 with multi-try (alpha 10): the GPU batch
    without it gives the pairwise partition (checked against the oracle pair
    by pair elsewhere); the oracle's multi-try phase on that partition must
    equal the GPU batch with it, move counts included.  C3's todo lists exceed
    the LDS sort (the rank-sort path)."""
    import torch

    w = gen.config(cid)
    c = gpu_lib.Context()
    c.set_validation(False)
    try:
        dg = gpu_lib.DeviceGraph.from_host(w.graph)
        part0 = torch.as_tensor(w.part).cuda()
        edges, colour = gpu_lib.fr_quotient_matchings(c, dg, part0, w.k)
        cls = int(np.argmax(np.bincount(colour)))
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour.tolist()) if cc == cls]
        base = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                         "max_iters", "eps_ppm")}
        print(f"{cid} largest round with multi-try, {len(pairs)} pairs", flush=True)
        d0 = part0.clone()
        res0, _ = gpu_lib.flow_refine_batch(c, dg, d0, w.k, pairs, gpu_lib.params(**base))
        d1 = part0.clone()
        res1, _ = gpu_lib.flow_refine_batch(c, dg, d1, w.k, pairs,
                                            gpu_lib.params(**base, mt_alpha=10, mt_seed=1))
        st = gpu_lib.stats_dict(c)
        m = oracle.multitry(w.graph, d0.cpu().numpy(), w.k, pairs, w.params["eps_ppm"], 10, 1,
                            max_events=None)
        assert np.array_equal(d1.cpu().numpy(), m.part)
        assert [r["mt_kept"] for r in res1] == m.kept
        assert (st["mt_searches"], st["mt_moves"], st["mt_kept"]) == (
            m.stats["searches"], m.stats["moves"], m.stats["kept"])
        for r0, r1 in zip(res0, res1):
            assert {x: r0[x] for x in KEYS if x != "mt_kept"} == \
                   {x: r1[x] for x in KEYS if x != "mt_kept"}
        print(f"  multi-try: {st['mt_searches']} searches, {st['mt_moves']} moves, "
              f"{st['mt_kept']} kept", flush=True)
    finally:
        c.close()

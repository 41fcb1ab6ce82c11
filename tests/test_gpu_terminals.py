"""GPU parity of the contracted terminals (terminals = 1): the parts of the
two blocks outside the corridor contracted into s and t with the weights of
the edges into them as capacities, so that no corridor vertex is pinned.
The HIP path through the C ABI against the oracle, bit for bit (records,
results, partitions, side codes), alone and with every other option."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import csr_from_edges, random_graph
from tests.test_gpu_parity import RESULT_KEYS

pytestmark = pytest.mark.gpu

PKEYS = ("area_mode", "depth", "alpha", "alpha_max", "adaptive", "max_iters", "eps_ppm",
         "mb_reps", "mb_seed", "fm_limit", "fm_seed", "active_blocks", "cut_side", "terminals")


def _prm(fr, d):
    unknown = set(d) - set(PKEYS)
    assert not unknown, unknown  # every oracle parameter must reach the library too
    return fr.params(**{k: d[k] for k in PKEYS if k in d})


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def _compare(fr, ctx, g, part, k, a, b, p):
    import torch

    print(f"terminals case n={g.n} k={k} pair=({a},{b}) params={p}", flush=True)
    o = oracle.refine_pair(g, part, k, a, b, p)
    assert o.rc == 0
    dg = fr.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, trace, side = fr.flow_refine_pair(ctx, dg, dpart, k, a, b, _prm(fr, p), want_side=True)
    for key in RESULT_KEYS:
        assert res[key] == o.result[key], (key, res[key], o.result[key])
    assert len(trace) == len(o.trace)
    for t_gpu, t_or in zip(trace, o.trace):
        assert t_gpu == t_or, (t_gpu, t_or)
    assert np.array_equal(side, o.side)
    assert np.array_equal(dpart.cpu().numpy(), o.part)
    return res, trace


def test_hand_example(gpu_lib, ctx):
    # vertex 1 (block 0) is tied to block 1 by two edges of weight 5: pinned
    # it cannot move (cut 10 stays); contracted it crosses and the cut is 1
    g = csr_from_edges(5, [(0, 1), (1, 2), (1, 3), (2, 4), (3, 4)], weights=[1, 5, 5, 1, 1],
                       vwgt=[3, 1, 1, 1, 1])
    part = np.array([0, 0, 1, 1, 1], dtype=np.int32)
    p = dict(area_mode=1, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=30000)
    res, _ = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    assert res["cut_after"] == 10
    res, trace = _compare(gpu_lib, ctx, g, part, 2, 0, 1, dict(p, terminals=1))
    assert (trace[0]["flow"], res["cut_after"]) == (1, 1)


@pytest.mark.parametrize("seed", range(20))
def test_tiny_random(gpu_lib, ctx, seed):
    rng = np.random.default_rng(1500 + seed)
    n = int(rng.integers(6, 60))
    k = 3 if seed % 4 == 3 else 2
    g = random_graph(n, 0.15, 1500 + seed, wmax=int(rng.choice([1, 3, 9])),
                     vwmax=int(rng.choice([1, 4])))
    part = rng.integers(0, k, n).astype(np.int32)
    part[0], part[1] = 0, 1
    a, b = (0, 1) if seed % 2 == 0 else (1, 0)
    al = int(rng.choice([1, 2, 4, 8, 16]))
    p = dict(area_mode=0, depth=0, alpha=al, alpha_max=16, adaptive=int(seed % 3 != 0),
             max_iters=6, eps_ppm=int(rng.choice([0, 30000, 100000, 300000])), terminals=1)
    if seed % 5 == 0:
        p = dict(p, area_mode=1, depth=int(rng.integers(0, 3)))
    if seed % 7 == 1:
        p = dict(p, cut_side=int(rng.integers(1, 3)))
    _compare(gpu_lib, ctx, g, part, k, a, b, p)


@pytest.mark.parametrize("n,seed,whi", [(1 << 12, 3, 1), (1 << 13, 4, 10), (1 << 15, 6, 3),
                                        (1 << 17, 8, 10)])
def test_rgg_adaptive(gpu_lib, ctx, n, seed, whi):
    g = gen.rgg(n, 2, 8.0, seed, 1, whi)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.02, seed)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, terminals=1)
    res, _ = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    o0 = oracle.refine_pair(g, part, 2, 0, 1, dict(p, terminals=0), want_side=False)
    print("cut pinned", o0.result["cut_after"], "contracted", res["cut_after"])


@pytest.mark.parametrize("opt", ["mb", "fm", "fm_mb", "largest"])
def test_with_other_options(gpu_lib, ctx, opt):
    g = gen.rgg(1 << 14, 2, 7.0, 31, 1, 5)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, 31)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, terminals=1)
    extra = dict(mb=dict(mb_reps=8, mb_seed=7), fm=dict(fm_limit=50, fm_seed=7),
                 fm_mb=dict(mb_reps=8, mb_seed=7, fm_limit=50, fm_seed=7),
                 largest=dict(cut_side=2))[opt]
    _compare(gpu_lib, ctx, g, part, 2, 0, 1, dict(p, **extra))


@pytest.mark.parametrize("spec", [False, True])
def test_speculation_on_off(gpu_lib, spec):
    g = gen.rgg(1 << 14, 2, 7.0, 41, 1, 1)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, 41)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, terminals=1)
    c = gpu_lib.Context()
    try:
        c.set_speculation(spec)
        c.set_fused(not spec)  # launch chains with speculation, else the fused round kernel
        _compare(gpu_lib, c, g, part, 2, 0, 1, p)
    finally:
        c.close()


@pytest.mark.parametrize("seed,n,k,dim,whi", [(81, 1 << 14, 8, 2, 1), (82, 1 << 15, 16, 3, 1),
                                              (83, 1 << 15, 16, 2, 10)])
def test_batch_round(gpu_lib, ctx, seed, n, k, dim, whi):
    import torch

    g = gen.rgg(n, dim, 8.0 if dim == 2 else 12.0, seed=seed, wlo=1, whi=whi)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.02, seed)
    edges, colour = oracle.quotient_colouring(g, part, k)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, terminals=1)
    dg = gpu_lib.DeviceGraph.from_host(g)
    for c in sorted(set(colour.tolist()))[:2]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        print(f"terminals batch n={n} k={k} colour={c} pairs={len(pairs)}", flush=True)
        rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
        assert rc == 0
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, _prm(gpu_lib, p))
        for i in range(len(pairs)):
            for key in RESULT_KEYS:
                assert res[i][key] == ores[i][key], (i, key)
            assert trace[i] == otr[i]
        assert np.array_equal(dpart.cpu().numpy(), opart)


@pytest.mark.parametrize("active", [0, 1])
def test_sweep(gpu_lib, ctx, active):
    import torch

    g = gen.rgg(1 << 14, 2, 7.0, 91, 1, 3)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.02, 91)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, terminals=1, active_blocks=active)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=4)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 4)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


def test_corridor_beyond_lds_bitmaps(gpu_lib, ctx):
    """More than 131,072 corridor vertices: the relabel start list, labels and
    marks live in device memory."""
    import torch

    w = gen.config("C2", n_override=1 << 19)
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "eps_ppm")}
    p.update(adaptive=0, max_iters=1, terminals=1)
    o = oracle.refine_pair(w.graph, w.part, 2, 0, 1, p, want_side=True)
    assert o.result["region_vertices"] > 131072
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part.copy()).cuda()
    res, trace, side = gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 1, _prm(gpu_lib, p),
                                                want_side=True)
    for key in RESULT_KEYS:
        assert res[key] == o.result[key], key
    assert trace == o.trace
    assert np.array_equal(side, o.side)
    assert np.array_equal(dpart.cpu().numpy(), o.part)


def test_rejects_unknown_mode(gpu_lib, ctx):
    g = csr_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    part = np.array([0, 0, 1, 1], dtype=np.int32)
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, g, part, 2, 0, 1, gpu_lib.params(terminals=2))
    assert e.value.code == -8


def test_contracted_capacity_overflow(gpu_lib, ctx):
    # vertex 1 (block 0, on the boundary) has three edges of weight 2^30 - 1
    # into block 0 outside the boundary-only corridor: pinned, they are not
    # capacities at all; contracted, they make the arc s -> 1 exceed 2^31
    w = (1 << 30) - 1
    g = csr_from_edges(6, [(1, 0), (1, 2), (1, 3), (1, 4), (4, 5)], weights=[w, w, w, 1, 1])
    part = np.array([0, 0, 0, 0, 1, 1], dtype=np.int32)
    p = dict(area_mode=1, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=30000)
    _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, g, part, 2, 0, 1, _prm(gpu_lib, dict(p, terminals=1)))
    assert e.value.code == -5
    assert gpu_lib.stats_dict(ctx)["diag"] == 5  # the capacity bound of the network

"""GPU parity of the pairwise 2-way FM local search with TopGain (Sec. 2.2)
that runs before the flow: whole pair, batch and sweep results against the
oracle, bit for bit, and the FM move counts against the oracle's FM alone.
The queues are ordered by (gain, per-vertex key), which fixes the move
sequence however the heaps are built."""
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


def _compare(fr, ctx, g, part, k, a, b, p, fm_only_check=True):
    import torch

    print(f"fm case n={g.n} k={k} pair=({a},{b}) params={p}", flush=True)
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
    st = fr.stats_dict(ctx)
    if fm_only_check:
        _, info, _ = oracle.pair_fm(g, part, k, a, b, p["eps_ppm"], p["fm_limit"], p["fm_seed"])
        assert (st["fm_steps"], st["fm_kept"]) == (info["steps"], info["kept"])
    return res, st


def test_grid_misplaced_vertex(gpu_lib, ctx):
    g = gen.grid2d(10, 10)
    x = np.arange(100) % 10
    part = (x >= 5).astype(np.int32)
    part[45] = 0
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=30000, fm_limit=10, fm_seed=3)
    res, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    assert res["cut_before"] == 12 and st["fm_kept"] == 1


def test_path_overloaded(gpu_lib, ctx):
    g = csr_from_edges(20, [(i, i + 1) for i in range(19)])
    part = (np.arange(20) >= 14).astype(np.int32)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=4, adaptive=1, max_iters=4, eps_ppm=0,
             fm_limit=5, fm_seed=1)
    res, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    assert st["fm_kept"] == 3 and (res["weight_a"], res["weight_b"]) == (11, 9)


@pytest.mark.parametrize("seed", range(16))
def test_tiny_random(gpu_lib, ctx, seed):
    rng = np.random.default_rng(1200 + seed)
    n = int(rng.integers(8, 60))
    g = random_graph(n, 0.15, 1200 + seed, wmax=int(rng.choice([1, 6])),
                     vwmax=int(rng.choice([1, 3])))
    k = int(rng.choice([2, 3]))
    part = rng.integers(0, k, n).astype(np.int32)
    part[0], part[1] = 0, 1
    al = int(rng.choice([1, 4, 16]))
    p = dict(area_mode=0, depth=0, alpha=al, alpha_max=16, adaptive=int(seed % 3 != 0),
             max_iters=5, eps_ppm=int(rng.choice([0, 30000, 300000])),
             fm_limit=int(rng.integers(1, 30)), fm_seed=int(rng.integers(0, 2**32)))
    if seed % 4 == 1:
        p = dict(p, mb_reps=3, mb_seed=seed)
    _compare(gpu_lib, ctx, g, part, k, 0, 1, p)


@pytest.mark.parametrize("n,seed,whi", [(1 << 12, 3, 1), (1 << 14, 4, 10), (1 << 15, 6, 3)])
def test_rgg_pairs(gpu_lib, ctx, n, seed, whi):
    g = gen.rgg(n, 2, 7.0, seed, 1, whi)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, seed)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, fm_limit=100, fm_seed=seed)
    _, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    print("fm", st["fm_steps"], st["fm_kept"])


def test_fm_with_most_balanced_and_speculation(gpu_lib):
    g = gen.rgg(1 << 14, 2, 7.0, 21, 1, 1)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, 21)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, mb_reps=8, mb_seed=3, fm_limit=60, fm_seed=9)
    for spec in (False, True):
        c = gpu_lib.Context()
        try:
            c.set_speculation(spec)
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
             eps_ppm=30000, fm_limit=80, fm_seed=seed)
    dg = gpu_lib.DeviceGraph.from_host(g)
    for c in sorted(set(colour.tolist()))[:2]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        print(f"fm batch n={n} k={k} colour={c} pairs={len(pairs)}", flush=True)
        rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
        assert rc == 0
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, _prm(gpu_lib, p))
        for i in range(len(pairs)):
            for key in RESULT_KEYS:
                assert res[i][key] == ores[i][key], (i, key)
            assert trace[i] == otr[i]
        assert np.array_equal(dpart.cpu().numpy(), opart)


def test_sweep(gpu_lib, ctx):
    import torch

    g = gen.rgg(1 << 14, 2, 7.0, 91, 1, 1)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.02, 91)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, fm_limit=50, fm_seed=91)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=3)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 3)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


def test_rejects_negative_limit(gpu_lib, ctx):
    g = csr_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    part = np.array([0, 0, 1, 1], dtype=np.int32)
    with pytest.raises(gpu_lib.FlowRefineError):
        gpu_lib.flow_refine_pair(ctx, g, part, 2, 0, 1, gpu_lib.params(fm_limit=-1))


def test_gain_overflow(gpu_lib, ctx):
    # vertex 0 has three edges of weight 2^30 - 1 into the other block: its
    # FM gain does not fit int32, so the FM pass reports FR_E_OVERFLOW
    w = (1 << 30) - 1
    g = csr_from_edges(5, [(0, 1), (0, 2), (0, 3), (3, 4)], weights=[w, w, w, 1])
    part = np.array([0, 1, 1, 1, 0], dtype=np.int32)
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, g, part, 2, 0, 1, gpu_lib.params(fm_limit=10))
    assert e.value.code == -5
    assert gpu_lib.stats_dict(ctx)["diag"] == 7  # raised by the FM pass


@pytest.mark.parametrize("fm", [0, 50])
def test_sweep_active_blocks(gpu_lib, ctx, fm):
    import torch

    g = gen.rgg(1 << 14, 2, 7.0, 93, 1, 1)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.03, 93)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, fm_limit=fm, fm_seed=93, active_blocks=1)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=8)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 8)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


@pytest.mark.parametrize("seed", range(20))
def test_random_rounds_all_options(gpu_lib, seed):
    """Randomised whole rounds mixing every option: most balanced cuts, FM
    before the flow, the candidate side, the terminals, speculation, weights
    and k; and a short sweep with active blocks on every fourth seed."""
    import torch

    rng = np.random.default_rng(3100 + seed)
    dim = int(rng.choice([2, 3]))
    n = int(rng.choice([1 << 11, 1 << 12, 1 << 13]))
    whi = int(rng.choice([1, 1, 4, 10]))
    g = gen.rgg(n, dim, 8.0 if dim == 2 else 11.0, 3100 + seed, 1, whi)
    k = int(rng.choice([2, 4, 8, 16]))
    part = gen.rcb(g, k)
    gen.global_noise(g, part, float(rng.choice([0.01, 0.03, 0.06])), seed)
    amax = int(rng.choice([1, 3, 8, 16]))
    mb = int(rng.choice([0, 0, 1, 5, 17]))
    p = dict(area_mode=0, depth=0, alpha=int(rng.integers(1, amax + 1)), alpha_max=amax,
             adaptive=int(rng.integers(0, 2)), max_iters=int(rng.integers(1, 12)),
             eps_ppm=int(rng.choice([0, 30000, 100000])), mb_reps=mb,
             mb_seed=int(rng.integers(0, 2**32)), fm_limit=int(rng.choice([0, 0, 5, 60, 300])),
             fm_seed=int(rng.integers(0, 2**32)), cut_side=int(rng.integers(0, 3)))
    c = gpu_lib.Context()
    try:
        c.set_speculation(bool(rng.integers(0, 2)))
        c.set_validation(bool(rng.integers(0, 2)))
        c.set_fused(seed % 2 == 0)
        p["terminals"] = int(rng.integers(0, 2))
        dg = gpu_lib.DeviceGraph.from_host(g)
        if seed % 4 == 3:
            p["active_blocks"] = 1
            print(f"sweep seed={seed} n={n} k={k} params={p}", flush=True)
            rc, tc, stats, opart = oracle.sweep(g, part, k, p, max_sweeps=3)
            assert rc == 0
            dpart = torch.as_tensor(part.copy()).cuda()
            tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(c, dg, dpart, k, _prm(gpu_lib, p), 3)
            assert tc_gpu == tc and st_gpu.tolist() == stats.tolist()
            assert np.array_equal(dpart.cpu().numpy(), opart)
            return
        edges, colour = oracle.quotient_colouring(g, part, k)
        cls = int(rng.integers(0, colour.max() + 1))
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == cls]
        print(f"round seed={seed} n={n} k={k} pairs={len(pairs)} params={p}", flush=True)
        rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
        assert rc == 0
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace = gpu_lib.flow_refine_batch(c, dg, dpart, k, pairs, _prm(gpu_lib, p))
        for i in range(len(pairs)):
            for key in RESULT_KEYS:
                assert res[i][key] == ores[i][key], (i, key)
            assert trace[i] == otr[i]
        assert np.array_equal(dpart.cpu().numpy(), opart)
    finally:
        c.close()

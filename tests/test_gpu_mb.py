"""GPU parity of the most balanced minimum cut (Sec. 4.1.1) and of the
balanced adaptive flow iterations: the HIP path through the C ABI against
the oracle, bit for bit (records, results, partitions, side codes).  The
residual components and their reachability order are the same for every
maximum flow or preflow, and the sweeps use nothing else, so the outputs are
unique given the seed."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import csr_from_edges, random_graph
from tests.test_gpu_parity import RESULT_KEYS

pytestmark = pytest.mark.gpu

PKEYS = ("area_mode", "depth", "alpha", "alpha_max", "adaptive", "max_iters", "eps_ppm",
         "mb_reps", "mb_seed", "cut_side")


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

    print(f"mb case n={g.n} k={k} pair=({a},{b}) params={p}", flush=True)
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
    return res, trace, fr.stats_dict(ctx)


def _ladder(cols):
    edges = []
    for c in range(cols):
        edges.append((c, cols + c))
        if c + 1 < cols:
            edges += [(c, c + 1), (cols + c + 1, cols + c)]
    return csr_from_edges(2 * cols, edges)


def test_ladder_closed_form(gpu_lib, ctx):
    """2 x 100 ladder with a jagged cut of 3: the most balanced minimum cut
    is the vertical cut between columns 49 and 50 (100 : 100, cut 2)."""
    g = _ladder(100)
    col = np.arange(200) % 100
    part = (col >= 40).astype(np.int32)
    part[40] = 0
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=30000, mb_reps=4, mb_seed=12345)
    res, trace, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    assert (trace[0]["wa"], trace[0]["wb"], trace[0]["decision"]) == (100, 100, 1)
    assert res["cut_after"] == 2
    assert st["mb_free"] > 0 and st["mb_comp"] > 0 and st["mb_big"] == 0


@pytest.mark.parametrize("seed", range(16))
def test_tiny_random(gpu_lib, ctx, seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(6, 50))
    g = random_graph(n, 0.2, 900 + seed, wmax=3, vwmax=4 if seed % 2 else 1)
    part = (rng.random(n) < 0.5).astype(np.int32)
    if part.min() == part.max():
        part[0] = 1 - part[0]
    al = int(rng.choice([1, 2, 4, 8, 16]))
    p = dict(area_mode=0, depth=0, alpha=al, alpha_max=16, adaptive=int(seed % 3 != 0),
             max_iters=6, eps_ppm=int(rng.choice([30000, 100000, 300000])),
             mb_reps=int(rng.choice([1, 3, 16, 64, 65])), mb_seed=int(rng.integers(0, 2**32)))
    if seed % 5 == 0:
        p = dict(p, area_mode=1, depth=int(rng.integers(0, 3)))
    _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)


@pytest.mark.parametrize("n,seed,whi", [(1 << 12, 3, 1), (1 << 13, 4, 10), (1 << 14, 5, 1),
                                        (1 << 15, 6, 3)])
def test_rgg_balanced_adaptive(gpu_lib, ctx, n, seed, whi):
    g = gen.rgg(n, 2, 7.0, seed, 1, whi)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, seed)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, mb_reps=8, mb_seed=seed)
    _, _, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    print("mb stats", {k: st[k] for k in ("mb_free", "mb_comp", "mb_big", "mb_kernel_ms")})


def _path(n):
    return csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])


@pytest.mark.parametrize("n", [3000, 5000, 12000])
def test_path_many_components(gpu_lib, ctx, n):
    """Unit path split at 40 %: flow 1 saturates every corridor edge, so every
    free vertex is its own component.  n = 3000: about 1,400 components (the
    device-memory Tarjan, the component graph in LDS); n = 5000 and 12,000:
    more than 2,048 components, so the component graph and the sweep state
    are in device memory -- the sweeps still run and match the oracle."""
    g = _path(n)
    part = (np.arange(n) >= int(0.4 * n)).astype(np.int32)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=4,
             eps_ppm=30000, mb_reps=5, mb_seed=99)
    _, _, st = _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)
    if n >= 5000:
        assert st["mb_big"] > 0 and st["mb_comp"] > 2048
    else:
        assert st["mb_big"] == 0 and st["mb_comp"] > 1024


@pytest.mark.parametrize("case", ["ladder", "rgg", "path"])
def test_lds_and_device_memory_paths_agree(gpu_lib, case):
    """mb_lds = 0 keeps the quotient graph, Tarjan's scratch and the component
    arcs in device memory; the results equal the LDS path's and the oracle's."""
    if case == "ladder":
        g = _ladder(100)
        part = ((np.arange(200) % 100) >= 40).astype(np.int32)
        part[40] = 0
    elif case == "rgg":
        g = gen.rgg(1 << 13, 2, 6.0, 11, 1, 1)
        part = gen.rcb(g, 2, force_axis=0)
        gen.pair_swap_noise(g, part, 0.03, 11)
    else:
        g = _path(3000)
        part = (np.arange(3000) >= 1200).astype(np.int32)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=30000, mb_reps=6, mb_seed=5)
    c = gpu_lib.Context()
    try:
        c.set_tuning(mb_lds=0)
        _compare(gpu_lib, c, g, part, 2, 0, 1, p)
    finally:
        c.close()


def test_speculation_on_off(gpu_lib):
    g = gen.rgg(1 << 14, 2, 7.0, 21, 1, 1)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, 21)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
             eps_ppm=30000, mb_reps=8, mb_seed=3)
    for spec in (False, True):
        c = gpu_lib.Context()
        try:
            c.set_speculation(spec)
            _compare(gpu_lib, c, g, part, 2, 0, 1, p)
        finally:
            c.close()


@pytest.mark.parametrize("seed,n,k,dim,whi", [(61, 1 << 14, 8, 2, 1), (62, 1 << 15, 16, 3, 1),
                                              (63, 1 << 15, 16, 2, 10)])
def test_batch_round(gpu_lib, ctx, seed, n, k, dim, whi):
    import torch

    g = gen.rgg(n, dim, 8.0 if dim == 2 else 12.0, seed=seed, wlo=1, whi=whi)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.02, seed)
    edges, colour = oracle.quotient_colouring(g, part, k)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, mb_reps=16, mb_seed=seed)
    dg = gpu_lib.DeviceGraph.from_host(g)
    for c in sorted(set(colour.tolist()))[:2]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        print(f"mb batch n={n} k={k} colour={c} pairs={len(pairs)}", flush=True)
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

    g = gen.rgg(1 << 14, 2, 7.0, 71, 1, 1)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.02, 71)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, mb_reps=8, mb_seed=71)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=3)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 3)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


def test_rejects_too_many_sweeps(gpu_lib, ctx):
    g = _ladder(10)
    part = ((np.arange(20) % 10) >= 5).astype(np.int32)
    with pytest.raises(gpu_lib.FlowRefineError):
        gpu_lib.flow_refine_pair(ctx, g, part, 2, 0, 1, gpu_lib.params(mb_reps=257))


@pytest.mark.parametrize("seed", range(12))
def test_largest_source_side_candidates(gpu_lib, ctx, seed):
    """cut_side 1 (the largest minimum source side) and 2 (the largest only
    when the smallest is infeasible and it is feasible) against the oracle."""
    rng = np.random.default_rng(1500 + seed)
    if seed < 6:
        n = int(rng.integers(8, 50))
        g = random_graph(n, 0.2, 1500 + seed, wmax=3, vwmax=int(rng.choice([1, 4])))
        part = (rng.random(n) < 0.5).astype(np.int32)
        part[0], part[1] = 0, 1
    else:
        g = gen.rgg(1 << 13, 2, 7.0, 1500 + seed, 1, int(rng.choice([1, 5])))
        part = gen.rcb(g, 2, force_axis=0)
        gen.pair_swap_noise(g, part, 0.03, seed)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=int(rng.choice([30000, 300000])), cut_side=1 + seed % 2)
    _compare(gpu_lib, ctx, g, part, 2, 0, 1, p)


def test_largest_source_side_batch(gpu_lib, ctx):
    import torch

    g = gen.rgg(1 << 15, 2, 8.0, seed=64, wlo=1, whi=1)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.02, 64)
    edges, colour = oracle.quotient_colouring(g, part, 16)
    pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == 0]
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, cut_side=2)
    rc, ores, otr, opart = oracle.refine_batch(g, part, 16, pairs, p)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    res, trace = gpu_lib.flow_refine_batch(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                           pairs, _prm(gpu_lib, p))
    for i in range(len(pairs)):
        for key in RESULT_KEYS:
            assert res[i][key] == ores[i][key], (i, key)
        assert trace[i] == otr[i]
    assert np.array_equal(dpart.cpu().numpy(), opart)

"""Sliced rounds (fr_tuning.slice_us): a flow launch stops a solve at a due
global relabel once its time is used and at most a quarter of the launch's
solves still run; the solve continues in a later launch while the other
pairs move on.  With slices of 1 and 300 microseconds nearly every such
point ends a launch, so solves span many launches and pairs drift far
apart in their iterations.  Everything is compared with the oracle:
randomised rounds, matching rounds, FM before and multi-try after the
round, the learned start with its restart, and timed sweeps (the sweeps
that launch round by round).  The outputs are unique, so the bar is
bit-exact."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import random_graph
from tests.test_gpu_parity import RESULT_KEYS, _batch_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[1, 300])
def ctx(gpu_lib, request):
    c = gpu_lib.Context()
    c.set_tuning(slice_us=request.param)
    yield c
    c.close()


def _prm(fr, p):
    return fr.params(**{k: v for k, v in p.items() if k in dict(fr.FrParams._fields_)})


def _batch_vs_oracle(fr, ctx, g, part, k, pairs, p, keys=RESULT_KEYS):
    import torch

    print(f"sliced batch n={g.n} k={k} pairs={len(pairs)} {p} tuning {ctx.get_tuning()}",
          flush=True)
    rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr = fr.flow_refine_batch(ctx, fr.DeviceGraph.from_host(g), dpart, k, pairs, _prm(fr, p))
    for i in range(len(pairs)):
        for key in keys:
            assert res[i][key] == ores[i][key], (pairs[i], key, res[i][key], ores[i][key])
        assert tr[i] == otr[i], pairs[i]
    assert np.array_equal(dpart.cpu().numpy(), opart)
    return res, fr.stats_dict(ctx)


@pytest.mark.parametrize("seed", range(10))
def test_random_rounds(gpu_lib, ctx, seed):
    rng = np.random.default_rng(7000 + seed)
    if seed % 2:
        g = gen.rgg(int(rng.integers(3000, 12000)), 2, float(rng.choice([6.0, 8.0])),
                    seed=seed, wlo=1, whi=int(rng.choice([1, 10])))
    else:
        g = random_graph(int(rng.integers(60, 160)), 0.06, seed, wmax=5,
                         vwmax=2 if seed % 4 == 0 else 1)
    k = int(rng.choice([4, 8, 16]))
    part = gen.rcb(g, k) if g.coords is not None else rng.integers(0, k, g.n).astype(np.int32)
    amax = int(rng.choice([2, 6, 16]))
    p = dict(area_mode=0, depth=0, alpha=int(rng.integers(1, amax + 1)), alpha_max=amax,
             adaptive=1, max_iters=int(rng.choice([2, 3, 16])),
             eps_ppm=int(rng.choice([0, 10000, 30000, 100000])),
             terminals=int(seed % 3 == 1), cut_side=int(seed % 5 == 2) * 2)
    edges, colour = oracle.quotient_colouring(g, part, k)
    if len(edges) == 0:
        pytest.skip("no adjacent blocks")
    cls = int(np.argmax(np.bincount(colour)))
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == cls]
    _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)


@pytest.mark.parametrize("seed,n,k,dim", [(41, 1 << 15, 8, 2), (42, 1 << 15, 16, 3)])
def test_matching_rounds(gpu_lib, ctx, seed, n, k, dim):
    """Rounds whose solves are long enough to span launches (with 1 us
    slices some do)."""
    g, part = _batch_case(seed, n, k, dim=dim, deg=8.0 if dim == 2 else 12.0)
    edges, colour = oracle.quotient_colouring(g, part, k)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    slices = []
    for c in sorted(set(colour.tolist()))[:2]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        _, st = _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)
        slices.append(st["slices"])
    if ctx.get_tuning()["slice_us"] == 1:
        assert max(slices) > 0, slices


def test_round_with_fm_and_multitry(gpu_lib, ctx):
    g, part = _batch_case(78, 6000, 8, frac=0.04)
    edges, colour = oracle.quotient_colouring(g, part, 8)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6, eps_ppm=30000,
             fm_limit=20, fm_seed=5, mt_alpha=10, mt_seed=2)
    res, _ = _batch_vs_oracle(gpu_lib, ctx, g, part, 8, pairs, p, RESULT_KEYS + ("mt_kept",))
    assert sum(r["mt_kept"] for r in res) > 0


def test_learned_start(gpu_lib, ctx):
    import torch

    gpu_lib.load_trained_mlp(ctx)
    g, part = _batch_case(92, 1 << 14, 16, frac=0.02)
    edges, colour = oracle.quotient_colouring(g, part, 16)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr = gpu_lib.flow_refine_batch(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16, pairs,
                                        _prm(gpu_lib, dict(p, use_mlp=1)))
    cur = part.copy()
    for i, (a, b) in enumerate(pairs):
        o = oracle.refine_pair(g, part, 16, a, b,
                               dict(p, alpha=res[i]["start_alpha"], restart_alpha=16))
        for key in RESULT_KEYS:
            assert res[i][key] == o.result[key], ((a, b), key)
        assert tr[i] == o.trace
        mine = (part == a) | (part == b)
        cur[mine] = o.part[mine]
    assert np.array_equal(dpart.cpu().numpy(), cur)


@pytest.mark.parametrize("active", [0, 1])
def test_timed_sweep(gpu_lib, ctx, active):
    """Sweeps with per-phase timing launch their rounds one by one, so they
    run sliced (captured sweeps cannot)."""
    import torch

    g, part = _batch_case(53 + active, 1 << 14, 16, frac=0.02)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, active_blocks=active, fm_limit=20 * active, fm_seed=3)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=4)
    assert rc == 0
    ctx.set_timing(True)
    try:
        dpart = torch.as_tensor(part.copy()).cuda()
        tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart,
                                                   16, _prm(gpu_lib, p), 4)
    finally:
        ctx.set_timing(False)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)

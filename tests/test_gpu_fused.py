"""The fused round kernel (fr_set_fused 1: each workgroup runs one pair's
whole adaptive loop in one launch) against the oracle: randomised rounds,
matching rounds, a round at the pair limit, sweeps with and without active
blocks, the options it runs with (contracted terminals, the largest minimum
source side, FM before the flow, multi-try FM after the round, the learned
start), the pair call with its side codes, and the entry point without
device allocation.  The outputs compared are unique, so the bar is
bit-exact."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import random_graph
from tests.test_gpu_parity import RESULT_KEYS, _batch_case, _compare_pair, _pair_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    c.set_fused(True)
    yield c
    c.close()


def _prm(fr, p):
    return fr.params(**{k: v for k, v in p.items() if k in dict(fr.FrParams._fields_)})


def _batch_vs_oracle(fr, ctx, g, part, k, pairs, p, keys=RESULT_KEYS):
    import torch

    print(f"fused batch n={g.n} k={k} pairs={len(pairs)} {p}", flush=True)
    rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr = fr.flow_refine_batch(ctx, fr.DeviceGraph.from_host(g), dpart, k, pairs, _prm(fr, p))
    for i in range(len(pairs)):
        for key in keys:
            assert res[i][key] == ores[i][key], (pairs[i], key, res[i][key], ores[i][key])
        assert tr[i] == otr[i], pairs[i]
    assert np.array_equal(dpart.cpu().numpy(), opart)
    st = fr.stats_dict(ctx)
    assert st["slots"] == 1 and st["flow_launches"] == 1  # one entry per pair, one launch
    return res


@pytest.mark.parametrize("seed", range(16))
def test_random_rounds(gpu_lib, ctx, seed):
    """Randomised rounds as in the launch-chain tests: RGG or random graphs,
    k in 4..16, factor caps that need not be powers of two, iteration caps
    1..16, eps 0..10 %, optionally contracted terminals or the largest
    minimum source side."""
    rng = np.random.default_rng(5000 + seed)
    if seed % 2:
        g = gen.rgg(int(rng.integers(2000, 12000)), 2, float(rng.choice([6.0, 8.0])),
                    seed=seed, wlo=1, whi=int(rng.choice([1, 10])))
    else:
        g = random_graph(int(rng.integers(60, 160)), 0.06, seed, wmax=5,
                         vwmax=2 if seed % 4 == 0 else 1)
    k = int(rng.choice([4, 8, 16]))
    part = gen.rcb(g, k) if g.coords is not None else rng.integers(0, k, g.n).astype(np.int32)
    amax = int(rng.choice([1, 2, 6, 12, 16]))
    p = dict(area_mode=0, depth=0, alpha=int(rng.integers(1, amax + 1)), alpha_max=amax,
             adaptive=int(rng.random() < 0.85), max_iters=int(rng.choice([1, 2, 3, 16])),
             eps_ppm=int(rng.choice([0, 10000, 30000, 100000])),
             terminals=int(seed % 3 == 1), cut_side=int(seed % 5 == 2) * 2)
    edges, colour = oracle.quotient_colouring(g, part, k)
    if len(edges) == 0:
        pytest.skip("no adjacent blocks")
    cls = int(rng.integers(0, colour.max() + 1))
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == cls]
    _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)


@pytest.mark.parametrize("seed,n,k,dim", [(31, 1 << 14, 8, 2), (32, 1 << 15, 16, 3)])
def test_matching_rounds(gpu_lib, ctx, seed, n, k, dim):
    g, part = _batch_case(seed, n, k, dim=dim, deg=8.0 if dim == 2 else 12.0)
    edges, colour = oracle.quotient_colouring(g, part, k)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    for c in sorted(set(colour.tolist()))[:2]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)


def test_pair_limit(gpu_lib, ctx):
    """4096 pairs of 2x2-vertex blocks in one launch (more pairs than
    workgroups: the queue hands them out)."""
    g, part, k, pairs = _pair_grid()
    p = dict(area_mode=0, depth=0, alpha=4, alpha_max=8, adaptive=1, max_iters=4, eps_ppm=300000)
    _batch_vs_oracle(gpu_lib, ctx, g, part, k, pairs, p)


def test_pair_with_side_codes(gpu_lib, ctx):
    w = gen.config("C2", seed=9, n_override=1 << 14)
    _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params)


@pytest.mark.parametrize("active", [0, 1])
def test_sweep(gpu_lib, ctx, active):
    import torch

    g, part = _batch_case(51 + active, 1 << 14, 16, frac=0.02)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, active_blocks=active, fm_limit=20 * active, fm_seed=3)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=4)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 4)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


def test_round_with_fm_and_multitry(gpu_lib, ctx):
    g, part = _batch_case(77, 6000, 8, frac=0.04)
    edges, colour = oracle.quotient_colouring(g, part, 8)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6, eps_ppm=30000,
             fm_limit=20, fm_seed=5, mt_alpha=10, mt_seed=2)
    res = _batch_vs_oracle(gpu_lib, ctx, g, part, 8, pairs, p, RESULT_KEYS + ("mt_kept",))
    assert sum(r["mt_kept"] for r in res) > 0


def test_learned_start(gpu_lib, ctx):
    """With the shipped network the start factor is the network's; the
    oracle started at the same factors gives the same results."""
    import torch

    gpu_lib.load_trained_mlp(ctx)
    g, part = _batch_case(91, 1 << 14, 16, frac=0.02)
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


def test_static_entry_point(gpu_lib, ctx):
    """The entry point without device allocation runs the fused kernel too."""
    import torch

    w = gen.config("C2", seed=4, n_override=1 << 13)
    o = oracle.refine_pair(w.graph, w.part, 2, 0, 1, w.params)
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part.copy()).cuda()
    res, tr = gpu_lib.flow_refine_pair_static(ctx, dg, dpart, 2, 0, 1, _prm(gpu_lib, w.params))
    for key in RESULT_KEYS:
        assert res[key] == o.result[key], key
    assert tr == o.trace
    assert np.array_equal(dpart.cpu().numpy(), o.part)

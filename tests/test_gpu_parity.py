"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same seeded inputs.  Every compared output is unique
(flow value, smallest source set, partition, cut, block weights, factor
sequence), so the bar is bit-exact."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import random_graph

pytestmark = pytest.mark.gpu

RESULT_KEYS = ("status", "iters", "final_alpha", "applied", "iter_cap", "flow_value",
               "cut_before", "cut_after", "weight_a", "weight_b", "region_vertices",
               "region_edges")


def _prm(fr, d):
    return fr.params(**{k: d[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                          "max_iters", "eps_ppm")})


def _gpu_pair(fr, ctx, g, part, k, a, b, p, device_graph=True):
    import torch

    if device_graph:
        dg = fr.DeviceGraph.from_host(g)
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace, side = fr.flow_refine_pair(ctx, dg, dpart, k, a, b, _prm(fr, p), want_side=True)
        return res, trace, side, dpart.cpu().numpy()
    hp = part.copy()
    res, trace, side = fr.flow_refine_pair(ctx, g, hp, k, a, b, _prm(fr, p), want_side=True)
    return res, trace, side, hp


def _compare_pair(fr, ctx, g, part, k, a, b, p, device_graph=True):
    print(f"case n={g.n} arcs={g.narcs} k={k} pair=({a},{b}) params={p}", flush=True)
    o = oracle.refine_pair(g, part, k, a, b, p)
    assert o.rc == 0
    res, trace, side, newpart = _gpu_pair(fr, ctx, g, part, k, a, b, p, device_graph)
    for key in RESULT_KEYS:
        assert res[key] == o.result[key], (key, res[key], o.result[key])
    assert len(trace) == len(o.trace)
    for t_gpu, t_or in zip(trace, o.trace):
        assert t_gpu == t_or, (t_gpu, t_or)
    assert np.array_equal(side, o.side)
    assert np.array_equal(newpart, o.part)
    return res, trace


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def test_c1_depth_corridor(gpu_lib, ctx):
    w = gen.config("C1")
    res, trace = _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params)
    assert res["flow_value"] == 128 and res["status"] == gpu_lib.FR_REJECTED_IMBALANCE


def test_c1b_factor_corridor(gpu_lib, ctx):
    w = gen.config("C1B")
    res, _ = _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params)
    assert res["status"] == gpu_lib.FR_ACCEPTED


def test_c1_host_pointers(gpu_lib, ctx):
    w = gen.config("C1B")
    _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params, device_graph=False)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_random(gpu_lib, ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 40))
    g = random_graph(n, 0.25, seed, wmax=6, vwmax=3 if seed % 3 == 0 else 1)
    part = (rng.random(n) < 0.5).astype(np.int32)
    if part.min() == part.max():
        part[0] = 1 - part[0]
    al = int(rng.choice([1, 2, 4, 8, 16]))
    p = dict(area_mode=0, depth=0, alpha=al, alpha_max=al, adaptive=0, max_iters=1,
             eps_ppm=int(rng.choice([30000, 100000, 300000])))
    if seed % 4 == 0:
        p = dict(p, area_mode=1, depth=int(rng.integers(0, 3)))
    _compare_pair(gpu_lib, ctx, g, part, 2, 0, 1, p)


@pytest.mark.parametrize("n,seed", [(1 << 12, 3), (1 << 14, 4), (1 << 15, 5)])
def test_rgg_adaptive(gpu_lib, ctx, n, seed):
    w = gen.config("C2", seed=seed, n_override=n)
    _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params)


def test_c2_full(gpu_lib, ctx):
    """2D RGG n=2^18, weights 1..10, alpha 16 adaptive, at full size."""
    w = gen.config("C2")
    _compare_pair(gpu_lib, ctx, w.graph, w.part, 2, 0, 1, w.params)


def test_reversed_orientation_and_kway(gpu_lib, ctx):
    g = gen.rgg(6000, 2, 8.0, seed=17, wlo=1, whi=10)
    part = gen.rcb(g, 8)
    gen.global_noise(g, part, 0.03, 17)
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=16, adaptive=1, max_iters=8, eps_ppm=30000)
    _compare_pair(gpu_lib, ctx, g, part, 8, 3, 2, p)
    _compare_pair(gpu_lib, ctx, g, part, 8, 0, 1, p)


def test_zero_weight_vertices(gpu_lib, ctx):
    g = gen.rgg(3000, 2, 7.0, seed=77, wlo=1, whi=5)
    g.vwgt = (np.arange(g.n) % 3).astype(np.int32)
    part = gen.rcb(g, 2)
    for p in (dict(area_mode=1, depth=3, alpha=1, alpha_max=1, adaptive=0, max_iters=1, eps_ppm=30000),
              dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6, eps_ppm=30000)):
        _compare_pair(gpu_lib, ctx, g, part, 2, 0, 1, p)


def test_not_adjacent(gpu_lib, ctx):
    from tests.helpers import csr_from_edges
    g = csr_from_edges(6, [(0, 1), (1, 2), (3, 4), (4, 5)])
    part = np.array([0, 0, 1, 2, 2, 3], dtype=np.int32)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1, eps_ppm=30000)
    res, _ = _compare_pair(gpu_lib, ctx, g, part, 4, 0, 2, p)
    assert res["status"] == gpu_lib.FR_NOT_ADJACENT


def test_empty_corridor_side(gpu_lib, ctx):
    """eps = 0 on a perfectly balanced bisection: both area bounds are 0."""
    g = gen.rgg(4000, 2, 8.0, seed=8)
    part = gen.rcb(g, 2)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1, eps_ppm=0)
    res, trace = _compare_pair(gpu_lib, ctx, g, part, 2, 0, 1, p)
    assert trace[0]["region_vertices"] == 0


def _batch_case(seed, n, k, frac=0.02, dim=2, deg=8.0):
    g = gen.rgg(n, dim, deg, seed=seed, wlo=1, whi=10)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, frac, seed)
    return g, part


@pytest.mark.parametrize("seed,n,k,dim", [(31, 1 << 14, 8, 2), (32, 1 << 15, 16, 3),
                                          (33, 1 << 16, 32, 2)])
def test_batch_matching_round(gpu_lib, ctx, seed, n, k, dim):
    import torch

    g, part = _batch_case(seed, n, k, dim=dim, deg=8.0 if dim == 2 else 12.0)
    edges, colour = oracle.quotient_colouring(g, part, k)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    dg = gpu_lib.DeviceGraph.from_host(g)
    for c in sorted(set(colour.tolist()))[:3]:
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == c]
        print(f"batch n={n} k={k} colour={c} pairs={len(pairs)}", flush=True)
        rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
        assert rc == 0
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, _prm(gpu_lib, p))
        for i in range(len(pairs)):
            for key in RESULT_KEYS:
                assert res[i][key] == ores[i][key], (i, key)
            assert trace[i] == otr[i]
        assert np.array_equal(dpart.cpu().numpy(), opart)


def test_quotient_matchings(gpu_lib, ctx):
    g, part = _batch_case(41, 1 << 14, 16)
    e_gpu, c_gpu = gpu_lib.fr_quotient_matchings(ctx, gpu_lib.DeviceGraph.from_host(g),
                                                 __import__("torch").as_tensor(part).cuda(), 16)
    e_or, c_or = oracle.quotient_colouring(g, part, 16)
    assert np.array_equal(e_gpu, e_or) and np.array_equal(c_gpu, c_or)


def test_sweep_matches_oracle(gpu_lib, ctx):
    import torch

    g, part = _batch_case(51, 1 << 14, 16, frac=0.02)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16, eps_ppm=30000)
    rc, tc, stats, opart = oracle.sweep(g, part, 16, p, max_sweeps=4)
    assert rc == 0
    dpart = torch.as_tensor(part.copy()).cuda()
    tc_gpu, st_gpu = gpu_lib.flow_refine_sweep(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 16,
                                               _prm(gpu_lib, p), 4)
    assert tc_gpu == tc
    assert st_gpu.tolist() == stats.tolist()
    assert np.array_equal(dpart.cpu().numpy(), opart)


@pytest.mark.parametrize("tune", [dict(block_threads=256, blocks_per_cu=1, tpv=1, relabel_period=1),
                                  dict(block_threads=1024, blocks_per_cu=2, tpv=16, relabel_period=50),
                                  dict(block_threads=512, blocks_per_cu=4, tpv=4, relabel_period=3),
                                  dict(block_threads=256, blocks_per_cu=8, tpv=2, relabel_period=12)])
def test_launch_parameters_do_not_change_results(gpu_lib, tune):
    c = gpu_lib.Context()
    try:
        c.set_tuning(**tune)
        w = gen.config("C2", seed=9, n_override=1 << 14)
        _compare_pair(gpu_lib, c, w.graph, w.part, 2, 0, 1, w.params)
    finally:
        c.close()


def test_error_paths(gpu_lib, ctx):
    import torch

    w = gen.config("C1B")
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    prm = _prm(gpu_lib, w.params)
    dpart = torch.as_tensor(w.part.copy()).cuda()
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 0, prm)
    assert e.value.code == -3
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_batch(ctx, dg, dpart, 4, [(0, 1), (1, 2)], prm)
    assert e.value.code == -4
    bad = dpart.clone()
    bad[5] = 7
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, dg, bad, 2, 0, 1, prm)
    assert e.value.code == -2
    assert torch.equal(bad.cpu()[:5], dpart.cpu()[:5])
    g2 = gen.grid2d(8, 8)
    g2.adjwgt = g2.adjwgt.copy()
    g2.adjwgt[3] = 2  # asymmetric weight
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, gpu_lib.DeviceGraph.from_host(g2),
                                 torch.zeros(64, dtype=torch.int32).cuda(), 2, 0, 1, prm)
    assert e.value.code == -1
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 1, gpu_lib.params(max_iters=0))
    assert e.value.code == -8
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        ctx.set_tuning(blocks_per_cu=9)
    assert e.value.code == -8


@pytest.mark.parametrize("spec,fused", [(True, False), (False, False), (True, True)])
def test_speculation_on_off_match_oracle(gpu_lib, spec, fused):
    """The adaptive loop with every factor of the halving chain solved at once
    (speculation, launch chains per iteration), one solve per launch, and the
    fused round kernel (one solve at a time inside one launch) give the
    oracle's trace, result and partition; with speculation the C2 pair runs
    its 5 factors side by side."""
    import torch

    w = gen.config("C2", n_override=1 << 16)
    o = oracle.refine_pair(w.graph, w.part, 2, 0, 1, w.params, want_side=True)
    ctx = gpu_lib.Context()
    try:
        ctx.set_speculation(spec)
        ctx.set_fused(fused)
        spec = spec and not fused
        dg = gpu_lib.DeviceGraph.from_host(w.graph)
        dpart = torch.as_tensor(w.part.copy()).cuda()
        res, trace, side = gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 1,
                                                    gpu_lib.params(**w.params), want_side=True)
        assert gpu_lib.stats_dict(ctx)["slots"] == (5 if spec else 1)
        for key in RESULT_KEYS:
            assert res[key] == o.result[key], key
        assert trace == o.trace
        assert np.array_equal(side, o.side)
        assert np.array_equal(dpart.cpu().numpy(), o.part)
    finally:
        ctx.close()


@pytest.mark.parametrize("seed", range(24))
def test_random_batches_vs_oracle(gpu_lib, ctx, seed):
    """Randomised whole rounds: RGG or random graphs, k in 4..16, a factor cap
    that may not be a power of two, iteration caps 1..16, eps 0..10 %; the
    batched call (speculative factor chains on) against the oracle pair by
    pair."""
    import torch

    rng = np.random.default_rng(1000 + seed)
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
             eps_ppm=int(rng.choice([0, 10000, 30000, 100000])))
    edges, colour = oracle.quotient_colouring(g, part, k)
    if len(edges) == 0:
        pytest.skip("no adjacent blocks")
    cls = int(rng.integers(0, colour.max() + 1))
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == cls]
    dg = gpu_lib.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, gpu_lib.params(**p))
    cur = part.copy()
    for i, (a, b) in enumerate(pairs):
        o = oracle.refine_pair(g, cur, k, a, b, p, want_side=False)
        for key in RESULT_KEYS:
            assert res[i][key] == o.result[key], (seed, (a, b), key, p)
        assert trace[i] == o.trace, (seed, (a, b))
        cur = o.part
    assert np.array_equal(dpart.cpu().numpy(), cur)


def _pair_grid(width=256, height=128, seed=5):
    """A weighted grid cut into 2x2-vertex blocks; pairs (2i, 2i+1) are
    horizontal neighbours: 8192 blocks, 4096 disjoint adjacent pairs."""
    from tests.helpers import csr_from_edges

    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for y in range(height):
        for x in range(width):
            v = y * width + x
            if x + 1 < width:
                edges.append((v, v + 1))
                ws.append(int(rng.integers(1, 6)))
            if y + 1 < height:
                edges.append((v, v + width))
                ws.append(int(rng.integers(1, 6)))
    g = csr_from_edges(width * height, edges, ws)
    xs, ys = np.arange(g.n) % width, np.arange(g.n) // width
    part = ((ys // 2) * (width // 2) + xs // 2).astype(np.int32)
    k = (width // 2) * (height // 2)
    pairs = [(2 * i, 2 * i + 1) for i in range(k // 2)]
    for a, b in pairs[::3]:  # move one vertex of every third pair across
        part[np.where(part == a)[0][0]] = b
    return g, part, k, pairs


def test_batch_at_the_pair_limit(gpu_lib, ctx):
    """4096 pairs in one call (the per-round maximum) against the oracle;
    one more pair is rejected without touching the partition."""
    import torch

    g, part, k, pairs = _pair_grid()
    p = dict(area_mode=0, depth=0, alpha=4, alpha_max=8, adaptive=1, max_iters=4,
             eps_ppm=300000)
    dg = gpu_lib.DeviceGraph.from_host(g)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, k, pairs, gpu_lib.params(**p))
    rc, ores, otr, opart = oracle.refine_batch(g, part, k, pairs, p)
    assert rc == 0 and len(res) == 4096
    for i in range(len(pairs)):
        for key in RESULT_KEYS:
            assert res[i][key] == ores[i][key], (i, key)
        assert trace[i] == otr[i]
    assert np.array_equal(dpart.cpu().numpy(), opart)
    too_many = pairs + [(k - 1, k - 2)]
    dpart2 = torch.as_tensor(part.copy()).cuda()
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        gpu_lib.flow_refine_batch(ctx, dg, dpart2, k, too_many, gpu_lib.params(**p))
    assert e.value.code == -8
    assert np.array_equal(dpart2.cpu().numpy(), part)


@pytest.mark.parametrize("spec", [False, True])
def test_boundary_pass_modes(gpu_lib, spec):
    """The boundary pass walks all vertices once (results handed to every
    live slot) while the live pairs cover at least a quarter of the graph, and
    the live pairs' vertex lists otherwise: one pair of a 64-way partition
    without speculation takes the lists, a whole matching round the vertex
    walk (and the lists once most pairs stopped); both against the oracle.
    The pass's work counters count each live pair's vertices and arcs of its
    two blocks once per launch: for one pair, arcs over vertices is exactly
    that pair's ratio; for the round, it lies within the degree range."""
    import torch

    def counters_ok(c, g, part, pairs):
        st = gpu_lib.stats_dict(c)
        deg = np.diff(g.xadj)
        nv, na = st["bnd_verts"], st["bnd_arcs"]
        assert nv > 0 and na > 0
        if len(pairs) == 1:
            mine = np.isin(part, pairs[0])
            assert na * int(mine.sum()) == nv * int(deg[mine].sum())
        else:
            assert nv * int(deg.min()) <= na <= nv * int(deg.max())

    g = gen.rgg(1 << 14, 2, 8.0, 57, 1, 4)
    part = gen.rcb(g, 64)
    gen.global_noise(g, part, 0.02, 57)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000)
    edges, colour = oracle.quotient_colouring(g, part, 64)
    c = gpu_lib.Context()
    try:
        c.set_speculation(spec)
        c.set_fused(False)  # the boundary pass of the launch chains
        a, b = (int(x) for x in edges[0])
        _compare_pair(gpu_lib, c, g, part, 64, a, b, p)
        counters_ok(c, g, part, [(a, b)])
        # the 64 blocks merged into two halves: the pair covers the graph, so
        # every pass walks all vertices
        part2 = (part >= 32).astype(np.int32)
        _compare_pair(gpu_lib, c, g, part2, 2, 0, 1, p)
        counters_ok(c, g, part2, [(0, 1)])
        cls = int(np.argmax(np.bincount(colour)))
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour) if cc == cls]
        print(f"round of {len(pairs)} pairs, speculation {spec}", flush=True)
        rc, ores, otr, opart = oracle.refine_batch(g, part, 64, pairs, p)
        assert rc == 0
        dpart = torch.as_tensor(part.copy()).cuda()
        res, trace = gpu_lib.flow_refine_batch(c, gpu_lib.DeviceGraph.from_host(g), dpart, 64,
                                               pairs, _prm(gpu_lib, p))
        for i in range(len(pairs)):
            for key in RESULT_KEYS:
                assert res[i][key] == ores[i][key], (i, key)
            assert trace[i] == otr[i]
        assert np.array_equal(dpart.cpu().numpy(), opart)
        counters_ok(c, g, part, pairs)
    finally:
        c.close()

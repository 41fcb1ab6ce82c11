"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (validation off, default tuning).

The pairs of one matching touch disjoint blocks, hence a pair's batched
result equals the oracle's result for that pair alone on the round's start
partition.  The largest rounds of C3 and C5 on the default path are checked
pair by pair for every pair, with the oracle spread over a thread pool; one
C5 sweep is checked against the sweep restated over the oracle's colouring
and per-class pair refinements.  The option variants check sampled pairs."""
import functools
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

# the workloads are read-only in these tests: generate each once per module
_config = functools.lru_cache(maxsize=4)(gen.config)

KEYS = ("status", "iters", "final_alpha", "applied", "iter_cap", "flow_value", "cut_before",
        "cut_after", "weight_a", "weight_b", "region_vertices", "region_edges")


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    c.set_validation(False)
    yield c
    c.close()


def _round_vs_oracle(gpu_lib, ctx, w, sample, use_mlp=0, extra=None):
    import torch

    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges, colour = gpu_lib.fr_quotient_matchings(ctx, dg, part0, w.k)
    cls = int(np.argmax(np.bincount(colour)))
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == cls]
    dpart = part0.clone()
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                  "max_iters", "eps_ppm")}
    p.update(extra or {})
    res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, w.k, pairs,
                                           gpu_lib.params(**p, use_mlp=use_mlp))
    out = dpart.cpu().numpy()
    # the largest pair (most corridor edges) and a few others
    order = sorted(range(len(pairs)), key=lambda i: -res[i]["region_edges"])
    picks = order[:1] + order[1:][:: max(1, (len(order) - 1) // max(1, sample - 1))][: sample - 1]
    for i in picks:
        a, b = pairs[i]
        q = dict(p, alpha=res[i]["start_alpha"], restart_alpha=p["alpha"]) if use_mlp else p
        o = oracle.refine_pair(w.graph, w.part, w.k, a, b, q, want_side=False)
        for key in KEYS:
            assert res[i][key] == o.result[key], (w.name, (a, b), key)
        assert trace[i] == o.trace
        mine = (w.part == a) | (w.part == b)
        assert np.array_equal(out[mine], o.part[mine]), (w.name, (a, b))
    # vertices of blocks outside the round never move
    inround = np.isin(w.part, np.asarray(pairs).reshape(-1))
    assert np.array_equal(out[~inround], w.part[~inround])
    return res


def _pool():
    return ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))


def _oracle_pairs(w, part, pairs, p):
    """The oracle's refinement of every pair of one matching, each on the
    same start partition, over a thread pool (the C code releases the GIL)."""
    with _pool() as ex:
        return list(ex.map(lambda ab: oracle.refine_pair(w.graph, part, w.k, ab[0], ab[1], p,
                                                         want_side=False), pairs))


def _merge(part, pairs, outs):
    """The round's partition: each pair's blocks take that pair's result."""
    new = part.copy()
    for (a, b), o in zip(pairs, outs):
        mine = (part == a) | (part == b)
        new[mine] = o.part[mine]
    return new


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_largest_round_every_pair(gpu_lib, ctx, cid):
    """The largest round of C3 (8 pairs) and of C5 (128 pairs) on the default
    path (pinned border, smallest source set, alpha' = 16 adaptive), as the
    benchmark times it, with the fused round kernel and with the per-iteration
    launch chains: every pair's result record and trace, and the whole
    partition, equal the oracle's."""
    import torch

    w = _config(cid)
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges, colour = gpu_lib.fr_quotient_matchings(ctx, dg, part0, w.k)
    cls = int(np.argmax(np.bincount(colour)))
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == cls]
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                  "max_iters", "eps_ppm")}
    outs = _oracle_pairs(w, w.part, pairs, p)
    merged = _merge(w.part, pairs, outs)
    try:
        for fused in (True, False):
            print(f"{cid} largest round, {len(pairs)} pairs, every pair, "
                  f"{'fused round kernel' if fused else 'launch chains'}", flush=True)
            ctx.set_fused(fused)
            dpart = part0.clone()
            res, trace = gpu_lib.flow_refine_batch(ctx, dg, dpart, w.k, pairs, gpu_lib.params(**p))
            out = dpart.cpu().numpy()
            for i, ((a, b), o) in enumerate(zip(pairs, outs)):
                assert o.rc == 0
                for key in KEYS:
                    assert res[i][key] == o.result[key], (cid, fused, (a, b), key, res[i][key],
                                                          o.result[key])
                assert trace[i] == o.trace, (cid, fused, (a, b))
            assert np.array_equal(out, merged)
            assert sum(r["applied"] > 0 for r in res) > 0
    finally:
        ctx.set_fused(False)


def test_c5_sweep_every_pair(gpu_lib, ctx):
    """One sweep of C5 (every colour class in colour order, alpha' = 16
    adaptive, no learned start), against the sweep written out over the
    oracle: its quotient colouring, then class by class every pair refined
    on the class's start partition and the results merged.  Partition, total
    cut, solves, changed pairs and region edges must be equal."""
    import torch

    w = _config("C5")
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                  "max_iters", "eps_ppm")}
    print("C5 one sweep vs the oracle, class by class", flush=True)
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part).cuda()
    cut, stats = gpu_lib.flow_refine_sweep(ctx, dg, dpart, w.k, gpu_lib.params(**p), 1)
    got = dpart.cpu().numpy()
    part = w.part.copy()
    edges, colour = oracle.quotient_colouring(w.graph, part, w.k)
    solves = changed = region_edges = 0
    for c in sorted(set(colour.tolist())):
        pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour.tolist()) if cc == c]
        outs = _oracle_pairs(w, part, pairs, p)
        for o in outs:
            assert o.rc == 0
            solves += o.result["iters"]
            region_edges += o.result["region_edges"]
            changed += o.result["status"] == oracle.ST_ACCEPTED
        part = _merge(part, pairs, outs)
        print(f"  class {c}: {len(pairs)} pairs", flush=True)
    assert np.array_equal(got, part)
    assert cut == oracle.total_cut(w.graph, part)
    assert stats[0] == 1 and stats[1] == solves and stats[2] == changed
    assert stats[3] == region_edges


def test_c3_largest_round_sampled(gpu_lib, ctx):
    w = _config("C3")
    print("C3 largest round", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3)


def test_c4_round_with_learned_factor_sampled(gpu_lib, ctx):
    w = _config("C4")
    gpu_lib.load_trained_mlp(ctx)
    print("C4 largest round, learned start factor", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, use_mlp=1)


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_most_balanced_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with balanced adaptive flow iterations
    (16 sweeps), as the benchmark runs it."""
    w = _config(cid)
    print(f"{cid} largest round, most balanced cuts", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(mb_reps=16, mb_seed=1))


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_fm_then_most_balanced_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with 2-way FM before the flow and most
    balanced cuts, as the benchmark's quality leg runs it."""
    w = _config(cid)
    print(f"{cid} largest round, FM then most balanced cuts", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3,
                     extra=dict(fm_limit=100, fm_seed=1, mb_reps=16, mb_seed=1))


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_fm_then_flow_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with 2-way FM before the plain flow, as
    the benchmark's quality leg runs it."""
    w = _config(cid)
    print(f"{cid} largest round, FM then flow", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(fm_limit=100, fm_seed=1))


@pytest.mark.parametrize("cid", ["C2", "C3", "C5"])
def test_round_contracted_terminals_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 (C2: its one pair) with the blocks'
    outside parts contracted into s and t, as the benchmark's quality leg
    runs it."""
    w = _config(cid)
    print(f"{cid} largest round, contracted terminals", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(terminals=1))


def test_c5_sweep_properties(gpu_lib, ctx):
    """One full sweep of C5 (every colour class, learned start): the reported
    cut is the cut of the returned partition, it does not grow, and blocks
    that were balanced stay balanced (only feasible candidates are applied)."""
    import torch

    w = _config("C5")
    print("C5 one sweep", flush=True)
    gpu_lib.load_trained_mlp(ctx)
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part).cuda()
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                  "max_iters", "eps_ppm")}
    cut, stats = gpu_lib.flow_refine_sweep(ctx, dg, dpart, w.k, gpu_lib.params(**p, use_mlp=1),
                                           1)
    out = dpart.cpu().numpy()
    cut0 = oracle.total_cut(w.graph, w.part)
    assert cut == oracle.total_cut(w.graph, out)
    assert cut <= cut0 and stats[0] == 1 and stats[1] > 0
    assert (cut < cut0) == (stats[2] > 0)
    lmax = (1_000_000 + w.params["eps_ppm"]) * int(w.graph.vwgt.sum()) // (1_000_000 * w.k) + \
        int(w.graph.vwgt.max())
    bw0 = np.bincount(w.part, weights=w.graph.vwgt, minlength=w.k)
    bw1 = np.bincount(out, weights=w.graph.vwgt, minlength=w.k)
    assert np.all(bw1[bw0 <= lmax] <= lmax)
    assert out.min() >= 0 and out.max() < w.k


def test_corridor_beyond_lds_bitmaps(gpu_lib, ctx):
    """A corridor of more than 131,072 vertices (2D RGG n=2^19, alpha 16):
    the flow phases run on the global label and mark arrays instead of the
    LDS bitmaps; flow, smallest source side and decision still match."""
    import torch

    w = _config("C2", n_override=1 << 19)
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "eps_ppm")}
    p.update(adaptive=0, max_iters=1)
    o = oracle.refine_pair(w.graph, w.part, 2, 0, 1, p, want_side=True)
    assert o.result["region_vertices"] > 131072
    dg = gpu_lib.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part.copy()).cuda()
    res, trace, side = gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 1, gpu_lib.params(**p),
                                                want_side=True)
    for key in KEYS:
        assert res[key] == o.result[key], key
    assert trace == o.trace
    assert np.array_equal(side, o.side)
    assert np.array_equal(dpart.cpu().numpy(), o.part)

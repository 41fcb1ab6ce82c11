"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (validation off, default tuning).

The oracle cannot refine whole rounds of these graphs in test time, so
sampled pairs are checked one by one: the pairs of one matching touch
disjoint blocks, hence a pair's batched result equals the oracle's result for
that pair alone on the round's start partition.  The full sweep of the
largest workload is checked through properties that hold at any size."""
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
        q = dict(p, alpha=res[i]["start_alpha"]) if use_mlp else p
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


def test_c3_largest_round_sampled(gpu_lib, ctx):
    w = gen.config("C3")
    print("C3 largest round", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3)


def test_c4_round_with_learned_factor_sampled(gpu_lib, ctx):
    w = gen.config("C4")
    gpu_lib.load_trained_mlp(ctx)
    print("C4 largest round, learned start factor", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, use_mlp=1)


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_most_balanced_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with balanced adaptive flow iterations
    (16 sweeps), as the benchmark runs it."""
    w = gen.config(cid)
    print(f"{cid} largest round, most balanced cuts", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(mb_reps=16, mb_seed=1))


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_fm_then_most_balanced_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with 2-way FM before the flow and most
    balanced cuts, as the benchmark's quality leg runs it."""
    w = gen.config(cid)
    print(f"{cid} largest round, FM then most balanced cuts", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3,
                     extra=dict(fm_limit=100, fm_seed=1, mb_reps=16, mb_seed=1))


@pytest.mark.parametrize("cid", ["C3", "C5"])
def test_round_fm_then_flow_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 with 2-way FM before the plain flow, as
    the benchmark's quality leg runs it."""
    w = gen.config(cid)
    print(f"{cid} largest round, FM then flow", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(fm_limit=100, fm_seed=1))


@pytest.mark.parametrize("cid", ["C2", "C3", "C5"])
def test_round_contracted_terminals_sampled(gpu_lib, ctx, cid):
    """The largest round of C3 / C5 (C2: its one pair) with the blocks'
    outside parts contracted into s and t, as the benchmark's quality leg
    runs it."""
    w = gen.config(cid)
    print(f"{cid} largest round, contracted terminals", flush=True)
    _round_vs_oracle(gpu_lib, ctx, w, sample=3, extra=dict(terminals=1))


def test_c5_sweep_properties(gpu_lib, ctx):
    """One full sweep of C5 (every colour class, learned start): the reported
    cut is the cut of the returned partition, it does not grow, and blocks
    that were balanced stay balanced (only feasible candidates are applied)."""
    import torch

    w = gen.config("C5")
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

    w = gen.config("C2", n_override=1 << 19)
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

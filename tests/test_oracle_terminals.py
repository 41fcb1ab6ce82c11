"""Pins of the oracle's contracted terminals (terminals = 1): instead of
pinning the corridor border to s and t with infinite arcs (Sec. 4.1), the
parts of blocks a and b outside the corridor are contracted into s and t, the
weights of the edges into them becoming arc capacities, so that every
corridor vertex may change sides.  A minimum s-t cut of that network is then
the best reassignment of the corridor vertices, which brute force finds with
no network at all: over all 2^|corridor| reassignments, the candidate cut must
be the smallest pair cut, the smallest source side the intersection of the
optimal reassignments (itself optimal), the largest their union, and the
flow value the smallest pair cut minus the a-b edges outside the corridor."""
import numpy as np
import pytest

import oracle
from tests.helpers import area_bound, corridor_by_sorting, csr_from_edges, random_graph


def _pair_cuts(g, part, a, b, verts):
    """Pair cut of every reassignment of verts (row r: verts[i] goes to a iff
    bit i of r is set); the rest of the partition stays."""
    nc = len(verts)
    x = ((np.arange(1 << nc)[:, None] >> np.arange(nc)[None, :]) & 1).astype(bool)
    col = {int(u): i for i, u in enumerate(verts)}
    cuts = np.zeros(1 << nc, dtype=np.int64)
    for u in range(g.n):
        for e in range(g.xadj[u], g.xadj[u + 1]):
            v = int(g.adjncy[e])
            if v <= u or part[u] not in (a, b) or part[v] not in (a, b):
                continue

            def in_a(z):
                return x[:, col[z]] if z in col else np.full(1 << nc, part[z] == a)

            cuts += np.where(in_a(u) != in_a(v), int(g.adjwgt[e]), 0)
    return x, cuts


def _outside_cut(g, part, a, b, corridor):
    """Weight of the a-b edges with no end in the corridor."""
    cs = set(int(u) for u in corridor)
    tot = 0
    for u in range(g.n):
        for e in range(g.xadj[u], g.xadj[u + 1]):
            v = int(g.adjncy[e])
            if u < v and {int(part[u]), int(part[v])} == {a, b} and u not in cs and v not in cs:
                tot += int(g.adjwgt[e])
    return tot


def test_hand_example_moves_a_pinned_border_vertex():
    # vertex 1 (block 0) hangs on block 1 by two edges of weight 5 and on
    # block 0 by one of weight 1; the boundary-only corridor {1, 2, 3} has
    # every vertex on its border: pinned, nothing can move (cut stays 10);
    # contracted, vertex 1 crosses over and the pair cut drops to 1
    g = csr_from_edges(5, [(0, 1), (1, 2), (1, 3), (2, 4), (3, 4)], weights=[1, 5, 5, 1, 1],
                       vwgt=[3, 1, 1, 1, 1])
    part = np.array([0, 0, 1, 1, 1], dtype=np.int32)
    p = dict(area_mode=1, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=30000)
    pinned = oracle.refine_pair(g, part, 2, 0, 1, p)
    assert pinned.trace[0]["flow"] == 10
    assert pinned.trace[0]["decision"] == oracle.DEC_EQUAL
    assert pinned.side.tolist() == [-1, 2, 3, 3, -1]
    contracted = oracle.refine_pair(g, part, 2, 0, 1, dict(p, terminals=1))
    t = contracted.trace[0]
    assert t["flow"] == 1 and t["cut_candidate"] == 1 and t["source_side"] == 0
    assert (t["wa"], t["wb"]) == (3, 4)  # L_max = floor(1.03 * 7 / 2) + 3 = 6
    assert t["decision"] == oracle.DEC_APPLY
    assert contracted.side.tolist() == [-1, 1, 1, 1, -1]
    assert contracted.part.tolist() == [0, 1, 1, 1, 1]
    assert contracted.result["cut_after"] == 1


@pytest.mark.parametrize("seed", range(30))
def test_min_cut_is_the_best_corridor_reassignment(seed):
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(8, 17))
    k = 3 if seed % 3 == 2 else 2
    g = random_graph(n, 0.3, 3000 + seed, wmax=int(rng.choice([1, 4, 9])),
                     vwmax=int(rng.choice([1, 3])))
    part = rng.integers(0, k, n).astype(np.int32)
    part[0], part[1] = 0, 1
    a, b = (0, 1) if seed % 2 == 0 else (1, 0)
    eps = int(rng.choice([30000, 300000, 1000000]))
    alpha = int(rng.choice([1, 2, 8]))
    p = dict(area_mode=0, depth=0, alpha=alpha, alpha_max=alpha, adaptive=0, max_iters=1,
             eps_ppm=eps, terminals=1)
    ua = area_bound(g, part, k, b, alpha, eps)
    ub = area_bound(g, part, k, a, alpha, eps)
    corridor = np.sort(np.concatenate([corridor_by_sorting(g, part, a, b, 0, 0, ua),
                                       corridor_by_sorting(g, part, b, a, 0, 0, ub)]))
    o = oracle.refine_pair(g, part, k, a, b, p)
    assert o.rc == 0
    t = o.trace[0]
    if t["decision"] == oracle.DEC_NOT_ADJ:
        return
    assert np.array_equal(np.nonzero(o.side >= 0)[0], corridor)
    assert set(o.side[corridor].tolist()) <= {0, 1}  # nothing pinned
    x, cuts = _pair_cuts(g, part, a, b, corridor)
    best = cuts.min()
    opt = x[cuts == best]
    inter, union = opt.all(axis=0), opt.any(axis=0)
    assert cuts[int((inter * (1 << np.arange(len(corridor)))).sum())] == best  # a lattice
    assert t["cut_candidate"] == best
    assert t["flow"] == best - _outside_cut(g, part, a, b, corridor)
    assert np.array_equal(o.side[corridor] == 0, inter)
    assert t["source_side"] == int(inter.sum())
    o1 = oracle.refine_pair(g, part, k, a, b, dict(p, cut_side=1))
    assert o1.trace[0]["cut_candidate"] == best
    assert np.array_equal(o1.side[corridor] == 0, union)
    # pinning only removes reassignments
    o0 = oracle.refine_pair(g, part, k, a, b, dict(p, terminals=0))
    assert o0.trace[0]["cut_candidate"] >= best
    assert o0.trace[0]["region_vertices"] == t["region_vertices"] == len(corridor)


@pytest.mark.parametrize("seed", range(6))
def test_applied_solve_takes_the_intersection(seed):
    """With a loose balance bound the first solve applies whenever it
    improves, and the partition becomes the smallest optimal reassignment."""
    rng = np.random.default_rng(4000 + seed)
    n = 14
    g = random_graph(n, 0.35, 4000 + seed, wmax=5)
    part = (rng.random(n) < 0.5).astype(np.int32)
    part[0], part[1] = 0, 1
    p = dict(area_mode=1, depth=1, alpha=1, alpha_max=1, adaptive=0, max_iters=1,
             eps_ppm=1000000, terminals=1)
    o = oracle.refine_pair(g, part, 2, 0, 1, p)
    corridor = np.nonzero(o.side >= 0)[0]
    x, cuts = _pair_cuts(g, part, 0, 1, corridor)
    inter = x[cuts == cuts.min()].all(axis=0)
    t = o.trace[0]
    if t["cut_candidate"] < t["cut_before"] and t["decision"] == oracle.DEC_APPLY:
        want = part.copy()
        want[corridor] = np.where(inter, 0, 1)
        assert np.array_equal(o.part, want)
        assert o.result["cut_after"] == cuts.min()
    else:
        assert np.array_equal(o.part, part)


def test_rejects_unknown_terminal_mode():
    g = csr_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    part = np.array([0, 0, 1, 1], dtype=np.int32)
    o = oracle.refine_pair(g, part, 2, 0, 1, dict(alpha=1, alpha_max=1, adaptive=0, max_iters=1,
                                                  eps_ppm=30000, terminals=2))
    assert o.rc == -8

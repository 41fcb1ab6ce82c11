"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics, never against the oracle itself: brute-force minimum cuts,
independent max-flow algorithms (pure-Python Edmonds-Karp, scipy, networkx
preflow-push), closed forms, a corridor derived by sorting, and the invariants
stated in Section 4.1 (cut property C, adaptive rule, smallest source set)."""
import itertools

import networkx as nx
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import maximum_flow

import gen
from gen import Graph
import oracle
from tests.helpers import (area_bound, brute_force_min_cut, corridor_by_sorting, csr_from_edges,
                           edges_of, edmonds_karp, l_max, pair_network, random_graph)

# ------------------------------------------------------------ max flow ---


def _random_network(rng, nn, p, cmax):
    arcs = []
    for u in range(nn):
        for v in range(nn):
            if u != v and rng.random() < p:
                arcs.append((u, v, int(rng.integers(0, cmax + 1))))
    return arcs


def _of(arcs):
    t, h, c = zip(*arcs) if arcs else ((), (), ())
    return list(t), list(h), list(c)


@pytest.mark.parametrize("seed", range(40))
def test_maxflow_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    nn = int(rng.integers(3, 13))
    arcs = _random_network(rng, nn, 0.35, 6)
    if not arcs:
        arcs = [(0, 1, 1)]
    s, t = 0, nn - 1
    val, reach = oracle.maxflow(nn, *_of(arcs), s, t)
    best, inter, count = brute_force_min_cut(nn, arcs, s, t)
    assert val == best
    # the smallest source set is the intersection of all minimum source sets
    # (they form a lattice), and it is itself a minimum cut
    assert np.array_equal(reach, inter)
    cap = sum(c for u, v, c in arcs if reach[u] and not reach[v])
    assert cap == best


@pytest.mark.parametrize("seed", range(15))
def test_maxflow_vs_edmonds_karp(seed):
    rng = np.random.default_rng(100 + seed)
    nn = 40
    arcs = _random_network(rng, nn, 0.12, 20)
    val, reach = oracle.maxflow(nn, *_of(arcs), 0, nn - 1)
    ek_val, ek_reach = edmonds_karp(nn, arcs, 0, nn - 1)
    assert val == ek_val
    assert np.array_equal(reach, ek_reach)


@pytest.mark.parametrize("seed", range(6))
def test_maxflow_vs_scipy_and_networkx(seed):
    rng = np.random.default_rng(200 + seed)
    nn = 300
    arcs = {}
    for _ in range(2400):
        u, v = (int(x) for x in rng.integers(0, nn, 2))
        if u != v:
            arcs[(u, v)] = int(rng.integers(1, 50))
    arcs = [(u, v, c) for (u, v), c in arcs.items()]
    val, reach = oracle.maxflow(nn, *_of(arcs), 0, nn - 1)
    t, h, c = _of(arcs)
    m = csr_matrix((np.array(c, dtype=np.int32), (np.array(t), np.array(h))), shape=(nn, nn))
    assert maximum_flow(m, 0, nn - 1).flow_value == val
    G = nx.DiGraph()
    G.add_nodes_from(range(nn))
    for u, v, cap in arcs:
        G.add_edge(u, v, capacity=cap)
    R = nx.algorithms.flow.preflow_push(G, 0, nn - 1)
    assert R.graph["flow_value"] == val
    # smallest source set from networkx's own residual network
    seen, stack = {0}, [0]
    while stack:
        x = stack.pop()
        for y, d in R[x].items():
            if d["capacity"] - d["flow"] > 0 and y not in seen:
                seen.add(y)
                stack.append(y)
    assert set(np.nonzero(reach)[0].tolist()) == seen


def test_maxflow_closed_forms():
    # path: bottleneck
    caps = [7, 3, 9, 4]
    arcs = [(i, i + 1, c) for i, c in enumerate(caps)]
    val, reach = oracle.maxflow(5, *_of(arcs), 0, 4)
    assert val == 3 and reach.tolist() == [True, True, False, False, False]
    # disjoint parallel paths: sum of bottlenecks
    arcs, nxt, bott = [], 2, 0
    rng = np.random.default_rng(7)
    for _ in range(6):
        cs = rng.integers(1, 30, size=4)
        chain = [0] + list(range(nxt, nxt + 3)) + [1]
        nxt += 3
        arcs += [(chain[i], chain[i + 1], int(cs[i])) for i in range(4)]
        bott += int(cs.min())
    assert oracle.maxflow(nxt, *_of(arcs), 0, 1)[0] == bott
    # unit grid R x C, left column fed by s, right column drained to t:
    # R edge-disjoint row paths and a straight column cut of R (Menger)
    R, C = 9, 13
    g = gen.grid2d(R, C)
    s, t = R * C, R * C + 1
    arcs = [(u, v, 1) for u in range(g.n) for v in g.adjncy[g.xadj[u]:g.xadj[u + 1]]]
    arcs += [(s, y * C, 10 ** 6) for y in range(R)] + [(y * C + C - 1, t, 10 ** 6) for y in range(R)]
    val, reach = oracle.maxflow(R * C + 2, *_of(arcs), s, t)
    assert val == R
    # every row arc leaving column 0 is saturated, so the smallest source set
    # is s plus the fed column
    assert set(np.nonzero(reach[:R * C])[0].tolist()) == {y * C for y in range(R)}


def test_maxflow_tree():
    # tree: s-t path bottleneck decides, side branches do not matter
    edges = [(0, 1, 5), (1, 2, 2), (1, 3, 8), (3, 4, 6), (3, 5, 1), (5, 6, 9)]
    arcs = [(u, v, c) for u, v, c in edges] + [(v, u, c) for u, v, c in edges]
    assert oracle.maxflow(7, *_of(arcs), 0, 6)[0] == 1
    assert oracle.maxflow(7, *_of(arcs), 0, 4)[0] == 5


def test_maxflow_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.maxflow(3, [0], [5], [1], 0, 2)
    with pytest.raises(ValueError):
        oracle.maxflow(3, [0], [1], [1], 1, 1)


# --------------------------------------------------- pair refinement ---

SINGLE = dict(area_mode=0, depth=0, alpha=1, alpha_max=1, adaptive=0, max_iters=1, eps_ppm=30000)


def _independent_solve(g, part, k, a, b, p):
    """Everything the oracle computes for one solve, derived independently."""
    if p["area_mode"] == 1:
        in_a = corridor_by_sorting(g, part, a, b, 1, p["depth"], 0)
        in_b = corridor_by_sorting(g, part, b, a, 1, p["depth"], 0)
    else:
        ua = area_bound(g, part, k, b, p["alpha"], p["eps_ppm"])
        ub = area_bound(g, part, k, a, p["alpha"], p["eps_ppm"])
        in_a = corridor_by_sorting(g, part, a, b, 0, 0, ua)
        in_b = corridor_by_sorting(g, part, b, a, 0, 0, ub)
    nn, arcs, s, t, verts, border = pair_network(g, part, a, b, in_a, in_b)
    if nn - 2 <= 14:
        flow, inter, _ = brute_force_min_cut(nn, arcs, s, t)
        reach = inter
    else:
        flow, reach = edmonds_karp(nn, arcs, s, t)
    side = np.full(g.n, -1, dtype=np.int8)
    in_a_set = set(in_a.tolist())
    for i, u in enumerate(verts):
        side[u] = (2 if border[i] else 0) + (0 if reach[i] else 1)
    newpart = part.copy()
    for i, u in enumerate(verts):
        newpart[u] = a if reach[i] else b
    cut0 = sum(w for u, v, w in edges_of(g) if {part[u], part[v]} == {a, b})
    cut1 = sum(w for u, v, w in edges_of(g) if {newpart[u], newpart[v]} == {a, b})
    wa = int(g.vwgt[newpart == a].sum())
    wb = int(g.vwgt[newpart == b].sum())
    return dict(flow=flow, side=side, cut0=cut0, cut1=cut1, wa=wa, wb=wb,
                nv=len(verts), ne=sum(1 for (u, v, c) in arcs if u < v and v < nn - 2),
                in_a=in_a_set, newpart=newpart)


def _check_solve(g, part, k, a, b, p):
    p = dict(p, alpha_max=p["alpha"])
    o = oracle.refine_pair(g, part, k, a, b, p)
    assert o.rc == 0
    ind = _independent_solve(g, part, k, a, b, p)
    tr = o.trace[0]
    if ind["cut0"] == 0:
        assert tr["decision"] == oracle.DEC_NOT_ADJ
        return o, ind
    assert tr["flow"] == ind["flow"]
    assert np.array_equal(o.side, ind["side"])
    assert tr["region_vertices"] == ind["nv"]
    assert tr["region_edges"] == ind["ne"]
    assert tr["cut_before"] == ind["cut0"]
    assert tr["cut_candidate"] == ind["cut1"]  # cut - C_in + flow == recomputed cut
    assert (tr["wa"], tr["wb"]) == (ind["wa"], ind["wb"])
    lm = l_max(g, k, p["eps_ppm"])
    feasible = ind["wa"] <= lm and ind["wb"] <= lm
    expect = (oracle.DEC_INFEASIBLE if not feasible else
              oracle.DEC_APPLY if ind["cut1"] < ind["cut0"] else oracle.DEC_EQUAL)
    assert tr["decision"] == expect
    assert ind["cut1"] <= ind["cut0"]  # the old partition is a cut of G'
    if expect == oracle.DEC_APPLY:
        assert np.array_equal(o.part, ind["newpart"])
    else:
        assert np.array_equal(o.part, part)
    return o, ind


@pytest.mark.parametrize("seed", range(30))
def test_pair_solve_tiny_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 16))
    g = random_graph(n, 0.35, seed, wmax=6, vwmax=3 if seed % 3 == 0 else 1)
    part = (rng.random(n) < 0.5).astype(np.int32)
    p = dict(SINGLE, alpha=int(rng.choice([1, 2, 4, 8, 16])),
             eps_ppm=int(rng.choice([30000, 100000, 300000])))
    if seed % 5 == 0:
        p = dict(p, area_mode=1, depth=int(rng.integers(0, 3)))
    _check_solve(g, part, 2, 0, 1, p)


@pytest.mark.parametrize("seed", range(8))
def test_pair_solve_rgg_edmonds_karp(seed):
    g = gen.rgg(1500, 2, 8.0, seed=seed + 50, wlo=1, whi=10)
    k = 4
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.05, seed)
    a, b = [(0, 1), (1, 0), (2, 3), (0, 2)][seed % 4]
    p = dict(SINGLE, alpha=[1, 4, 16, 2][seed % 4], eps_ppm=[30000, 30000, 100000, 50000][seed % 4])
    _check_solve(g, part, k, a, b, p)


def test_pair_solve_depth_mode_and_zero_weights():
    g = gen.rgg(1200, 2, 7.0, seed=77, wlo=1, whi=5)
    g.vwgt = (np.arange(g.n) % 3).astype(np.int32)  # weights 0, 1, 2
    part = gen.rcb(g, 2)
    for p in (dict(SINGLE, area_mode=1, depth=3), dict(SINGLE, alpha=8),
              dict(SINGLE, alpha=16, eps_ppm=200000)):
        _check_solve(g, part, 2, 0, 1, p)
        _check_solve(g, part, 2, 1, 0, p)


def test_cut_property_alpha_one_always_feasible():
    """Sec. 4.1: with the corridor bound at eps' = eps every min cut of G' is
    balanced in G, for balanced inputs."""
    for seed in range(12):
        g = gen.rgg(2000, 2, 8.0, seed=300 + seed, wlo=1, whi=10)
        k = [2, 4, 8][seed % 3]
        part = gen.rcb(g, k)
        gen.global_noise(g, part, 0.03, seed)
        lm = l_max(g, k, 30000)
        if np.bincount(part, minlength=k).max() > lm:
            continue
        for a, b in [(0, 1), (1, 0)]:
            o = oracle.refine_pair(g, part, k, a, b, SINGLE)
            if o.trace[0]["decision"] != oracle.DEC_NOT_ADJ:
                assert o.trace[0]["decision"] != oracle.DEC_INFEASIBLE


def test_adaptive_rule_traces():
    """Sec. 4.1 adaptive flow iterations: accept -> min(2a, a'), reject ->
    max(a/2, 1), stop on a feasible cut without improvement."""
    for seed in range(6):
        g = gen.rgg(6000, 2, 8.0, seed=400 + seed, wlo=1, whi=10)
        part = gen.rcb(g, 2, force_axis=0)
        gen.pair_swap_noise(g, part, 0.1, seed)
        p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=12,
                 eps_ppm=30000)
        o = oracle.refine_pair(g, part, 2, 0, 1, p)
        tr = o.trace
        assert tr[0]["alpha"] == 16
        for prev, nxt in zip(tr, tr[1:]):
            if prev["decision"] == oracle.DEC_APPLY:
                assert nxt["alpha"] == min(2 * prev["alpha"], 16)
                assert nxt["cut_before"] == prev["cut_candidate"]
            else:
                assert prev["decision"] == oracle.DEC_INFEASIBLE and prev["alpha"] > 1
                assert nxt["alpha"] == max(prev["alpha"] // 2, 1)
                assert nxt["cut_before"] == prev["cut_before"]
        last = tr[-1]["decision"]
        if len(tr) < 12:
            assert last in (oracle.DEC_EQUAL, oracle.DEC_NOT_ADJ) or (
                last == oracle.DEC_INFEASIBLE and tr[-1]["alpha"] == 1)
        assert o.result["cut_after"] <= o.result["cut_before"]
        assert o.result["applied"] == sum(r["decision"] == oracle.DEC_APPLY for r in tr)
        lm = l_max(g, 2, 30000)
        assert o.result["weight_a"] <= lm and o.result["weight_b"] <= lm
        assert o.result["region_edges"] == sum(r["region_edges"] for r in tr)


def _wavy(seed, amp, f):
    """A 2D RGG (n = 3000) split along x = 0.5 + amp sin(2 pi f y): a long
    boundary that small corridors cannot straighten."""
    g = gen.rgg(3000, 2, 8.0, seed=seed, wlo=1, whi=int([1, 10][seed % 2]))
    x, y = g.coords[:, 0], g.coords[:, 1]
    return g, (x > 0.5 + amp * np.sin(2 * np.pi * f * y)).astype(np.int32)


def _swapped(seed):
    g = gen.rgg(3000, 2, 8.0, seed=seed, wlo=1, whi=int([1, 10][seed % 2]))
    part = gen.rcb(g, 2, force_axis=seed % 2)
    gen.pair_swap_noise(g, part, [0.002, 0.01, 0.05][(seed - 700) % 3], seed - 700)
    return g, part


def test_restart_rule_composes():
    """R6b (the one restart of a learned start): when a search that started
    below the restart factor applies nothing and meets a feasible,
    non-improving solve, the
    restarted call is that search followed by the plain search from the
    restart factor on the same partition with the iterations left; records,
    result and partition are those of the two calls in sequence."""
    cases = [(_wavy(902, 0.2, 1), 1), (_wavy(911, 0.2, 1), 1), (_swapped(715), 1)]
    for (g, part), a0 in cases:
        p = dict(area_mode=0, depth=0, alpha=a0, alpha_max=16, adaptive=1, max_iters=8,
                 eps_ppm=30000)
        first = oracle.refine_pair(g, part, 2, 0, 1, p)
        assert first.result["applied"] == 0 and first.trace[-1]["decision"] == oracle.DEC_EQUAL
        assert first.trace[-1]["alpha"] < 16
        used = len(first.trace)
        second = oracle.refine_pair(g, part, 2, 0, 1, dict(p, alpha=16, max_iters=8 - used))
        both = oracle.refine_pair(g, part, 2, 0, 1, dict(p, restart_alpha=16))
        assert both.trace == first.trace + second.trace
        assert both.trace[used]["alpha"] == 16
        assert np.array_equal(both.part, second.part)
        for key in ("applied", "cut_after", "weight_a", "weight_b", "final_alpha", "iter_cap"):
            assert both.result[key] == second.result[key], key
        assert both.result["iters"] == used + second.result["iters"]
        assert both.result["region_edges"] == (first.result["region_edges"] +
                                               second.result["region_edges"])
        assert both.result["cut_after"] < first.result["cut_after"]
        # capped below the restart factor by alpha_max: the restart runs from 8
        capped = oracle.refine_pair(g, part, 2, 0, 1, dict(p, alpha_max=8, restart_alpha=16))
        assert capped.trace[used]["alpha"] == 8


def test_restart_rule_leaves_other_searches_alone():
    """R6b changes nothing for a search that applied a cut, ended on an
    infeasible cut at factor 1 or started at the restart factor; with no
    iteration left it changes only the iteration-cap flag; a negative
    restart factor is rejected."""
    seen = set()
    for seed in range(700, 712):
        g, part = _swapped(seed)
        for a0 in (1, 2, 16):
            p = dict(area_mode=0, depth=0, alpha=a0, alpha_max=16, adaptive=1, max_iters=8,
                     eps_ppm=30000)
            o = oracle.refine_pair(g, part, 2, 0, 1, p)
            last = o.trace[-1]["decision"]
            if o.result["applied"] > 0 or last != oracle.DEC_EQUAL or a0 == 16:
                q = oracle.refine_pair(g, part, 2, 0, 1, dict(p, restart_alpha=16))
                assert q.trace == o.trace and np.array_equal(q.part, o.part)
                seen.add("start" if a0 == 16 else ("applied" if o.result["applied"] else last))
    assert "applied" in seen and "start" in seen
    g, part = _wavy(902, 0.2, 1)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=16, adaptive=1, max_iters=1, eps_ppm=30000)
    o = oracle.refine_pair(g, part, 2, 0, 1, p)
    q = oracle.refine_pair(g, part, 2, 0, 1, dict(p, restart_alpha=16))
    # the restart is due but no iteration is left: the same solve, and the
    # iteration cap reports the search as cut off
    assert len(q.trace) == 1 and q.trace == o.trace
    assert o.result["iter_cap"] == 0 and q.result["iter_cap"] == 1
    assert np.array_equal(q.part, o.part)
    assert oracle.refine_pair(g, part, 2, 0, 1, dict(p, restart_alpha=-1)).rc == -8


def test_restart_rule_in_batches():
    """R6b inside a batch: two wavy cases side by side as one graph (k = 4,
    the same balance bound as each alone with k = 2).  The batch with a
    restart factor equals the pairs refined one after the other with it, and
    each pair ends exactly as its case refined alone."""
    (g1, p1), (g2, p2) = _wavy(902, 0.2, 1), _wavy(911, 0.2, 1)
    n1 = g1.n
    xadj = np.concatenate([g1.xadj, g2.xadj[1:] + g1.xadj[-1]]).astype(np.int32)
    adj = np.concatenate([g1.adjncy, g2.adjncy + n1]).astype(np.int32)
    g = Graph(xadj, adj, np.concatenate([g1.adjwgt, g2.adjwgt]).astype(np.int32),
              np.concatenate([g1.vwgt, g2.vwgt]).astype(np.int32))
    part = np.concatenate([p1, p2 + 2]).astype(np.int32)
    p = dict(area_mode=0, depth=0, alpha=1, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=30000, restart_alpha=16)
    pairs = [(0, 1), (2, 3)]
    rc, res, tr, bpart = oracle.refine_batch(g, part, 4, pairs, p)
    assert rc == 0
    cur = part.copy()
    for i, (a, b) in enumerate(pairs):
        o = oracle.refine_pair(g, cur, 4, a, b, p)
        assert o.result == res[i] and o.trace == tr[i]
        cur = o.part
    assert np.array_equal(cur, bpart)
    for i, (gi, pi) in enumerate(((g1, p1), (g2, p2))):
        alone = oracle.refine_pair(gi, pi, 2, 0, 1, p)
        assert alone.trace == tr[i] and alone.result["cut_after"] == res[i]["cut_after"]
        assert len(tr[i]) > 1 and tr[i][1]["alpha"] == 16  # the restart fired


def test_c1_closed_form():
    """128x128 unit grid, depth-8 corridor: 128 row-disjoint paths join the
    pinned borders and a straight column cut costs 128, so the flow is 128
    (Menger).  The smallest source set is cut right of the pinned left border,
    which moves the left corridor to block 1 and breaks L_max = 8438."""
    w = gen.config("C1")
    o = oracle.refine_pair(w.graph, w.part, 2, 0, 1, w.params)
    tr = o.trace[0]
    assert tr["flow"] == 128
    assert l_max(w.graph, 2, 30000) == 8438
    assert tr["decision"] == oracle.DEC_INFEASIBLE and tr["wb"] > 8438
    assert o.result["status"] == oracle.ST_REJECTED
    assert np.array_equal(o.part, w.part)
    # every source-side corridor vertex lies left of every sink-side one in its row
    side = o.side
    for y in range(128):
        row = side[y * 128:(y + 1) * 128]
        xs_src = np.nonzero((row == 0) | (row == 2))[0]
        xs_snk = np.nonzero((row == 1) | (row == 3))[0]
        assert xs_src.max() < xs_snk.min()
    _check_solve(w.graph, w.part, 2, 0, 1, w.params)


def test_c1b_accepts_balanced():
    w = gen.config("C1B")
    o, ind = _check_solve(w.graph, w.part, 2, 0, 1, w.params)
    assert o.result["status"] == oracle.ST_ACCEPTED
    lm = l_max(w.graph, 2, 30000)
    assert o.result["weight_a"] <= lm and o.result["weight_b"] <= lm
    assert o.result["cut_after"] < o.result["cut_before"]


def test_not_adjacent_and_bad_pairs():
    g = csr_from_edges(6, [(0, 1), (1, 2), (3, 4), (4, 5)])
    part = np.array([0, 0, 1, 2, 2, 3], dtype=np.int32)
    o = oracle.refine_pair(g, part, 4, 0, 2, dict(SINGLE))
    assert o.rc == 0 and o.result["status"] == oracle.ST_NOT_ADJACENT
    assert oracle.refine_pair(g, part, 4, 0, 0, dict(SINGLE)).rc == -3
    assert oracle.refine_pair(g, part, 4, 0, 9, dict(SINGLE)).rc == -3
    rc, *_ = oracle.refine_batch(g, part, 4, [(0, 1), (1, 2)], dict(SINGLE))
    assert rc == -4


def test_validate_graph():
    g = random_graph(20, 0.3, 1)
    assert oracle.validate_graph(g)
    bad = random_graph(20, 0.3, 1)
    bad.adjwgt = bad.adjwgt.copy()
    bad.adjwgt[0] += 1  # asymmetric weight
    assert not oracle.validate_graph(bad)
    loop = csr_from_edges(3, [(0, 1)])
    loop.adjncy = loop.adjncy.copy()
    loop.adjncy[0] = 0  # self loop
    assert not oracle.validate_graph(loop)


# ------------------------------------------------------ batch / sweep ---

def test_batch_order_independent():
    g = gen.rgg(8000, 2, 8.0, seed=21, wlo=1, whi=10)
    k = 16
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.02, 21)
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour) if c == 0]
    assert len(pairs) >= 4
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8, eps_ppm=30000)
    rc, res0, tr0, part0 = oracle.refine_batch(g, part, k, pairs, p)
    assert rc == 0
    rng = np.random.default_rng(0)
    for _ in range(3):
        perm = rng.permutation(len(pairs))
        rc, res1, tr1, part1 = oracle.refine_batch(g, part, k, [pairs[i] for i in perm], p)
        assert rc == 0 and np.array_equal(part0, part1)
        for j, i in enumerate(perm):
            assert res1[j] == res0[i] and tr1[j] == tr0[i]
    # and equal to the pairs one by one
    cur = part.copy()
    for i, (a, b) in enumerate(pairs):
        o = oracle.refine_pair(g, cur, k, a, b, p, want_side=False)
        assert o.result == res0[i]
        cur = o.part
    assert np.array_equal(cur, part0)


def test_quotient_colouring_is_greedy_matching():
    g = gen.rgg(6000, 2, 8.0, seed=31)
    k = 16
    part = gen.rcb(g, k)
    edges, colour = oracle.quotient_colouring(g, part, k)
    # edges = exactly the adjacent block pairs, sorted
    adj = set()
    for u, v, _ in edges_of(g):
        if part[u] != part[v]:
            adj.add((min(part[u], part[v]), max(part[u], part[v])))
    assert [tuple(e) for e in edges.tolist()] == sorted(adj)
    for c in set(colour.tolist()):
        blocks = [x for e, cc in zip(edges.tolist(), colour) if cc == c for x in e]
        assert len(blocks) == len(set(blocks))  # a matching
    for i, (x, y) in enumerate(edges.tolist()):  # smallest free colour
        used = {colour[j] for j in range(i) if {x, y} & set(edges[j].tolist())}
        assert colour[i] == min(set(range(colour[i] + 1)) - used)


def test_sweep_monotone():
    g = gen.rgg(8000, 2, 6.0, seed=41)
    k = 16
    part = gen.rcb(g, k)
    gen.global_noise(g, part, 0.02, 41)
    c0 = oracle.total_cut(g, part)
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8, eps_ppm=30000)
    rc, c1, stats, newpart = oracle.sweep(g, part, k, p, max_sweeps=8)
    assert rc == 0 and c1 <= c0 and stats[0] >= 1
    assert c1 == sum(w for u, v, w in edges_of(g) if newpart[u] != newpart[v])
    lm = l_max(g, k, 30000)
    assert np.bincount(newpart, minlength=k).max() <= max(lm, np.bincount(part, minlength=k).max())


# ------------------------------------------------------------ features ---

def test_pair_features_direct():
    g = gen.rgg(3000, 2, 8.0, seed=61, wlo=1, whi=10)
    k = 8
    part = gen.rcb(g, k)
    a, b = 0, 1
    f = oracle.pair_features(g, part, k, a, b, 30000)
    da = [u for u in range(g.n) if part[u] == a and any(part[v] == b for v in g.adjncy[g.xadj[u]:g.xadj[u + 1]])]
    db = [u for u in range(g.n) if part[u] == b and any(part[v] == a for v in g.adjncy[g.xadj[u]:g.xadj[u + 1]])]
    cv = g.vwgt.sum()
    W = cv / k
    ca, cb = g.vwgt[part == a].sum(), g.vwgt[part == b].sum()
    cut = sum(w for u, v, w in edges_of(g) if {part[u], part[v]} == {a, b})
    lm = l_max(g, k, 30000)
    u1 = area_bound(g, part, k, b, 1, 30000)
    expect = [np.log2(1 + len(da)), np.log2(1 + len(db)), ca / W, cb / W, np.log2(1 + cut),
              (lm - ca) / W, (lm - cb) / W, np.log2(1 + u1 / max(1, g.vwgt[da].sum()))]
    assert np.allclose(f, expect, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------ MLP ref ---

def _mlp_params(rng):
    return {"W1": rng.normal(0, 0.5, (8, 64)), "b1": rng.normal(0, 0.1, 64),
            "W2": rng.normal(0, 0.2, (64, 64)), "b2": rng.normal(0, 0.1, 64),
            "W3": rng.normal(0, 0.2, (64, 5)), "b3": rng.normal(0, 0.1, 5)}


def test_mlp_reference_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    P = _mlp_params(rng)
    x = rng.normal(0, 1, (33, 8))
    y = rng.integers(0, 5, 33)
    loss, grads = oracle.mlp_loss_grad(P, x, y)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    xt = torch.tensor(x)
    h = torch.relu(xt @ T["W1"] + T["b1"])
    h = torch.relu(h @ T["W2"] + T["b2"])
    z = h @ T["W3"] + T["b3"]
    lt = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12
    for k in P:
        assert np.allclose(T[k].grad.numpy(), grads[k], rtol=1e-10, atol=1e-12)


def test_mlp_cost_reference_matches_torch_autograd():
    """The expected-cost loss mean_i sum_c p_ic cost_ic and its hand-written
    gradient against torch autograd on the same network."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    P = _mlp_params(rng)
    x = rng.normal(0, 1, (29, 8))
    costs = rng.uniform(-1, 3, (29, 5))
    loss, grads = oracle.mlp_loss_grad_cost(P, x, costs)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    xt = torch.tensor(x)
    h = torch.relu(xt @ T["W1"] + T["b1"])
    h = torch.relu(h @ T["W2"] + T["b2"])
    z = h @ T["W3"] + T["b3"]
    lt = (torch.softmax(z, 1) * torch.tensor(costs)).sum(1).mean()
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12
    for k in P:
        assert np.allclose(T[k].grad.numpy(), grads[k], rtol=1e-10, atol=1e-12)


def test_mlp_cost_reference_invariants():
    """Costs equal across the classes of a sample leave nothing to learn (loss
    = their mean, gradient 0); adding a constant to a sample's costs moves
    the loss by its mean share and leaves the gradient unchanged; central
    differences agree with the gradient."""
    rng = np.random.default_rng(14)
    P = _mlp_params(rng)
    x = rng.normal(0, 1, (11, 8))
    flat = np.repeat(rng.uniform(0, 2, (11, 1)), 5, axis=1)
    loss, grads = oracle.mlp_loss_grad_cost(P, x, flat)
    assert abs(loss - flat[:, 0].mean()) < 1e-12
    assert all(np.abs(g).max() < 1e-12 for g in grads.values())
    costs = rng.uniform(0, 1, (11, 5))
    shift = rng.uniform(-2, 2, (11, 1))
    l0, g0 = oracle.mlp_loss_grad_cost(P, x, costs)
    l1, g1 = oracle.mlp_loss_grad_cost(P, x, costs + shift)
    assert abs((l1 - l0) - shift.mean()) < 1e-12
    for k in P:
        assert np.allclose(g0[k], g1[k], rtol=1e-9, atol=1e-12)
    h = 1e-6
    for k in P:
        fl = P[k].reshape(-1)
        for idx in itertools.islice(rng.permutation(fl.size), 4):
            old = fl[idx]
            fl[idx] = old + h
            lp, _ = oracle.mlp_loss_grad_cost(P, x, costs)
            fl[idx] = old - h
            lm, _ = oracle.mlp_loss_grad_cost(P, x, costs)
            fl[idx] = old
            assert abs((lp - lm) / (2 * h) - g0[k].reshape(-1)[idx]) < 1e-6


def test_mlp_reference_finite_differences():
    rng = np.random.default_rng(4)
    P = _mlp_params(rng)
    x = rng.normal(0, 1, (9, 8))
    y = rng.integers(0, 5, 9)
    _, grads = oracle.mlp_loss_grad(P, x, y)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in itertools.islice(rng.permutation(flat.size), 6):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = oracle.mlp_loss_grad(P, x, y)
            flat[idx] = old - h
            lm, _ = oracle.mlp_loss_grad(P, x, y)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - grads[k].reshape(-1)[idx]) < 1e-6

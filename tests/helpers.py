"""Independent test helpers: tiny graphs, brute-force minimum cuts, a
pure-Python Edmonds-Karp, and a corridor derived by sorting instead of by a
level walk.  None of this calls the oracle or the GPU library."""
from __future__ import annotations

from collections import deque

import numpy as np

from gen import Graph


def csr_from_edges(n: int, edges, weights=None, vwgt=None) -> Graph:
    """Symmetric CSR from an undirected edge list (u, v), u != v, no duplicates."""
    edges = [(int(u), int(v)) for u, v in edges]
    if weights is None:
        weights = [1] * len(edges)
    adj = [[] for _ in range(n)]
    for (u, v), w in zip(edges, weights):
        adj[u].append((v, int(w)))
        adj[v].append((u, int(w)))
    xadj = np.zeros(n + 1, dtype=np.int32)
    adjncy, adjwgt = [], []
    for u in range(n):
        lst = sorted(adj[u])
        xadj[u + 1] = xadj[u] + len(lst)
        adjncy += [v for v, _ in lst]
        adjwgt += [w for _, w in lst]
    vw = np.ones(n, dtype=np.int32) if vwgt is None else np.asarray(vwgt, dtype=np.int32)
    return Graph(xadj, np.asarray(adjncy, dtype=np.int32), np.asarray(adjwgt, dtype=np.int32), vw)


def random_graph(n: int, p: float, seed: int, wmax: int = 10, vwmax: int = 1) -> Graph:
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.append((u, v))
                ws.append(int(rng.integers(1, wmax + 1)))
    vw = rng.integers(0 if vwmax > 1 else 1, vwmax + 1, size=n) if vwmax > 1 else None
    return csr_from_edges(n, edges, ws, vw)


def edges_of(g: Graph):
    for u in range(g.n):
        for e in range(g.xadj[u], g.xadj[u + 1]):
            v = int(g.adjncy[e])
            if u < v:
                yield u, v, int(g.adjwgt[e])


def brute_force_min_cut(nn: int, arcs, s: int, t: int):
    """All 2^(nn-2) source sets containing s and not t.  Returns (min cut
    value, the intersection of all minimum source sets as a bool array, the
    number of minimum cuts).  arcs = [(u, v, cap)] directed."""
    others = [v for v in range(nn) if v not in (s, t)]
    m = len(others)
    assert m <= 20
    tails = np.array([a[0] for a in arcs], dtype=np.int64)
    heads = np.array([a[1] for a in arcs], dtype=np.int64)
    caps = np.array([a[2] for a in arcs], dtype=np.int64)
    masks = np.arange(1 << m, dtype=np.int64)
    side = np.zeros((1 << m, nn), dtype=bool)  # True = source side
    for j, v in enumerate(others):
        side[:, v] = (masks >> j) & 1
    side[:, s] = True
    side[:, t] = False
    cutcap = (side[:, tails] & ~side[:, heads]).astype(np.int64) @ caps
    best = cutcap.min()
    mins = side[cutcap == best]
    return int(best), mins.all(axis=0), int(mins.shape[0])


def edmonds_karp(nn: int, arcs, s: int, t: int):
    """Shortest augmenting paths (Edmonds & Karp 1972), pure Python.  Returns
    (flow, reach) with reach = nodes reachable from s in the final residual
    graph."""
    res = {}
    nbr = [set() for _ in range(nn)]
    for u, v, c in arcs:
        res[(u, v)] = res.get((u, v), 0) + c
        res.setdefault((v, u), 0)
        nbr[u].add(v)
        nbr[v].add(u)
    flow = 0
    while True:
        par = [-1] * nn
        par[s] = s
        q = deque([s])
        while q and par[t] < 0:
            u = q.popleft()
            for v in nbr[u]:
                if par[v] < 0 and res[(u, v)] > 0:
                    par[v] = u
                    q.append(v)
        if par[t] < 0:
            break
        b, v = None, t
        while v != s:
            u = par[v]
            b = res[(u, v)] if b is None else min(b, res[(u, v)])
            v = u
        v = t
        while v != s:
            u = par[v]
            res[(u, v)] -= b
            res[(v, u)] += b
            v = u
        flow += b
    reach = np.zeros(nn, dtype=bool)
    reach[s] = True
    q = deque([s])
    while q:
        u = q.popleft()
        for v in nbr[u]:
            if not reach[v] and res[(u, v)] > 0:
                reach[v] = True
                q.append(v)
    return flow, reach


def block_distances(g: Graph, part: np.ndarray, blk: int, other: int) -> np.ndarray:
    """Hop distance inside block blk from the vertices of blk that touch block
    other (multi-source BFS); -1 where unreachable or outside blk."""
    dist = np.full(g.n, -1, dtype=np.int64)
    q = deque()
    for u in range(g.n):
        if part[u] == blk and any(part[v] == other for v in g.adjncy[g.xadj[u]:g.xadj[u + 1]]):
            dist[u] = 0
            q.append(u)
    while q:
        u = q.popleft()
        for v in g.adjncy[g.xadj[u]:g.xadj[u + 1]]:
            if part[v] == blk and dist[v] < 0:
                dist[v] = dist[u] + 1
                q.append(v)
    return dist


def corridor_by_sorting(g: Graph, part, blk, other, mode, depth, bound) -> np.ndarray:
    """The corridor side of blk, derived differently from a level walk: sort
    the reachable vertices by (distance, id) and keep the longest prefix whose
    weight stays within the bound (FACTOR), or every vertex with distance <=
    depth (DEPTH)."""
    dist = block_distances(g, part, blk, other)
    cand = np.nonzero(dist >= 0)[0]
    if mode == 1:
        return cand[dist[cand] <= depth]
    order = cand[np.lexsort((cand, dist[cand]))]
    csum = np.cumsum(g.vwgt[order].astype(np.int64))
    bad = np.nonzero(csum > bound)[0]
    stop = bad[0] if bad.size else order.size
    return np.sort(order[:stop])


def area_bound(g: Graph, part, k, other, alpha, eps_ppm) -> int:
    cv = int(g.vwgt.astype(np.int64).sum())
    c_other = int(g.vwgt[part == other].astype(np.int64).sum())
    return max(0, (1_000_000 + alpha * eps_ppm) * cv // (1_000_000 * k) - c_other)


def l_max(g: Graph, k, eps_ppm) -> int:
    cv = int(g.vwgt.astype(np.int64).sum())
    return (1_000_000 + eps_ppm) * cv // (1_000_000 * k) + int(g.vwgt.max())


def pair_network(g: Graph, part, a, b, in_a: np.ndarray, in_b: np.ndarray):
    """Corridor network G' from the corridor sides: node ids = corridor
    vertices in ascending id, then s, t; undirected corridor edges as two
    arcs; s -> left border and right border -> t with a capacity above every
    finite cut.  Returns (nn, arcs, s, t, verts, border)."""
    inb = np.zeros(g.n, dtype=bool)
    inb[in_a] = True
    inb[in_b] = True
    verts = np.nonzero(inb)[0]
    loc = {int(v): i for i, v in enumerate(verts)}
    side_a = np.zeros(g.n, dtype=bool)
    side_a[in_a] = True
    nn = len(verts) + 2
    s, t = nn - 2, nn - 1
    arcs, total = [], 0
    border = np.zeros(len(verts), dtype=bool)
    for u in verts:
        for e in range(g.xadj[u], g.xadj[u + 1]):
            v, w = int(g.adjncy[e]), int(g.adjwgt[e])
            if inb[v]:
                arcs.append((loc[int(u)], loc[v], w))
                total += w
            elif part[v] in (a, b):
                border[loc[int(u)]] = True
    big = total + 1
    for i, u in enumerate(verts):
        if border[i]:
            arcs.append((s, i, big) if side_a[u] else (i, t, big))
    return nn, arcs, s, t, verts, border


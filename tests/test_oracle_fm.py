"""Pins of the oracle's 2-way FM local search with TopGain (Sec. 2.2), the
pairwise improvement that runs before the flow.  The move log is replayed
from scratch: at every step the gains are recomputed from their definition
(never from the oracle's incremental updates), the queue is the boundary plus
the neighbours of moved vertices, and the moved vertex must be the one the
TopGain rule picks; the kept prefix must be the first best state of the
trajectory, and cut and weights are recomputed from the final partition.
Plus closed forms on grids and the stop rule."""
import numpy as np
import pytest

import gen
import oracle
from tests.helpers import csr_from_edges, l_max, random_graph

MASK = 2**64 - 1


def _sm(seed, n):
    return gen.splitmix64_stream((int(seed) + (int(n) - 1) * 0x9E3779B97F4A7C15) & MASK, 1)[0]


def _key(seed, v):
    return _sm(seed, v + 1)


def _bit(seed, t):
    return _sm(seed, (1 << 32) + t + 1) & 1


def _gains(g, part, a, b):
    gain = {}
    for v in range(g.n):
        if part[v] not in (a, b):
            continue
        other = b if part[v] == a else a
        ext = inn = 0
        for e in range(g.xadj[v], g.xadj[v + 1]):
            u, w = g.adjncy[e], int(g.adjwgt[e])
            if part[u] == other:
                ext += w
            elif part[u] == part[v]:
                inn += w
        gain[v] = (ext - inn, ext > 0)
    return gain


def _cut(g, part, a, b):
    c = 0
    for v in range(g.n):
        if part[v] != a:
            continue
        for e in range(g.xadj[v], g.xadj[v + 1]):
            if part[g.adjncy[e]] == b:
                c += int(g.adjwgt[e])
    return c


def _replay(g, part0, k, a, b, eps, limit, seed, log, info):
    lmax = l_max(g, k, eps)
    part = part0.copy()
    w = lambda blk: int(g.vwgt[part == blk].sum())
    gains0 = _gains(g, part, a, b)
    queued = {v for v, (_, bnd) in gains0.items() if bnd}
    moved = set()
    qual = []

    def quality():
        wa, wb = w(a), w(b)
        inf = not (wa <= lmax and wb <= lmax)
        return (int(inf), max(wa, wb) if inf else _cut(g, part, a, b))

    qual.append(quality())
    for t, v in enumerate(log):
        gains = _gains(g, part, a, b)
        tops = []
        for side in (a, b):
            cand = [u for u in queued if u not in moved and part[u] == side]
            tops.append(max(cand, key=lambda u: (gains[u][0], _key(seed, u))) if cand else None)
        wa, wb = w(a), w(b)
        if (wa > lmax or wb > lmax) and wa != wb:
            side = 0 if wa > wb else 1
        elif tops[0] is None or tops[1] is None:
            side = 1 if tops[0] is None else 0
        elif gains[tops[0]][0] != gains[tops[1]][0]:
            side = 0 if gains[tops[0]][0] > gains[tops[1]][0] else 1
        else:
            side = _bit(seed, t)
        if tops[side] is None:
            side = 1 - side
        assert v == tops[side], (t, v, tops)
        part[v] = b if part[v] == a else a
        moved.add(v)
        for e in range(g.xadj[v], g.xadj[v + 1]):
            u = g.adjncy[e]
            if part[u] in (a, b) and u not in moved:
                queued.add(u)
        qual.append(quality())
    # stop rule: after the first best state, at most `limit` further moves
    best = min(range(len(qual)), key=lambda i: (qual[i], i))
    assert info["kept"] == best
    assert len(log) - best <= limit
    final = part0.copy()
    for v in log[:best]:
        final[v] = b if final[v] == a else a
    return final, qual[best]


@pytest.mark.parametrize("seed", range(24))
def test_fm_replay_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(10, 60))
    g = random_graph(n, 0.15, seed, wmax=int(rng.choice([1, 5])), vwmax=int(rng.choice([1, 3])))
    k = int(rng.choice([2, 3]))
    part = rng.integers(0, k, n).astype(np.int32)
    part[0], part[1] = 0, 1
    eps = int(rng.choice([0, 30000, 300000]))
    limit = int(rng.integers(1, 12))
    fseed = int(rng.integers(0, 2**32))
    out, info, log = oracle.pair_fm(g, part, k, 0, 1, eps, limit, fseed)
    assert len(set(log.tolist())) == len(log)  # each vertex moves at most once
    final, q = _replay(g, part, k, 0, 1, eps, limit, fseed, log.tolist(), info)
    assert np.array_equal(out, final)
    assert info["cut_after"] == _cut(g, out, 0, 1)
    assert info["cut_before"] == _cut(g, part, 0, 1)
    assert info["weight_a"] == int(g.vwgt[out == 0].sum())
    assert info["weight_b"] == int(g.vwgt[out == 1].sum())
    assert np.array_equal(out[(part != 0) & (part != 1)], part[(part != 0) & (part != 1)])


@pytest.mark.parametrize("seed", range(6))
def test_fm_replay_rgg_pairs(seed):
    g = gen.rgg(2000, 2, 7.0, 60 + seed, 1, 4 if seed % 2 else 1)
    part = gen.rcb(g, 4)
    gen.global_noise(g, part, 0.05, seed)
    out, info, log = oracle.pair_fm(g, part, 4, 0, 1, 30000, 25, seed)
    final, _ = _replay(g, part, 4, 0, 1, 30000, 25, seed, log.tolist(), info)
    assert np.array_equal(out, final)
    assert info["cut_after"] <= info["cut_before"] or \
        max(info["weight_a"], info["weight_b"]) > l_max(g, 4, 30000)


def _grid(rows, cols):
    return gen.grid2d(rows, cols)


def test_fm_returns_a_misplaced_vertex():
    """10 x 10 unit grid, columns 0..4 | 5..9, with vertex (row 4, col 5) put
    in block 0: cut 10 - 1 + 3 = 12 (the vertex has one neighbour in block 0
    and three in block 1).  Its gain is 3 - 1 = 2, the only positive gain, so
    FM moves it first and the best state is the straight cut of 10."""
    g = _grid(10, 10)
    x = np.arange(100) % 10
    part = (x >= 5).astype(np.int32)
    part[4 * 10 + 5] = 0
    out, info, log = oracle.pair_fm(g, part, 2, 0, 1, 30000, 10, 3)
    assert info["cut_before"] == 12 and info["cut_after"] == 10
    assert log[0] == 45 and info["kept"] == 1
    assert np.array_equal(out, (x >= 5).astype(np.int32))


def test_fm_rebalances_an_overloaded_block():
    """A unit path of 20 split 14 | 6 with eps 0 (L_max = 11): block 0 is
    overloaded, so TopGain moves out of it.  Moving its end vertex 13 (gain 0:
    one edge each way) is forced first; every move shifts the single cut edge;
    the first feasible state is 11 | 9, three moves, cut 1 throughout."""
    g = csr_from_edges(20, [(i, i + 1) for i in range(19)])
    part = (np.arange(20) >= 14).astype(np.int32)
    out, info, log = oracle.pair_fm(g, part, 2, 0, 1, 0, 5, 1)
    assert log.tolist()[:3] == [13, 12, 11]
    assert info["kept"] == 3 and info["cut_after"] == 1
    assert (info["weight_a"], info["weight_b"]) == (11, 9)


def test_fm_off_and_pair_level():
    g = gen.rgg(3000, 2, 7.0, 5, 1, 1)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, 5)
    out, info, log = oracle.pair_fm(g, part, 2, 0, 1, 30000, 0, 1)
    assert len(log) == 0 and np.array_equal(out, part)
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=6,
             eps_ppm=30000)
    plain = oracle.refine_pair(g, part.copy(), 2, 0, 1, p)
    fm = oracle.refine_pair(g, part.copy(), 2, 0, 1, dict(p, fm_limit=50, fm_seed=2))
    assert fm.result["cut_before"] == plain.result["cut_before"]
    # the flow starts from the FM result
    fpart, finfo, _ = oracle.pair_fm(g, part, 2, 0, 1, 30000, 50, 2)
    assert fm.trace[0]["cut_before"] == finfo["cut_after"]
    assert fm.result["cut_after"] == oracle.total_cut(g, fm.part)


# ------------------------------------------------- active block scheduling --

def _active_sweeps(g, part, k, p, max_sweeps):
    """Active block scheduling (Sec. 4.3) written out over the oracle's
    quotient colouring and batch refinement: every block starts active; a
    sweep refines, class by class, the pairs with an active block; the blocks
    of the pairs it changed are the next sweep's active ones."""
    part = part.copy()
    active = np.ones(k, dtype=bool)
    solves = changed_pairs = sweeps = 0
    for _ in range(max_sweeps):
        edges, colour = oracle.quotient_colouring(g, part, k)
        nxt = np.zeros(k, dtype=bool)
        changed = 0
        for c in sorted(set(colour.tolist())):
            pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour.tolist())
                     if cc == c and (active[e[0]] or active[e[1]])]
            if not pairs:
                continue
            rc, res, _, part = oracle.refine_batch(g, part, k, pairs, p)
            assert rc == 0
            for (a, b), r in zip(pairs, res):
                solves += r["iters"]
                if r["status"] == oracle.ST_ACCEPTED:
                    changed += 1
                    nxt[a] = nxt[b] = True
        sweeps += 1
        changed_pairs += changed
        if changed == 0:
            break
        active = nxt
    return part, sweeps, solves, changed_pairs


@pytest.mark.parametrize("fm", [0, 30])
def test_active_block_sweeps(fm):
    g = gen.rgg(1 << 13, 2, 7.0, 17, 1, 1)
    part = gen.rcb(g, 16)
    gen.global_noise(g, part, 0.03, 17)
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=8,
             eps_ppm=30000, fm_limit=fm, fm_seed=4, active_blocks=1)
    want, sweeps, solves, changed = _active_sweeps(g, part, 16, p, 6)
    rc, tc, stats, got = oracle.sweep(g, part, 16, p, max_sweeps=6)
    assert rc == 0 and np.array_equal(got, want)
    assert stats[0] == sweeps and stats[1] == solves and stats[2] == changed
    # the first sweep refines every pair, as without active blocks
    rc1, _, s1, p1 = oracle.sweep(g, part, 16, p, max_sweeps=1)
    rc2, _, s2, p2 = oracle.sweep(g, part, 16, dict(p, active_blocks=0), max_sweeps=1)
    assert np.array_equal(p1, p2) and s1.tolist() == s2.tolist()

"""Pins of the oracle's multi-try FM (Sec. 4.2), against facts that do not
depend on it.

- A replay: the phase is restated here from the paper's description and
  driven by the oracle's event log.  At every pop the gains and targets of
  all queued vertices are recomputed from their definition (the k-way gain of
  Sec. 2.2), the keys come from the generator module's SplitMix64, the
  stopping rule is evaluated in the paper's form (p mu^2 > alpha sigma^2 +
  ln n, mean and variance of the gains since the last best state), and the
  rollback target is searched over the recorded states.  Every search start,
  move and end must agree, and so must the final partition.
- Closed forms: a vertex whose every neighbour lies in a third block moves
  there (a move no 2-way search can make); a unit path split in the middle
  has only zero-gain moves and keeps none; a move that would overload its
  target is not made.
- Invariants on random k-way partitions: the cut falls by exactly the gains
  of the kept moves and never rises from a balanced start, balanced blocks
  stay balanced, a vertex moves at most once per round.
- Composition: a batch with multi-try equals the pairwise refinements
  followed by the multi-try phase alone; a sweep with active blocks equals
  its restatement over batches.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle
from tests.helpers import csr_from_edges


def _sm(seed, n):
    # output number n of SplitMix64 started at seed, from the generator module
    return gen.splitmix64_stream((seed + (n - 1) * 0x9E3779B97F4A7C15) % 2**64, 1)[0]


def _key(seed, which, x):
    return _sm(seed, (1 << (40 + which)) + int(x) + 1)


def _lmax(g, k, eps_ppm):
    cV = int(g.vwgt.sum())
    return (1_000_000 + eps_ppm) * cV // (1_000_000 * k) + int(g.vwgt.max())


def _nbrs(g, v):
    return [(int(g.adjncy[e]), int(g.adjwgt[e])) for e in range(g.xadj[v], g.xadj[v + 1])]


def _gain(g, part, k, seed, v):
    """(gain, target) of v by definition, or None without a foreign neighbour."""
    w = {}
    for y, wy in _nbrs(g, v):
        w[int(part[y])] = w.get(int(part[y]), 0) + wy
    own = int(part[v])
    cands = [(w[P] - w.get(own, 0), P) for P in w if P != own]
    if not cands:
        return None
    best = max(gv for gv, _ in cands)
    tied = [P for gv, P in cands if gv == best]
    return best, min(tied, key=lambda P: _key(seed, 2, v * k + P))


def _stops(p, gains, alpha, n):
    mu = Fraction(sum(gains), p)
    var = Fraction(sum(x * x for x in gains), p) - mu * mu
    lhs = p * mu * mu - alpha * var
    assert abs(float(lhs) - math.log(n)) > 1e-4, "too close to the threshold to decide"
    return float(lhs) > math.log(n)


def _replay(g, part0, k, pairs, eps_ppm, alpha, seed, m):
    n = g.n
    part = part0.copy()
    lmax = _lmax(g, k, eps_ppm)
    bw = np.bincount(part, weights=g.vwgt, minlength=k).astype(np.int64)
    boundary = lambda v: any(part[y] != part[v] for y, _ in _nbrs(g, v))  # noqa: E731
    todos = []
    for a, b in pairs:
        t = [v for v in range(n) if part[v] in (a, b) and boundary(v)]
        t.sort(key=lambda v: ((_key(seed, 0, v) >> 32), v))
        todos.append(t)
    ev = list(m.events)
    pos = 0
    kept_total = 0
    for r, todo in enumerate(todos, 1):
        touched = set()
        for v in todo:
            if v in touched or not boundary(v):
                continue
            queue = [y for y in [v] + [y for y, _ in _nbrs(g, v)]
                     if y not in touched and _gain(g, part, k, seed, y) is not None]
            queue = list(dict.fromkeys(queue))
            touched |= set(queue)
            assert ev[pos] == (1, r, v, len(queue), 0), (ev[pos], r, v, len(queue))
            pos += 1
            over = int((bw > lmax).sum())
            states = [(over, 0)]  # (blocks above lmax, cut change) after each move
            moves, delta, since = [], 0, []
            while True:
                live = [(y, _gain(g, part, k, seed, y)) for y in queue]
                queue = [y for y, gt in live if gt is not None]  # no target: leaves
                if not queue:
                    break
                x, (gx, to) = max(((y, gt) for y, gt in live if gt is not None),
                                  key=lambda it: (it[1][0], _key(seed, 1, it[0])))
                queue.remove(x)
                if bw[to] + g.vwgt[x] > lmax:
                    continue
                frm = int(part[x])
                assert ev[pos] == (2, x, frm, to, gx), (ev[pos], (2, x, frm, to, gx))
                pos += 1
                part[x] = to
                bw[frm] -= g.vwgt[x]
                bw[to] += g.vwgt[x]
                delta -= gx
                moves.append((x, frm))
                st = (int((bw > lmax).sum()), delta)
                if st < min(states):
                    since = []
                else:
                    since.append(gx)
                states.append(st)
                if since and _stops(len(since), since, alpha, n):
                    break
                for y, _ in _nbrs(g, x):
                    if y not in touched and _gain(g, part, k, seed, y) is not None:
                        touched.add(y)
                        queue.append(y)
            best_n = states.index(min(states))  # earliest best state
            assert ev[pos] == (3, len(moves), best_n, 0, 0), (ev[pos], len(moves), best_n)
            pos += 1
            for x, frm in reversed(moves[best_n:]):
                bw[part[x]] -= g.vwgt[x]
                bw[frm] += g.vwgt[x]
                part[x] = frm
            kept_total += best_n
    assert pos == len(ev)
    assert np.array_equal(part, m.part)
    assert m.stats["kept"] == kept_total


def _case(seed, n=700, k=6, noise=0.08, wmax=1):
    g = gen.rgg(n, 2, 6.0, seed, 1, wmax)
    part = gen.rcb(g, k)
    gen.global_noise(g, part, noise, seed)
    return g, part


@pytest.mark.parametrize("seed", range(12))
def test_replay_random_kway(seed):
    k = 6
    g, part = _case(300 + seed, n=500 + 40 * seed, k=k, wmax=1 + seed % 3)
    pairs = [(0, 1), (2, 3), (4, 5)] if seed % 2 else [(1, 4), (0, 3)]
    alpha = (1, 4, 10)[seed % 3]
    m = oracle.multitry(g, part, k, pairs, 30000, alpha, 1000 + seed)
    assert m.stats["searches"] > 0
    _replay(g, part, k, pairs, 30000, alpha, 1000 + seed, m)


def test_replay_with_overloaded_start():
    """A start with an overloaded block: moves out of it are preferred by the
    rollback (fewer blocks above L_max first)."""
    k = 4
    g, part = _case(77, n=600, k=k)
    heavy = np.nonzero(part == 2)[0][:40]
    part[heavy] = 0  # block 0 grows past L_max
    lmax = _lmax(g, k, 30000)
    assert np.bincount(part, weights=g.vwgt, minlength=k)[0] > lmax
    m = oracle.multitry(g, part, k, [(0, 1), (2, 3)], 30000, 10, 5)
    _replay(g, part, k, [(0, 1), (2, 3)], 30000, 10, 5, m)


def test_third_block_move():
    """Vertex 0 of block 0 has its three neighbours in block 2; the round of
    pair (0, 1) moves it there (gain 3), cut 3 -> 0."""
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (4, 5), (5, 6), (1, 7), (7, 8), (4, 8)]
    g = csr_from_edges(9, edges)
    part = np.array([0, 2, 2, 2, 1, 1, 1, 2, 2], dtype=np.int32)
    # blocks: 0 = {0}, 1 = {4,5,6}, 2 = {1,2,3,7,8}; eps large so nothing overloads
    m = oracle.multitry(g, part, 3, [(0, 1)], 1_000_000, 10, 3)
    assert m.part[0] == 2
    assert oracle.total_cut(g, m.part) == oracle.total_cut(g, part) - 3
    assert m.kept == [m.stats["kept"]] and m.stats["kept"] >= 1
    assert m.changed[0] and m.changed[2]


def test_unit_path_zero_gains_keep_nothing():
    """A unit path split in the middle, eps 0 (L_max = 21): the one move the
    balance allows has gain 0 (one cut edge before and after), so the best
    state stays the start and nothing is kept."""
    n = 40
    g = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    part = (np.arange(n) >= n // 2).astype(np.int32)
    assert _lmax(g, 2, 0) == 21
    m = oracle.multitry(g, part, 2, [(0, 1)], 0, 10, 9)
    moves = [e for e in m.events if e[0] == 2]
    assert moves and all(e[4] == 0 for e in moves)
    assert m.stats["kept"] == 0 and np.array_equal(m.part, part)


def test_move_into_a_full_block_is_not_made():
    """Vertex 0 would gain 3 by joining block 2, but block 2 sits at L_max:
    the move is not made."""
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (4, 5), (5, 6)]
    g = csr_from_edges(7, edges)
    part = np.array([0, 2, 2, 2, 1, 1, 0], dtype=np.int32)
    # c(V) = 7, k = 3, eps 0: L_max = floor(7 / 3) + 1 = 3 = c(block 2)
    assert _lmax(g, 3, 0) == 3
    m = oracle.multitry(g, part, 3, [(0, 1)], 0, 10, 3)
    assert m.part[0] == 0
    assert not any(e[0] == 2 and e[1] == 0 for e in m.events)


@pytest.mark.parametrize("seed", range(8))
def test_invariants(seed):
    k = 8
    g, part = _case(500 + seed, n=3000, k=k, noise=0.05, wmax=3)
    pairs = [(0, 1), (2, 3), (4, 5), (6, 7)]
    lmax = _lmax(g, k, 30000)
    bw0 = np.bincount(part, weights=g.vwgt, minlength=k)
    m = oracle.multitry(g, part, k, pairs, 30000, 10, seed)
    cut0, cut1 = oracle.total_cut(g, part), oracle.total_cut(g, m.part)
    # the cut falls by the gains of the kept moves
    gains, i, cur = 0, 0, []
    for e in m.events:
        if e[0] == 1:
            cur = []
        elif e[0] == 2:
            cur.append(e[4])
        else:
            gains += sum(cur[:e[2]])
    assert cut0 - cut1 == gains
    if np.all(bw0 <= lmax):
        assert cut1 <= cut0
    bw1 = np.bincount(m.part, weights=g.vwgt, minlength=k)
    assert np.all(bw1[bw0 <= lmax] <= lmax)
    # each vertex moves at most once per round
    rnd, seen = 0, set()
    for e in m.events:
        if e[0] == 1 and e[1] != rnd:
            rnd, seen = e[1], set()
        if e[0] == 2:
            assert e[1] not in seen
            seen.add(e[1])
    # a vertex that changed blocks flags both of them
    moved = m.part != part
    assert np.all(m.changed[part[moved]]) and np.all(m.changed[m.part[moved]])


@pytest.mark.parametrize("seed", range(4))
def test_batch_is_pairwise_then_multitry(seed):
    k = 8
    g, part = _case(900 + seed, n=4000, k=k, noise=0.03)
    edges, colour = oracle.quotient_colouring(g, part, k)
    pairs = [tuple(e) for e, c in zip(edges.tolist(), colour.tolist()) if c == 0]
    base = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=1, max_iters=8,
                eps_ppm=30000)
    rc, res0, tr0, p0 = oracle.refine_batch(g, part, k, pairs, base)
    rc1, res1, tr1, p1 = oracle.refine_batch(g, part, k, pairs, dict(base, mt_alpha=10, mt_seed=7))
    assert rc == 0 and rc1 == 0 and tr1 == tr0
    for r0, r1 in zip(res0, res1):
        assert {x: r0[x] for x in r0 if x != "mt_kept"} == {x: r1[x] for x in r1 if x != "mt_kept"}
    m = oracle.multitry(g, p0, k, pairs, 30000, 10, 7)
    assert np.array_equal(p1, m.part)
    assert [r["mt_kept"] for r in res1] == m.kept


def test_sweep_with_multitry_and_active_blocks():
    """The sweep restated over batches: a pair changed when its pairwise
    improvement did or its multi-try round kept a move; the next sweep's
    active blocks are the changed pairs' blocks and the blocks a kept move
    left or entered."""
    k = 8
    g, part = _case(44, n=3000, k=k, noise=0.04)
    p = dict(area_mode=0, depth=0, alpha=4, alpha_max=4, adaptive=1, max_iters=6,
             eps_ppm=30000, mt_alpha=10, mt_seed=2, active_blocks=1)
    cur = part.copy()
    active = np.ones(k, dtype=bool)
    sweeps = solves = changed_total = 0
    for _ in range(4):
        edges, colour = oracle.quotient_colouring(g, cur, k)
        nxt = np.zeros(k, dtype=bool)
        changed = 0
        for c in sorted(set(colour.tolist())):
            pairs = [tuple(e) for e, cc in zip(edges.tolist(), colour.tolist())
                     if cc == c and (active[e[0]] or active[e[1]])]
            if not pairs:
                continue
            before = cur.copy()
            rc, res, _, after_pairwise = oracle.refine_batch(g, cur, k, pairs,
                                                            dict(p, mt_alpha=0))
            m = oracle.multitry(g, after_pairwise, k, pairs, 30000, 10, 2)
            rc2, res2, _, cur = oracle.refine_batch(g, before, k, pairs, p)
            assert np.array_equal(cur, m.part)
            for (a, b), r, kept in zip(pairs, res, m.kept):
                solves += r["iters"]
                if r["status"] == oracle.ST_ACCEPTED:
                    nxt[a] = nxt[b] = True
                if r["status"] == oracle.ST_ACCEPTED or kept > 0:
                    changed += 1
            nxt |= m.changed
        sweeps += 1
        changed_total += changed
        if changed == 0:
            break
        active = nxt
    rc, tc, stats, got = oracle.sweep(g, part, k, p, max_sweeps=4)
    assert rc == 0 and np.array_equal(got, cur)
    assert stats[0] == sweeps and stats[1] == solves and stats[2] == changed_total
    assert tc == oracle.total_cut(g, cur)

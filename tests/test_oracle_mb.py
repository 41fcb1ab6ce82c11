"""Pins of the oracle's most balanced minimum cut (Sec. 4.1.1) against facts
that do not depend on it: published SplitMix64 outputs and a second
implementation of that generator, brute-force strongly connected components
and scipy's, brute-force enumeration of every cut of small networks (the
Picard-Queyranne correspondence: minimum cuts = closed sets of the residual
graph between the source closure and the sink closure), the exact optimum on
networks whose minimum cuts form a chain, the sweep order on an antichain,
and a ladder whose most balanced cut is known in closed form."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import gen
import oracle
from tests.helpers import csr_from_edges


def _key(seed, r, gid):
    # counter layout of the sweep keys: output number r * 2^32 + id + 1
    return _sm(seed, (r << 32) + gid + 1)


def _sm(seed, n):
    # output number n of SplitMix64 started at seed = first output of the
    # generator started at seed + (n - 1) * gamma
    return gen.splitmix64_stream((seed + (n - 1) * 0x9E3779B97F4A7C15) % 2**64, 1)[0]


def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 seeded with 0, as printed by its
    # reference implementation (fixture with its citation)
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for n, hexval in rows:
        assert oracle.splitmix64(0, int(n)) == int(hexval, 16)


@pytest.mark.parametrize("seed", [1, 7, 2**31 + 5, 2**64 - 1])
def test_splitmix64_matches_generator_module(seed):
    ref = gen.splitmix64_stream(seed, 20)
    assert [oracle.splitmix64(seed, n) for n in range(1, 21)] == ref
    assert oracle.splitmix64(seed, (3 << 32) + 11) == _sm(seed, (3 << 32) + 11)


# ------------------------------------------------------------------ SCC ---

def _closure(nn, tails, heads):
    r = np.eye(nn, dtype=bool)
    r[tails, heads] = True
    for k in range(nn):  # Warshall
        r |= r[:, [k]] & r[[k], :]
    return r


@pytest.mark.parametrize("seed", range(30))
def test_scc_vs_brute_force_and_scipy(seed):
    rng = np.random.default_rng(seed)
    nn = int(rng.integers(1, 16))
    m = int(rng.integers(0, 3 * nn + 1))
    tails = rng.integers(0, nn, m)
    heads = rng.integers(0, nn, m)
    comp = oracle.scc(nn, tails, heads)
    r = _closure(nn, tails, heads)
    same = r & r.T
    assert np.array_equal(comp[:, None] == comp[None, :], same)
    g = csr_matrix((np.ones(m), (tails, heads)), shape=(nn, nn))
    _, lab = connected_components(g, directed=True, connection="strong")
    assert np.array_equal(lab[:, None] == lab[None, :], same)


# -------------------------------------------------------- minimum cuts ---

def _random_corridor_network(rng, inner):
    """s = inner, t = inner + 1; undirected inner edges as two arcs of equal
    capacity, infinite arcs s -> some inner nodes and some inner nodes -> t
    (the shape of the corridor network), node weights >= 0."""
    s, t = inner, inner + 1
    arcs = []
    for u in range(inner):
        for v in range(u + 1, inner):
            if rng.random() < 0.35:
                c = int(rng.integers(1, 4))
                arcs += [(u, v, c), (v, u, c)]
    big = 10**6
    srcs = rng.choice(inner, size=max(1, inner // 4), replace=False)
    rest = [v for v in range(inner) if v not in set(srcs.tolist())]
    snks = rng.choice(rest, size=max(1, len(rest) // 4), replace=False)
    arcs += [(s, int(v), big) for v in srcs] + [(int(v), t, big) for v in snks]
    w = np.concatenate([rng.integers(0, 6, inner), [0, 0]])
    return s, t, arcs, w


def _all_cuts(nn, arcs, s, t):
    others = [v for v in range(nn) if v not in (s, t)]
    m = len(others)
    masks = np.arange(1 << m, dtype=np.int64)
    side = np.zeros((1 << m, nn), dtype=bool)
    for j, v in enumerate(others):
        side[:, v] = (masks >> j) & 1
    side[:, s] = True
    tl = np.array([a[0] for a in arcs], dtype=np.int64)
    hd = np.array([a[1] for a in arcs], dtype=np.int64)
    cp = np.array([a[2] for a in arcs], dtype=np.int64)
    cap = (side[:, tl] & ~side[:, hd]).astype(np.int64) @ cp
    return side, cap


def _bal(side, w, base_s, base_t):
    ws = side.astype(np.int64) @ w
    return np.maximum(base_s + ws, base_t + (w.sum() - ws))


def _run(nn, arcs, s, t, w, base_s, base_t, reps, seed, gid=None):
    tl, hd, cp = zip(*arcs)
    if gid is None:
        gid = np.arange(nn)
    return oracle.mbcut(nn, tl, hd, cp, s, t, w, gid, base_s, base_t, reps, seed)


@pytest.mark.parametrize("seed", range(40))
def test_min_cuts_are_the_closed_sets_between_the_closures(seed):
    rng = np.random.default_rng(100 + seed)
    inner = int(rng.integers(3, 13))
    s, t, arcs, w = _random_corridor_network(rng, inner)
    nn = inner + 2
    base_s, base_t = int(rng.integers(0, 20)), int(rng.integers(0, 20))
    side, cap = _all_cuts(nn, arcs, s, t)
    best = cap.min()
    mins = side[cap == best]
    res = _run(nn, arcs, s, t, w, base_s, base_t, 4, seed)
    assert res.flow == best
    # smallest and largest minimum source sides
    assert np.array_equal(res.smin, mins.all(axis=0))
    assert np.array_equal(res.cls == 0, mins.all(axis=0))
    assert np.array_equal(res.cls != 2, mins.any(axis=0))
    # two remaining nodes share a component iff no minimum cut separates them
    rem = np.where(res.cls == 1)[0]
    for i in rem:
        for j in rem:
            insep = bool(np.all(mins[:, i] == mins[:, j]))
            assert (res.comp[i] == res.comp[j]) == insep
    # the chosen side is a minimum cut, balanced at least as well as both
    # extreme minimum cuts, and no better than the best minimum cut
    bal = _bal(mins, w, base_s, base_t)
    got = _bal(res.src[None, :], w, base_s, base_t)[0]
    assert any(np.array_equal(res.src, m) for m in mins)
    assert got <= _bal(res.smin[None, :], w, base_s, base_t)[0]
    assert got <= _bal((res.cls != 2)[None, :], w, base_s, base_t)[0]
    assert got >= bal.min()
    if res.info["reduced"] > 0:
        assert res.info["best_bal"] == got


@pytest.mark.parametrize("seed", range(10))
def test_no_sweeps_keeps_the_smallest_source_set(seed):
    rng = np.random.default_rng(300 + seed)
    s, t, arcs, w = _random_corridor_network(rng, 10)
    res = _run(12, arcs, s, t, w, 0, 0, 0, seed)
    assert np.array_equal(res.src, res.smin)


@pytest.mark.parametrize("seed", range(20))
def test_chain_of_minimum_cuts_gives_the_optimum(seed):
    """On a path s - v1 - ... - vk - t every minimum cut is one of its
    lightest edges, so the minimum cuts form a chain, every topological order
    is the same and one sweep visits all of them: the result is the most
    balanced minimum cut, the one with the larger source side on ties."""
    rng = np.random.default_rng(500 + seed)
    k = int(rng.integers(2, 13))
    s, t = k, k + 1
    nodes = [s] + list(range(k)) + [t]
    caps = rng.integers(1, 3, k + 1)
    arcs = []
    for (u, v), c in zip(zip(nodes[:-1], nodes[1:]), caps):
        arcs += [(u, v, int(c)), (v, u, int(c))]
    w = np.concatenate([rng.integers(0, 6, k), [0, 0]])
    base_s, base_t = int(rng.integers(0, 10)), int(rng.integers(0, 10))
    side, cap = _all_cuts(k + 2, arcs, s, t)
    mins = side[cap == cap.min()]
    bal = _bal(mins, w, base_s, base_t)
    cand = mins[bal == bal.min()]
    want = cand[np.argmax(cand.sum(axis=1))]
    res = _run(k + 2, arcs, s, t, w, base_s, base_t, 2, seed)
    assert np.array_equal(res.src, want)


@pytest.mark.parametrize("seed", range(12))
def test_antichain_sweep_follows_ascending_keys(seed):
    """Nodes x_i with saturated arcs s -> x_i -> t are independent remaining
    components: a sweep's topological order is the ascending order of their
    keys, and the chosen cut the first best prefix over the sweeps."""
    rng = np.random.default_rng(700 + seed)
    k = int(rng.integers(1, 9))
    reps = int(rng.integers(1, 4))
    mseed = int(rng.integers(0, 2**32))
    s, t = k, k + 1
    arcs = [(s, i, 1) for i in range(k)] + [(i, t, 1) for i in range(k)]
    w = np.concatenate([rng.integers(0, 9, k), [0, 0]])
    gid = np.concatenate([rng.permutation(1000)[:k], [2**31 - 1, 2**31 - 1]])
    base_s, base_t = int(rng.integers(0, 15)), int(rng.integers(0, 15))
    best = None
    for r in range(reps):
        order = sorted(range(k), key=lambda i: _key(mseed, r, int(gid[i])))
        src = np.ones(k + 2, dtype=bool)
        src[t] = False
        for j in range(k + 1):
            if j > 0:
                src[order[j - 1]] = False
            b = _bal(src[None, :], w, base_s, base_t)[0]
            if best is None or b < best[0]:
                best = (b, src.copy())
    res = _run(k + 2, arcs, s, t, w, base_s, base_t, reps, mseed, gid=gid)
    assert res.info["reduced"] == k
    assert np.array_equal(res.src, best[1])


@pytest.mark.parametrize("k", [2049, 3001, 5000])
def test_long_chain_beyond_two_thousand_components(k):
    """A path s - v1 - ... - vk - t of unit capacities: after the flow every
    inner node is a component of its own (more than 2,048 of them), the
    minimum cuts are the k + 1 prefix cuts, and the sweep must still run:
    the chosen source side {s, v1..vj} minimises max(base_s + j, base_t +
    k - j), the largest such j on ties (the sweep starts from the largest
    source side).  Unit weights make that j a closed form."""
    s, t = k, k + 1
    nodes = [s] + list(range(k)) + [t]
    arcs = []
    for u, v in zip(nodes[:-1], nodes[1:]):
        arcs += [(u, v, 1), (v, u, 1)]
    w = np.concatenate([np.ones(k, dtype=np.int64), [0, 0]])
    base_s, base_t = 7, 3
    res = _run(k + 2, arcs, s, t, w, base_s, base_t, 2, 11)
    assert res.flow == 1 and res.info["reduced"] == k
    bals = [max(base_s + j, base_t + k - j) for j in range(k + 1)]
    best = min(bals)
    j = max(i for i, b in enumerate(bals) if b == best)
    want = np.zeros(k + 2, dtype=bool)
    want[:j] = True
    want[s] = True
    assert np.array_equal(res.src, want)


def test_wide_antichain_beyond_two_thousand_components():
    """2,500 independent components (saturated s -> x_i -> t arcs): one
    sweep moves them to the sink side in ascending key order; the chosen cut
    is the first best prefix of that order, computed here from the
    generator module's SplitMix64."""
    k, mseed = 2500, 2024
    rng = np.random.default_rng(4)
    s, t = k, k + 1
    arcs = [(s, i, 1) for i in range(k)] + [(i, t, 1) for i in range(k)]
    w = np.concatenate([rng.integers(0, 5, k), [0, 0]])
    gid = np.concatenate([rng.permutation(10 * k)[:k], [2**31 - 1, 2**31 - 1]])
    base_s, base_t = 0, 1000
    order = sorted(range(k), key=lambda i: _key(mseed, 0, int(gid[i])))
    ws, wt = base_s + int(w[:k].sum()), base_t
    best, bj = max(ws, wt), 0
    for j, i in enumerate(order, 1):
        ws -= int(w[i])
        wt += int(w[i])
        if max(ws, wt) < best:
            best, bj = max(ws, wt), j
    want = np.ones(k + 2, dtype=bool)
    want[t] = False
    want[order[:bj]] = False
    res = _run(k + 2, arcs, s, t, w, base_s, base_t, 1, mseed, gid=gid)
    assert res.info["reduced"] == k
    assert np.array_equal(res.src, want)


# ------------------------------------------------------- pair refinement --

def _ladder(cols):
    edges = []
    for c in range(cols):
        edges.append((c, cols + c))
        if c + 1 < cols:
            edges += [(c, c + 1), (cols + c + 1, cols + c)]
    return csr_from_edges(2 * cols, edges)


def test_ladder_most_balanced_cut_closed_form():
    """2 x 100 ladder, unit weights; block 0 = columns 0..39 plus the top
    vertex of column 40 (cut 3), eps 3 %, alpha = alpha' = 16.  The corridor
    spans columns 26..73, whose minimum cuts (value 2) are the vertical cuts;
    the most balanced one is between columns 49 and 50 (100 : 100), so the
    first solve applies it (cut 3 -> 2) and the second finds nothing better.
    The smallest source set instead cuts right behind the source border
    (block 0 far too light), which is infeasible."""
    cols = 100
    g = _ladder(cols)
    col = np.arange(2 * cols) % cols
    part = (col >= 40).astype(np.int32)
    part[40] = 0
    p = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=8,
             eps_ppm=30000, mb_reps=4, mb_seed=12345)
    o = oracle.refine_pair(g, part.copy(), 2, 0, 1, p)
    t0 = o.trace[0]
    assert (t0["flow"], t0["cut_before"], t0["cut_candidate"]) == (2, 3, 2)
    assert (t0["wa"], t0["wb"], t0["decision"]) == (100, 100, oracle.DEC_APPLY)
    assert np.array_equal(o.part, (col >= 50).astype(np.int32))
    assert o.result["cut_after"] == 2 and o.result["iters"] == 2
    assert o.trace[1]["decision"] == oracle.DEC_EQUAL
    q = dict(p, mb_reps=0)
    o2 = oracle.refine_pair(g, part.copy(), 2, 0, 1, q)
    assert o2.trace[0]["decision"] == oracle.DEC_INFEASIBLE
    assert o2.trace[0]["flow"] == 2


@pytest.mark.parametrize("seed", range(6))
def test_pair_solve_balance_not_worse_than_smallest_source_set(seed):
    """The first solve of a pair with and without sweeps: same corridor and
    flow, the same candidate cut, and a balance at least as good."""
    g = gen.rgg(3000, 2, 7.0, 40 + seed, 1, 3 if seed % 2 else 1)
    part = gen.rcb(g, 2, force_axis=0)
    gen.pair_swap_noise(g, part, 0.03, seed)
    p = dict(area_mode=0, depth=0, alpha=8, alpha_max=8, adaptive=0, max_iters=1,
             eps_ppm=30000)
    a = oracle.refine_pair(g, part.copy(), 2, 0, 1, dict(p, mb_reps=0))
    b = oracle.refine_pair(g, part.copy(), 2, 0, 1, dict(p, mb_reps=8, mb_seed=seed))
    ta, tb = a.trace[0], b.trace[0]
    for key in ("flow", "region_vertices", "region_edges", "cut_candidate", "cut_before"):
        assert ta[key] == tb[key], key
    assert max(tb["wa"], tb["wb"]) <= max(ta["wa"], ta["wb"])


# ------------------------------------ the largest minimum source side --

@pytest.mark.parametrize("seed", range(20))
def test_largest_source_side_is_the_union_of_minimum_source_sides(seed):
    """cut_side = 1: the candidate is every corridor vertex that cannot reach
    t, which brute force finds as the union of all minimum source sides of
    the corridor network; cut_side = 2 takes it only when the smallest source
    set is infeasible and it is feasible."""
    from tests.helpers import area_bound, corridor_by_sorting, l_max, pair_network, random_graph

    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(8, 18))
    g = random_graph(n, 0.3, 2000 + seed, wmax=3, vwmax=int(rng.choice([1, 4])))
    part = (rng.random(n) < 0.5).astype(np.int32)
    part[0], part[1] = 0, 1
    eps = int(rng.choice([30000, 300000, 1000000]))
    p = dict(area_mode=0, depth=0, alpha=4, alpha_max=4, adaptive=0, max_iters=1, eps_ppm=eps)
    ua = area_bound(g, part, 2, 1, 4, eps)
    ub = area_bound(g, part, 2, 0, 4, eps)
    in_a = corridor_by_sorting(g, part, 0, 1, 0, 0, ua)
    in_b = corridor_by_sorting(g, part, 1, 0, 0, 0, ub)
    nn, arcs, s, t, verts, border = pair_network(g, part, 0, 1, in_a, in_b)
    side, cap = _all_cuts(nn, arcs, s, t)
    mins = side[cap == cap.min()]
    union, inter = mins.any(axis=0), mins.all(axis=0)
    lmax = l_max(g, 2, eps)

    def weights(src):
        new = part.copy()
        for i, u in enumerate(verts):
            new[u] = 0 if src[i] else 1
        return int(g.vwgt[new == 0].sum()), int(g.vwgt[new == 1].sum()), new

    o1 = oracle.refine_pair(g, part.copy(), 2, 0, 1, dict(p, cut_side=1))
    got = np.array([o1.side[u] in (0, 2) for u in verts], dtype=bool)
    assert np.array_equal(got, union[: len(verts)])
    assert (o1.trace[0]["wa"], o1.trace[0]["wb"]) == weights(union)[:2]
    o2 = oracle.refine_pair(g, part.copy(), 2, 0, 1, dict(p, cut_side=2))
    w1, w2 = weights(inter)[:2], weights(union)[:2]
    feas = lambda w: max(w) <= lmax
    want = union if (not feas(w1) and feas(w2)) else inter
    got2 = np.array([o2.side[u] in (0, 2) for u in verts], dtype=bool)
    assert np.array_equal(got2, want[: len(verts)])

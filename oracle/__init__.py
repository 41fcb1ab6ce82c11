"""ORACLE -- test infrastructure, not part of the product.

ctypes binding of ``oracle.c``: a plain sequential CPU implementation of
max-flow min-cut pair refinement (Section 4.1 of the paper: bounded BFS
corridor, s-t network with infinite border arcs, max flow, smallest source set
from the residual graph, balance check, adaptive flow iterations), plus the
quotient-graph colouring sweep and the per-pair features of the learned area
factor.  With ``mb_reps > 0`` a solve takes the most balanced minimum cut of
Section 4.1.1 (residual strongly connected components, removal of the s and t
closures, sweeps along random topological orders) instead of the smallest
source set.  With ``mt_alpha > 0`` a batch ends with the multi-try FM phase of
Section 4.2 (rounds of localized k-way searches, one round per pair in pair
order).  Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the GPU library and never calls it.

``mlp_*`` below is the float64 reference of the small area-factor network
(8 -> 64 -> 64 -> 5, ReLU, softmax cross-entropy), written with numpy matmuls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DEC_APPLY, DEC_INFEASIBLE, DEC_EQUAL, DEC_NOT_ADJ = 1, 2, 3, 4
ST_ACCEPTED, ST_REJECTED, ST_NO_IMPROVEMENT, ST_NOT_ADJACENT = 1, 2, 3, 4


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p)]


class OrParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in
                ("area_mode", "depth", "alpha", "alpha_max", "adaptive", "max_iters", "eps_ppm",
                 "mb_reps", "mb_seed", "fm_limit", "fm_seed", "active_blocks", "cut_side",
                 "terminals", "mt_alpha", "mt_seed", "restart_alpha")]


class OrSolve(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("decision", ctypes.c_int32)] + [
        (f, ctypes.c_int64) for f in ("flow", "region_vertices", "region_edges", "source_side",
                                      "cut_before", "cut_candidate", "wa", "wb")]


class OrResult(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in
                ("status", "iters", "final_alpha", "applied", "iter_cap", "pad")] + [
        (f, ctypes.c_int64) for f in ("flow_value", "cut_before", "cut_after", "weight_a",
                                      "weight_b", "region_vertices", "region_edges", "mt_kept")]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    G, P = ctypes.POINTER(OrGraph), ctypes.POINTER(OrParams)
    lib.or_validate_graph.restype = i32
    lib.or_validate_graph.argtypes = [G]
    lib.or_maxflow.restype = i32
    lib.or_maxflow.argtypes = [i32, i64, vp, vp, vp, i32, i32, ctypes.POINTER(i64), vp]
    lib.or_refine_pair.restype = i32
    lib.or_refine_pair.argtypes = [G, vp, i32, i32, i32, P, ctypes.POINTER(OrResult), vp, vp]
    lib.or_refine_batch.restype = i32
    lib.or_refine_batch.argtypes = [G, vp, i32, vp, i32, P, vp, vp]
    lib.or_quotient_colouring.restype = i32
    lib.or_quotient_colouring.argtypes = [G, vp, i32, vp, vp, i32]
    lib.or_total_cut.restype = i64
    lib.or_total_cut.argtypes = [G, vp]
    lib.or_sweep.restype = i32
    lib.or_sweep.argtypes = [G, vp, i32, P, i32, ctypes.POINTER(i64), vp]
    lib.or_pair_features.restype = i32
    lib.or_pair_features.argtypes = [G, vp, i32, i32, i32, i32, vp]
    lib.or_pair_fm.restype = i32
    lib.or_pair_fm.argtypes = [G, vp, i32, i32, i32, i32, i32, ctypes.c_uint32, vp, vp]
    lib.or_multitry.restype = i32
    lib.or_multitry.argtypes = [G, vp, i32, vp, i32, i32, i32, ctypes.c_uint32, vp, vp, vp, vp,
                                i64, ctypes.POINTER(i64)]
    lib.or_splitmix64.restype = ctypes.c_uint64
    lib.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.or_scc.restype = i32
    lib.or_scc.argtypes = [i32, i64, vp, vp, vp]
    lib.or_mbcut.restype = i32
    lib.or_mbcut.argtypes = [i32, i64, vp, vp, vp, i32, i32, vp, vp, i64, i64, i32,
                             ctypes.c_uint32, ctypes.POINTER(i64), vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous
    return a.ctypes.data


class _Bound:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, graph):
        self.xadj = np.ascontiguousarray(graph.xadj, dtype=np.int32)
        self.adjncy = np.ascontiguousarray(graph.adjncy, dtype=np.int32)
        self.vwgt = np.ascontiguousarray(graph.vwgt, dtype=np.int32)
        self.adjwgt = np.ascontiguousarray(graph.adjwgt, dtype=np.int32)
        self.s = OrGraph(self.xadj.shape[0] - 1, _ptr(self.xadj), _ptr(self.adjncy),
                         _ptr(self.vwgt), _ptr(self.adjwgt))


def _i32(x: int) -> int:
    x = int(x) & 0xFFFFFFFF
    return x - (1 << 32) if x >= 1 << 31 else x


def _params(p: dict) -> OrParams:
    return OrParams(p.get("area_mode", 0), p.get("depth", 0), p["alpha"], p["alpha_max"],
                    p["adaptive"], p["max_iters"], p["eps_ppm"], p.get("mb_reps", 0),
                    _i32(p.get("mb_seed", 0)), p.get("fm_limit", 0), _i32(p.get("fm_seed", 0)),
                    p.get("active_blocks", 0), p.get("cut_side", 0), p.get("terminals", 0),
                    p.get("mt_alpha", 0), _i32(p.get("mt_seed", 0)), p.get("restart_alpha", 0))


def _struct_dict(s) -> dict:
    return {f: getattr(s, f) for f, _ in s._fields_ if f != "pad"}


def validate_graph(graph) -> bool:
    b = _Bound(graph)
    return _load().or_validate_graph(ctypes.byref(b.s)) == 0


def maxflow(nn: int, tails, heads, caps, s: int, t: int):
    """Max flow on a directed network; returns (value, reach) where reach[v]
    marks the smallest source set."""
    tails = np.ascontiguousarray(tails, dtype=np.int32)
    heads = np.ascontiguousarray(heads, dtype=np.int32)
    caps = np.ascontiguousarray(caps, dtype=np.int64)
    reach = np.zeros(nn, dtype=np.uint8)
    val = ctypes.c_int64(0)
    rc = _load().or_maxflow(nn, tails.shape[0], _ptr(tails), _ptr(heads), _ptr(caps), s, t,
                            ctypes.byref(val), _ptr(reach))
    if rc != 0:
        raise ValueError("or_maxflow: bad input")
    return int(val.value), reach.astype(bool)


def pair_fm(graph, part: np.ndarray, k: int, a: int, b: int, eps_ppm: int, limit: int,
            seed: int):
    """One 2-way FM pass with TopGain on blocks a, b (Sec. 2.2); returns
    (new partition, info dict, move log)."""
    bnd = _Bound(graph)
    out = np.ascontiguousarray(part, dtype=np.int32).copy()
    info = np.zeros(6, dtype=np.int64)
    log = np.zeros(max(1, bnd.s.n), dtype=np.int32)
    rc = _load().or_pair_fm(ctypes.byref(bnd.s), _ptr(out), k, a, b, eps_ppm, limit,
                            seed & 0xFFFFFFFF, _ptr(info), _ptr(log))
    if rc != 0:
        raise ValueError(f"or_pair_fm: {rc}")
    keys = ("cut_before", "cut_after", "steps", "kept", "weight_a", "weight_b")
    d = dict(zip(keys, info.tolist()))
    return out, d, log[: d["steps"]].copy()


@dataclass
class MultiTry:
    part: np.ndarray      # the partition after the phase
    stats: dict           # searches, moves, kept
    kept: list            # moves kept per pair
    changed: np.ndarray   # [k] bool: blocks a kept move left or entered
    events: list          # (1, round, start, start set size, 0) / (2, v, from, to, gain) /
                          # (3, moves, kept, 0, 0)


def multitry(graph, part: np.ndarray, k: int, pairs, eps_ppm: int, alpha: int, seed: int,
             max_events: int | None = 1 << 20) -> MultiTry:
    """The multi-try FM phase (Sec. 4.2) alone: one round per pair of the
    block-disjoint `pairs`, in their order; part is copied, not modified.
    max_events=None keeps no event log."""
    bnd = _Bound(graph)
    part = np.array(part, dtype=np.int32, copy=True)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    npairs = pr.shape[0] // 2
    stats = np.zeros(3, dtype=np.int64)
    kept = np.zeros(max(1, npairs), dtype=np.int64)
    chg = np.zeros(k, dtype=np.uint8)
    ev = np.zeros(5 * max_events if max_events else 1, dtype=np.int64)
    nev = ctypes.c_int64(0)
    rc = _load().or_multitry(ctypes.byref(bnd.s), _ptr(part), k, _ptr(pr) if npairs else None,
                             npairs, eps_ppm, alpha, seed & 0xFFFFFFFF, _ptr(stats), _ptr(kept),
                             _ptr(chg), _ptr(ev) if max_events else None,
                             ev.shape[0] if max_events else 0, ctypes.byref(nev))
    if rc != 0:
        raise ValueError(f"or_multitry: {rc}")
    if max_events and nev.value > ev.shape[0]:
        raise ValueError("or_multitry: event log too small")
    if not max_events:
        nev.value = 0
    events = [tuple(int(x) for x in r) for r in ev[:nev.value].reshape(-1, 5)]
    return MultiTry(part, dict(zip(("searches", "moves", "kept"), stats.tolist())),
                    kept[:npairs].tolist(), chg.astype(bool), events)


def splitmix64(seed: int, n: int) -> int:
    """Output number n >= 1 of SplitMix64 started at `seed`."""
    return int(_load().or_splitmix64(seed & (2**64 - 1), n & (2**64 - 1)))


def scc(nn: int, tails, heads) -> np.ndarray:
    """Strongly connected components (Tarjan) of a directed graph: comp[v]."""
    tails = np.ascontiguousarray(tails, dtype=np.int32)
    heads = np.ascontiguousarray(heads, dtype=np.int32)
    comp = np.zeros(nn, dtype=np.int32)
    nc = _load().or_scc(nn, tails.shape[0], _ptr(tails), _ptr(heads), _ptr(comp))
    if nc < 0:
        raise ValueError("or_scc: bad input")
    return comp


@dataclass
class MBCut:
    flow: int
    src: np.ndarray    # chosen source side (bool [nn])
    smin: np.ndarray   # smallest source set
    cls: np.ndarray    # 0 with s, 1 remaining, 2 with t
    comp: np.ndarray   # residual strongly connected component
    info: dict


def mbcut(nn: int, tails, heads, caps, s: int, t: int, w, gid, base_s: int, base_t: int,
          reps: int, seed: int) -> MBCut:
    """Max flow, then the most balanced minimum cut (Sec. 4.1.1) of a directed
    network; the balance of a source side C is max(base_s + w(C),
    base_t + w(V minus C))."""
    tails = np.ascontiguousarray(tails, dtype=np.int32)
    heads = np.ascontiguousarray(heads, dtype=np.int32)
    caps = np.ascontiguousarray(caps, dtype=np.int64)
    w = np.ascontiguousarray(w, dtype=np.int64)
    gid = np.ascontiguousarray(gid, dtype=np.int32)
    src = np.zeros(nn, dtype=np.uint8)
    smin = np.zeros(nn, dtype=np.uint8)
    cls = np.zeros(nn, dtype=np.int8)
    comp = np.zeros(nn, dtype=np.int32)
    info = np.zeros(6, dtype=np.int64)
    val = ctypes.c_int64(0)
    rc = _load().or_mbcut(nn, tails.shape[0], _ptr(tails), _ptr(heads), _ptr(caps), s, t,
                          _ptr(w), _ptr(gid), base_s, base_t, reps, seed & 0xFFFFFFFF,
                          ctypes.byref(val), _ptr(src), _ptr(smin), _ptr(cls), _ptr(comp),
                          _ptr(info))
    if rc != 0:
        raise ValueError("or_mbcut: bad input")
    keys = ("ncomp", "reduced", "reduced_arcs", "best_rep", "best_pos", "best_bal")
    return MBCut(int(val.value), src.astype(bool), smin.astype(bool), cls, comp,
                 dict(zip(keys, info.tolist())))


@dataclass
class PairOutcome:
    rc: int
    result: dict
    trace: list
    side: np.ndarray | None
    part: np.ndarray


def refine_pair(graph, part: np.ndarray, k: int, a: int, b: int, params: dict,
                want_side: bool = True) -> PairOutcome:
    """Adaptive flow iterations on one pair; part is copied, not modified."""
    bnd = _Bound(graph)
    p = _params(params)
    part = np.array(part, dtype=np.int32, copy=True)
    res = OrResult()
    trace = (OrSolve * max(1, params["max_iters"]))()
    side = np.zeros(bnd.s.n, dtype=np.int8) if want_side else None
    rc = _load().or_refine_pair(ctypes.byref(bnd.s), _ptr(part), k, a, b, ctypes.byref(p),
                                ctypes.byref(res), _ptr(side) if want_side else None,
                                ctypes.addressof(trace))
    tr = [_struct_dict(trace[i]) for i in range(res.iters)]
    return PairOutcome(rc, _struct_dict(res), tr, side, part)


def refine_batch(graph, part: np.ndarray, k: int, pairs, params: dict):
    """Pairs of one matching in the given order; returns (rc, results,
    traces, new part)."""
    bnd = _Bound(graph)
    p = _params(params)
    part = np.array(part, dtype=np.int32, copy=True)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    npairs = pr.shape[0] // 2
    res = (OrResult * max(1, npairs))()
    mi = max(1, params["max_iters"])
    trace = (OrSolve * max(1, npairs * mi))()
    rc = _load().or_refine_batch(ctypes.byref(bnd.s), _ptr(part), k, _ptr(pr) if npairs else None,
                                 npairs, ctypes.byref(p), ctypes.addressof(res),
                                 ctypes.addressof(trace))
    results = [_struct_dict(res[i]) for i in range(npairs)]
    traces = [[_struct_dict(trace[i * mi + j]) for j in range(results[i]["iters"])]
              for i in range(npairs)] if rc == 0 else []
    return rc, results, traces, part


def quotient_colouring(graph, part: np.ndarray, k: int):
    """Returns (edges [ne,2], colours [ne])."""
    bnd = _Bound(graph)
    part = np.ascontiguousarray(part, dtype=np.int32)
    maxe = k * (k - 1) // 2 + 1
    edges = np.zeros(2 * maxe, dtype=np.int32)
    colour = np.zeros(maxe, dtype=np.int32)
    ne = _load().or_quotient_colouring(ctypes.byref(bnd.s), _ptr(part), k, _ptr(edges),
                                       _ptr(colour), maxe)
    if ne < 0:
        raise RuntimeError("or_quotient_colouring failed")
    return edges[:2 * ne].reshape(ne, 2), colour[:ne]


def total_cut(graph, part: np.ndarray) -> int:
    bnd = _Bound(graph)
    part = np.ascontiguousarray(part, dtype=np.int32)
    return int(_load().or_total_cut(ctypes.byref(bnd.s), _ptr(part)))


def sweep(graph, part: np.ndarray, k: int, params: dict, max_sweeps: int):
    """Returns (rc, total_cut, stats[sweeps, solves, changed pairs, region edges], part)."""
    bnd = _Bound(graph)
    p = _params(params)
    part = np.array(part, dtype=np.int32, copy=True)
    stats = np.zeros(4, dtype=np.int64)
    tc = ctypes.c_int64(0)
    rc = _load().or_sweep(ctypes.byref(bnd.s), _ptr(part), k, ctypes.byref(p), max_sweeps,
                          ctypes.byref(tc), _ptr(stats))
    return rc, int(tc.value), stats, part


def pair_features(graph, part: np.ndarray, k: int, a: int, b: int, eps_ppm: int) -> np.ndarray:
    bnd = _Bound(graph)
    part = np.ascontiguousarray(part, dtype=np.int32)
    f = np.zeros(8, dtype=np.float64)
    rc = _load().or_pair_features(ctypes.byref(bnd.s), _ptr(part), k, a, b, eps_ppm, _ptr(f))
    if rc != 0:
        raise ValueError("bad pair")
    return f


# ---------------------------------------------------------------- MLP ---
# float64 reference of the area-factor network: h1 = relu(x W1 + b1),
# h2 = relu(h1 W2 + b2), z = h2 W3 + b3, p = softmax(z), loss = mean CE.
# Weights are stored row-major [in, out].

ALPHAS = (1, 2, 4, 8, 16)


def mlp_forward(params: dict, x: np.ndarray):
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ params["W1"] + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ params["W3"] + params["b3"]
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (x, a1, h1, a2, h2, z)


def _mlp_backward(params: dict, cache, dz):
    x, a1, h1, a2, h2, z = cache
    g = {"W3": h2.T @ dz, "b3": dz.sum(axis=0)}
    dh2 = dz @ params["W3"].T
    da2 = dh2 * (a2 > 0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"].T
    da1 = dh1 * (a1 > 0)
    g["W1"] = x.T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def mlp_loss_grad_cost(params: dict, x: np.ndarray, costs: np.ndarray):
    """Mean expected cost over the samples, sum_c p_c costs_c with the softmax
    p, and its gradient: dL/dz_j = p_j (costs_j - sum_c p_c costs_c) / n."""
    p, cache = mlp_forward(params, x)
    costs = np.asarray(costs, dtype=np.float64)
    nrows = p.shape[0]
    pc = (p * costs).sum(axis=1, keepdims=True)
    loss = float(pc.mean())
    dz = p * (costs - pc) / nrows
    return loss, _mlp_backward(params, cache, dz)


def mlp_loss_grad(params: dict, x: np.ndarray, labels: np.ndarray):
    """Mean softmax cross-entropy and its gradient (hand-written backward)."""
    p, (x, a1, h1, a2, h2, z) = mlp_forward(params, x)
    nrows = x.shape[0]
    labels = np.asarray(labels, dtype=np.int64)
    loss = -np.mean(np.log(p[np.arange(nrows), labels]))
    dz = p.copy()
    dz[np.arange(nrows), labels] -= 1.0
    dz /= nrows
    g = {"W3": h2.T @ dz, "b3": dz.sum(axis=0)}
    dh2 = dz @ params["W3"].T
    da2 = dh2 * (a2 > 0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"].T
    da1 = dh1 * (a1 > 0)
    g["W1"] = x.T @ da1
    g["b1"] = da1.sum(axis=0)
    return loss, g

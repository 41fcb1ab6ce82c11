"""Seeded synthetic inputs (graphs, partitions, noise) for the flow-refinement
path.  This module builds inputs only; it holds none of the refinement
arithmetic, so both the CPU oracle and the GPU library are fed from it.

The workloads stand in for the paper's instance suites (Walshaw archive, road
networks, rggX / DelaunayX; Section 6, "Instances"), which are not available
here.  The random geometric graph keeps the rggX family shape (uniform points
in the unit square or cube, edge iff distance below a radius) with the radius
chosen for a target mean degree.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def build() -> str:
    """Compile gen.c into libgen.so (gcc, host only)."""
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _GenGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("narcs", ctypes.c_int64),
        ("radius", ctypes.c_double),
        ("xadj", ctypes.POINTER(ctypes.c_int32)),
        ("adjncy", ctypes.POINTER(ctypes.c_int32)),
        ("adjwgt", ctypes.POINTER(ctypes.c_int32)),
        ("coords", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gen_splitmix64_next.restype = ctypes.c_uint64
    lib.gen_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
    lib.gen_edge_hash.restype = ctypes.c_uint64
    lib.gen_edge_hash.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
    lib.gen_rgg.restype = ctypes.c_int
    lib.gen_rgg.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                            ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_GenGraph)]
    lib.gen_free.restype = None
    lib.gen_free.argtypes = [ctypes.POINTER(_GenGraph)]
    lib.gen_rcb.restype = ctypes.c_int
    lib.gen_rcb.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                            ctypes.c_int32, ctypes.c_int32, i32p]
    for name in ("gen_pair_swap_noise", "gen_global_noise"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_double, ctypes.c_uint64]
    _lib = lib
    return lib


def _i32p(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ---------------------------------------------------------------- PRNG ---

def splitmix64_stream(seed: int, count: int) -> list[int]:
    """Pure-Python splitmix64 (Steele, Lea, Flood 2014); used by tests to pin
    the C generator."""
    out, s = [], seed & MASK64
    for _ in range(count):
        s = (s + GOLDEN) & MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def splitmix64_c(seed: int, count: int) -> list[int]:
    lib = _load()
    st = ctypes.c_uint64(seed & MASK64)
    return [lib.gen_splitmix64_next(ctypes.byref(st)) for _ in range(count)]


# -------------------------------------------------------------- graphs ---

@dataclass
class Graph:
    """Undirected graph as symmetric CSR with int32 weights."""
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray
    vwgt: np.ndarray
    coords: np.ndarray | None = None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xadj.shape[0] - 1)

    @property
    def narcs(self) -> int:
        return int(self.adjncy.shape[0])


def grid2d(rows: int, cols: int) -> Graph:
    """rows x cols 4-neighbour grid, vertex id = cols*y + x, unit weights,
    adjacency sorted by id."""
    n = rows * cols
    ys, xs = np.divmod(np.arange(n, dtype=np.int64), cols)
    nbrs = []
    for dy, dx in ((-1, 0), (0, -1), (0, 1), (1, 0)):  # ascending id order
        ok = (ys + dy >= 0) & (ys + dy < rows) & (xs + dx >= 0) & (xs + dx < cols)
        nbrs.append(np.where(ok, (ys + dy) * cols + (xs + dx), -1))
    nb = np.stack(nbrs, axis=1)
    deg = (nb >= 0).sum(axis=1)
    xadj = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(deg, out=xadj[1:])
    adjncy = nb[nb >= 0].astype(np.int32)
    coords = np.stack([(xs + 0.5) / cols, (ys + 0.5) / rows], axis=1)
    return Graph(xadj, adjncy, np.ones_like(adjncy), np.ones(n, dtype=np.int32), coords,
                 f"grid{rows}x{cols}")


def rgg(n: int, dim: int, mean_degree: float, seed: int, wlo: int = 1, whi: int = 1) -> Graph:
    lib = _load()
    g = _GenGraph()
    rc = lib.gen_rgg(n, dim, float(mean_degree), seed & MASK64, wlo, whi, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError("gen_rgg failed")
    try:
        xadj = np.ctypeslib.as_array(g.xadj, shape=(n + 1,)).copy()
        m = int(g.narcs)
        adjncy = np.ctypeslib.as_array(g.adjncy, shape=(max(m, 1),))[:m].copy()
        adjwgt = np.ctypeslib.as_array(g.adjwgt, shape=(max(m, 1),))[:m].copy()
        coords = np.ctypeslib.as_array(g.coords, shape=(n * dim,)).reshape(n, dim).copy()
    finally:
        lib.gen_free(ctypes.byref(g))
    return Graph(xadj, adjncy, adjwgt, np.ones(n, dtype=np.int32), coords,
                 f"rgg{dim}d_n{n}_deg{mean_degree:g}_s{seed}")


def rcb(graph: Graph, k: int, force_axis: int = -1) -> np.ndarray:
    lib = _load()
    coords = np.ascontiguousarray(graph.coords, dtype=np.float64)
    part = np.zeros(graph.n, dtype=np.int32)
    rc = lib.gen_rcb(graph.n, coords.shape[1], coords.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     k, force_axis, _i32p(part))
    if rc != 0:
        raise RuntimeError("gen_rcb failed")
    return part


def pair_swap_noise(graph: Graph, part: np.ndarray, frac: float, seed: int) -> int:
    lib = _load()
    return int(lib.gen_pair_swap_noise(graph.n, _i32p(graph.xadj), _i32p(graph.adjncy),
                                       _i32p(part), frac, seed & MASK64))


def global_noise(graph: Graph, part: np.ndarray, frac: float, seed: int) -> int:
    lib = _load()
    return int(lib.gen_global_noise(graph.n, _i32p(graph.xadj), _i32p(graph.adjncy),
                                    _i32p(part), frac, seed & MASK64))


def edge_weight_hash(seed: int, u: int, v: int) -> int:
    return int(_load().gen_edge_hash(seed & MASK64, u, v))


# ------------------------------------------------------------- configs ---

# area modes / parameter defaults shared by callers (plain integers; the
# meaning of each field is fixed by the library's C header)
AREA_FACTOR = 0
AREA_DEPTH = 1


@dataclass
class Workload:
    name: str
    graph: Graph
    part: np.ndarray
    k: int
    pairs: list[tuple[int, int]]
    params: dict = field(default_factory=dict)


def config(cid: str, seed: int | None = None, n_override: int | None = None) -> Workload:
    """The five workloads (and C1b) with their seeded inputs.

    C1  128x128 unit grid, columns x<64 | x>=64, 5 % of each side's boundary
        swapped, eps 3 %, corridor = BFS depth 8, one solve.
    C1b same grid and noise, weight-bounded corridor at alpha = 1.
    C2  2D RGG n=2^18, mean degree 8, weights in [1,10], median-x bisection +
        2 % swap noise, eps 3 %, alpha 16 adaptive.
    C3  3D RGG n=2^20, mean degree 12, unit weights, k=16 RCB + 2 % noise.
    C4  2D RGG n=2^22, mean degree 8, weights in [1,10], k=64 RCB + 2 % noise.
    C5  2D RGG n=2^24, mean degree 6, unit weights, k=256 RCB + 1 % noise.
    n_override shrinks the RGG configs (same recipe) for quick tests.
    """
    cid = cid.upper()
    base = dict(area_mode=AREA_FACTOR, depth=0, alpha=16, alpha_max=16, adaptive=1,
                max_iters=16, eps_ppm=30000, use_mlp=0)
    if cid in ("C1", "C1B"):
        g = grid2d(128, 128)
        x = np.arange(g.n) % 128
        part = (x >= 64).astype(np.int32)
        pair_swap_noise(g, part, 0.05, 1 if seed is None else seed)
        if cid == "C1":
            p = dict(base, area_mode=AREA_DEPTH, depth=8, alpha=1, alpha_max=1, adaptive=0,
                     max_iters=1)
        else:
            p = dict(base, alpha=1, alpha_max=1, adaptive=0, max_iters=1)
        return Workload(cid, g, part, 2, [(0, 1)], p)
    if cid == "C2":
        n = n_override or (1 << 18)
        s = 2 if seed is None else seed
        g = rgg(n, 2, 8.0, s, 1, 10)
        part = rcb(g, 2, force_axis=0)
        pair_swap_noise(g, part, 0.02, s)
        return Workload(cid, g, part, 2, [(0, 1)], dict(base))
    if cid in ("C3", "C4", "C5"):
        n, dim, deg, wlo, whi, k, frac = {
            "C3": (1 << 20, 3, 12.0, 1, 1, 16, 0.02),
            "C4": (1 << 22, 2, 8.0, 1, 10, 64, 0.02),
            "C5": (1 << 24, 2, 6.0, 1, 1, 256, 0.01),
        }[cid]
        n = n_override or n
        s = int(cid[1]) if seed is None else seed
        g = rgg(n, dim, deg, s, wlo, whi)
        part = rcb(g, k)
        global_noise(g, part, frac, s)
        return Workload(cid, g, part, k, [], dict(base))
    raise ValueError(f"unknown config {cid}")

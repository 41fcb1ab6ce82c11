"""Python binding of libflowrefine (max-flow min-cut pair refinement on
MI355X).  Argument marshalling only: every step of the refinement runs in the
library's HIP kernels.  torch supplies device memory and the stream.

The names mirror the C ABI in include/flowrefine.h: fr_create, fr_destroy,
flow_refine_pair, flow_refine_batch, flow_refine_sweep, fr_quotient_matchings,
fr_set_tuning, fr_get_tuning, fr_last_stats.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflowrefine.so")
_lib = None

FR_OK = 0
FR_ERRORS = {-1: "INVALID_GRAPH", -2: "INVALID_PART", -3: "INVALID_PAIR",
             -4: "PAIRS_NOT_DISJOINT", -5: "OVERFLOW", -6: "DEVICE", -7: "OOM",
             -8: "INVALID_ARG", -9: "SOLVER_LIMIT", -10: "SCRATCH_LIMIT"}
FR_ACCEPTED, FR_REJECTED_IMBALANCE, FR_NO_IMPROVEMENT, FR_NOT_ADJACENT = 1, 2, 3, 4
FR_DEC_APPLY, FR_DEC_INFEASIBLE, FR_DEC_EQUAL, FR_DEC_NOT_ADJACENT = 1, 2, 3, 4
FR_AREA_FACTOR, FR_AREA_DEPTH = 0, 1

i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class FrGraph(ctypes.Structure):
    _fields_ = [("n", i32), ("on_device", i32), ("xadj", vp), ("adjncy", vp), ("adjwgt", vp),
                ("vwgt", vp)]


class FrParams(ctypes.Structure):
    _fields_ = [(f, i32) for f in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                   "max_iters", "eps_ppm", "use_mlp", "mb_reps", "mb_seed",
                                   "fm_limit", "fm_seed", "active_blocks", "cut_side",
                                   "terminals", "mt_alpha", "mt_seed", "mlp_restart")]


class FrResult(ctypes.Structure):
    _fields_ = [(f, i32) for f in ("status", "iters", "final_alpha", "applied", "iter_cap",
                                   "start_alpha")] + [
        (f, i64) for f in ("flow_value", "cut_before", "cut_after", "weight_a", "weight_b",
                           "region_vertices", "region_edges", "mt_kept")]


class FrSolve(ctypes.Structure):
    _fields_ = [("alpha", i32), ("decision", i32)] + [
        (f, i64) for f in ("flow", "region_vertices", "region_edges", "source_side",
                           "cut_before", "cut_candidate", "wa", "wb")]


class FrTuning(ctypes.Structure):
    _fields_ = [(f, i32) for f in ("block_threads", "blocks_per_cu", "tpv", "relabel_period",
                                   "mb_lds", "slice_us")]


EXPORTS = ("fr_create", "fr_destroy", "fr_strerror", "flow_refine_pair",
           "flow_refine_pair_static", "flow_refine_batch",
           "flow_refine_sweep", "fr_quotient_matchings", "fr_set_tuning", "fr_get_tuning",
           "fr_set_validation", "fr_set_speculation", "fr_set_fused", "fr_set_timing",
           "fr_last_stats",
           "fr_mlp_num_params", "fr_mlp_init", "fr_mlp_set_weights", "fr_mlp_get_weights", "fr_mlp_forward", "fr_mlp_loss_grad",
           "fr_mlp_train", "fr_mlp_loss_grad_cost", "fr_mlp_train_cost", "fr_pair_features", "fr_autotune", "fr_mlp_predict", "fr_eps_to_ppm")
ALPHAS = (1, 2, 4, 8, 16)


class FlowRefineError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {FR_ERRORS.get(code, code)} ({code})")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is not built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1012_0006_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.fr_create.restype = i32
    lib.fr_create.argtypes = [i32, vp, P(vp)]
    lib.fr_destroy.restype = i32
    lib.fr_destroy.argtypes = [vp]
    lib.fr_strerror.restype = ctypes.c_char_p
    lib.fr_strerror.argtypes = [i32]
    lib.flow_refine_pair.restype = i32
    lib.flow_refine_pair.argtypes = [vp, P(FrGraph), vp, i32, i32, i32, P(FrParams), vp, vp, vp]
    lib.flow_refine_pair_static.restype = i32
    lib.flow_refine_pair_static.argtypes = [vp, P(FrGraph), vp, i32, i32, i32, P(FrParams), vp,
                                            vp]
    lib.flow_refine_batch.restype = i32
    lib.flow_refine_batch.argtypes = [vp, P(FrGraph), vp, i32, vp, i32, P(FrParams), vp, vp]
    lib.flow_refine_sweep.restype = i32
    lib.flow_refine_sweep.argtypes = [vp, P(FrGraph), vp, i32, P(FrParams), i32, P(i64), vp]
    lib.fr_quotient_matchings.restype = i32
    lib.fr_quotient_matchings.argtypes = [vp, P(FrGraph), vp, i32, vp, vp, i32, P(i32)]
    lib.fr_set_tuning.restype = i32
    lib.fr_set_tuning.argtypes = [vp, P(FrTuning)]
    lib.fr_get_tuning.restype = i32
    lib.fr_get_tuning.argtypes = [vp, P(FrTuning)]
    lib.fr_set_validation.restype = i32
    lib.fr_set_validation.argtypes = [vp, i32]
    lib.fr_set_speculation.restype = i32
    lib.fr_set_speculation.argtypes = [vp, i32]
    lib.fr_set_fused.restype = i32
    lib.fr_set_fused.argtypes = [vp, i32]
    lib.fr_set_timing.restype = i32
    lib.fr_set_timing.argtypes = [vp, i32]
    lib.fr_last_stats.restype = i32
    lib.fr_last_stats.argtypes = [vp, vp, vp]
    lib.fr_mlp_num_params.restype = i32
    lib.fr_mlp_num_params.argtypes = []
    lib.fr_mlp_init.restype = i32
    lib.fr_mlp_init.argtypes = [vp, ctypes.c_uint64]
    lib.fr_mlp_set_weights.restype = i32
    lib.fr_mlp_set_weights.argtypes = [vp, vp, i32]
    lib.fr_mlp_get_weights.restype = i32
    lib.fr_mlp_get_weights.argtypes = [vp, vp, i32]
    lib.fr_mlp_predict.restype = i32
    lib.fr_mlp_predict.argtypes = [vp, vp, i32, vp]
    lib.fr_eps_to_ppm.restype = i32
    lib.fr_eps_to_ppm.argtypes = [ctypes.c_double, ctypes.POINTER(i32)]
    lib.fr_mlp_forward.restype = i32
    lib.fr_mlp_forward.argtypes = [vp, vp, i32, vp]
    lib.fr_mlp_loss_grad.restype = i32
    lib.fr_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.fr_mlp_train.restype = i32
    lib.fr_mlp_train.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, vp]
    lib.fr_mlp_loss_grad_cost.restype = i32
    lib.fr_mlp_loss_grad_cost.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.fr_mlp_train_cost.restype = i32
    lib.fr_mlp_train_cost.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64,
                                      vp]
    lib.fr_pair_features.restype = i32
    lib.fr_pair_features.argtypes = [vp, P(FrGraph), vp, i32, vp, i32, i32, vp]
    lib.fr_autotune.restype = i32
    lib.fr_autotune.argtypes = [vp, P(FrGraph), vp, i32, vp, i32, P(FrParams), vp, i32, i32, vp,
                                P(i32)]
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != FR_OK:
        raise FlowRefineError(rc, where)


def _struct_dict(s) -> dict:
    return {f: getattr(s, f) for f, _ in s._fields_}


def params(**kw) -> FrParams:
    """fr_params with the defaults below; mb_seed takes any int (its low 32
    bits are used)."""
    d = dict(area_mode=0, depth=0, alpha=16, alpha_max=16, adaptive=1, max_iters=16,
             eps_ppm=30000, use_mlp=0, mb_reps=0, mb_seed=0, fm_limit=0, fm_seed=0,
             active_blocks=0, cut_side=0, terminals=0, mt_alpha=0, mt_seed=0, mlp_restart=1)
    d.update(kw)
    for f in ("mb_seed", "fm_seed", "mt_seed"):
        seed = int(d[f]) & 0xFFFFFFFF
        d[f] = seed - (1 << 32) if seed >= 1 << 31 else seed
    return FrParams(**{k: int(d[k]) for k, _ in FrParams._fields_})


@dataclass
class DeviceGraph:
    """CSR graph held in device memory (torch int32 tensors)."""
    n: int
    xadj: object
    adjncy: object
    adjwgt: object
    vwgt: object

    @classmethod
    def from_host(cls, g, device="cuda"):
        import torch

        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(device)

        return cls(int(g.xadj.shape[0] - 1), t(g.xadj), t(g.adjncy), t(g.adjwgt), t(g.vwgt))

    def struct(self) -> FrGraph:
        return FrGraph(self.n, 1, self.xadj.data_ptr(), self.adjncy.data_ptr(),
                       self.adjwgt.data_ptr(), self.vwgt.data_ptr())

    @property
    def narcs(self) -> int:
        return int(self.adjncy.shape[0])


def host_graph_struct(g):
    """FrGraph over host numpy arrays (the library copies them); returns
    (struct, keepalive)."""
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (g.xadj, g.adjncy, g.adjwgt, g.vwgt)]
    s = FrGraph(int(arrs[0].shape[0] - 1), 0, *(a.ctypes.data for a in arrs))
    return s, arrs


class Context:
    """fr_create / fr_destroy around one HIP device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = vp()
        _check(lib.fr_create(device, stream, ctypes.byref(h)), "fr_create")
        self.handle = h
        self.lib = lib

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning ---------------------------------------------------------
    def set_tuning(self, block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=100,
                   mb_lds=1, slice_us=8000):
        t = FrTuning(block_threads, blocks_per_cu, tpv, relabel_period, mb_lds, slice_us)
        _check(self.lib.fr_set_tuning(self.handle, ctypes.byref(t)), "fr_set_tuning")

    def get_tuning(self) -> dict:
        t = FrTuning()
        _check(self.lib.fr_get_tuning(self.handle, ctypes.byref(t)), "fr_get_tuning")
        return _struct_dict(t)

    def set_validation(self, on: bool):
        _check(self.lib.fr_set_validation(self.handle, 1 if on else 0), "fr_set_validation")

    def set_speculation(self, on: bool = True):
        _check(self.lib.fr_set_speculation(self.handle, 1 if on else 0), "fr_set_speculation")

    def set_fused(self, on: bool = True):
        """Rounds as one persistent launch, or one launch chain per adaptive
        iteration (the default); results are identical."""
        _check(self.lib.fr_set_fused(self.handle, 1 if on else 0), "fr_set_fused")

    def set_timing(self, on: bool = True):
        _check(self.lib.fr_set_timing(self.handle, 1 if on else 0), "fr_set_timing")

    def last_stats(self):
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 32)()
        _check(self.lib.fr_last_stats(self.handle, ms, cnt), "fr_last_stats")
        return list(ms), list(cnt)


WORK_KEYS = ("bnd_verts", "bnd_arcs", "bfs_items", "bfs_arcs", "net_verts", "net_arcs",
             "sweep_items", "sweep_arcs", "gr_items", "gr_arcs", "cl_items", "cl_arcs")


def stats_dict(ctx) -> dict:
    """fr_last_stats as a dict: phase times (ms) and work counters."""
    ms, cnt = ctx.last_stats()
    d = dict(setup_ms=ms[0], round_ms=ms[1], corridor_ms=ms[2], build_ms=ms[3],
             call_ms=ms[4], relabel_ms=ms[5], push_ms=ms[6], flow_kernel_ms=ms[7],
             sweeps=cnt[0], relabels=cnt[1], bfs_levels=cnt[2], gr_levels=cnt[3],
             cl_levels=cnt[4], workgroups=cnt[5], diag=cnt[6], slots=cnt[7],
             mb_kernel_ms=cnt[8] / 1e6, mb_free=cnt[9], mb_comp=cnt[10], mb_big=cnt[11],
             fm_steps=cnt[12], fm_kept=cnt[13], flow_launches=cnt[14], restarts=cnt[15],
             mt_searches=cnt[28],
             mt_moves=cnt[29], mt_kept=cnt[30], slices=cnt[31])
    d.update({k: cnt[16 + i] for i, k in enumerate(WORK_KEYS)})
    return d


def _graph_arg(graph):
    if isinstance(graph, DeviceGraph):
        return graph.struct(), None
    return host_graph_struct(graph)


def _part_arg(part, on_device: bool):
    if on_device:
        import torch

        assert isinstance(part, torch.Tensor) and part.is_cuda and part.dtype == torch.int32
        assert part.is_contiguous()
        return part.data_ptr()
    assert isinstance(part, np.ndarray) and part.dtype == np.int32 and part.flags.c_contiguous
    return part.ctypes.data


def flow_refine_pair(ctx: Context, graph, part, k: int, a: int, b: int, prm: FrParams,
                     want_side: bool = False):
    """Adaptive flow refinement of one pair; part is updated in place.
    Returns (result, trace, side)."""
    gs, keep = _graph_arg(graph)
    res = FrResult()
    trace = (FrSolve * max(1, prm.max_iters))()
    side = np.zeros(gs.n, dtype=np.int8) if want_side else None
    rc = ctx.lib.flow_refine_pair(ctx.handle, ctypes.byref(gs), _part_arg(part, gs.on_device), k,
                                  a, b, ctypes.byref(prm), ctypes.addressof(res),
                                  side.ctypes.data if want_side else None,
                                  ctypes.addressof(trace))
    _check(rc, "flow_refine_pair")
    r = _struct_dict(res)
    return r, [_struct_dict(trace[i]) for i in range(r["iters"])], side


def flow_refine_pair_static(ctx: Context, graph, part, k: int, a: int, b: int, prm: FrParams):
    """flow_refine_pair without device allocation (the library's static
    scratch; graph and part on the device).  Returns (result, trace)."""
    gs, keep = _graph_arg(graph)
    res = FrResult()
    trace = (FrSolve * max(1, prm.max_iters))()
    rc = ctx.lib.flow_refine_pair_static(ctx.handle, ctypes.byref(gs),
                                         _part_arg(part, gs.on_device), k, a, b,
                                         ctypes.byref(prm), ctypes.addressof(res),
                                         ctypes.addressof(trace))
    _check(rc, "flow_refine_pair_static")
    r = _struct_dict(res)
    return r, [_struct_dict(trace[i]) for i in range(r["iters"])]


def flow_refine_batch(ctx: Context, graph, part, k: int, pairs, prm: FrParams):
    """All pairs of one matching in one batched solve; part updated in place.
    Returns (results, traces)."""
    gs, keep = _graph_arg(graph)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    npairs = pr.shape[0] // 2
    res = (FrResult * max(1, npairs))()
    mi = max(1, prm.max_iters)
    trace = (FrSolve * max(1, npairs * mi))()
    rc = ctx.lib.flow_refine_batch(ctx.handle, ctypes.byref(gs), _part_arg(part, gs.on_device), k,
                                   pr.ctypes.data, npairs, ctypes.byref(prm),
                                   ctypes.addressof(res), ctypes.addressof(trace))
    _check(rc, "flow_refine_batch")
    results = [_struct_dict(res[i]) for i in range(npairs)]
    traces = [[_struct_dict(trace[i * mi + j]) for j in range(results[i]["iters"])]
              for i in range(npairs)]
    return results, traces


def fr_quotient_matchings(ctx: Context, graph, part, k: int):
    gs, keep = _graph_arg(graph)
    maxe = k * (k - 1) // 2 + 1
    edges = np.zeros(2 * maxe, dtype=np.int32)
    colour = np.zeros(maxe, dtype=np.int32)
    ne = i32(0)
    rc = ctx.lib.fr_quotient_matchings(ctx.handle, ctypes.byref(gs), _part_arg(part, gs.on_device),
                                       k, edges.ctypes.data, colour.ctypes.data, maxe,
                                       ctypes.byref(ne))
    _check(rc, "fr_quotient_matchings")
    return edges[:2 * ne.value].reshape(-1, 2), colour[:ne.value]


def flow_refine_sweep(ctx: Context, graph, part, k: int, prm: FrParams, max_sweeps: int):
    """Returns (total cut, stats[sweeps, solves, changed pairs, region edges])."""
    gs, keep = _graph_arg(graph)
    tc = i64(0)
    stats = np.zeros(4, dtype=np.int64)
    rc = ctx.lib.flow_refine_sweep(ctx.handle, ctypes.byref(gs), _part_arg(part, gs.on_device), k,
                                   ctypes.byref(prm), max_sweeps, ctypes.byref(tc),
                                   stats.ctypes.data)
    _check(rc, "flow_refine_sweep")
    return int(tc.value), stats


# ------------------------------------------------------ learned factor ---

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def fr_mlp_num_params() -> int:
    return int(load().fr_mlp_num_params())


def fr_mlp_predict(ctx: Context, x) -> np.ndarray:
    """Start factor per sample from the loaded network (features [n, 8])."""
    xs = _f32(x).reshape(-1, 8)
    a = np.zeros(xs.shape[0], dtype=np.int32)
    _check(ctx.lib.fr_mlp_predict(ctx.handle, xs.ctypes.data, xs.shape[0], a.ctypes.data),
           "fr_mlp_predict")
    return a


def eps_to_ppm(eps: float) -> int:
    """fr_eps_to_ppm: eps as a fraction -> parts per million."""
    out = i32(0)
    _check(load().fr_eps_to_ppm(float(eps), ctypes.byref(out)), "fr_eps_to_ppm")
    return int(out.value)


def mlp_unpack(w: np.ndarray) -> dict:
    """Flat parameter array -> W1, b1, W2, b2, W3, b3 (row-major [in][out])."""
    w = np.asarray(w, dtype=np.float32)
    shapes = (("W1", (8, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (64, 5)), ("b3", (5,)))
    out, off = {}, 0
    for k, sh in shapes:
        cnt = int(np.prod(sh))
        out[k] = w[off:off + cnt].reshape(sh)
        off += cnt
    return out


def fr_mlp_init(ctx: Context, seed: int):
    _check(ctx.lib.fr_mlp_init(ctx.handle, seed), "fr_mlp_init")


def fr_mlp_set_weights(ctx: Context, w):
    w = _f32(w)
    _check(ctx.lib.fr_mlp_set_weights(ctx.handle, w.ctypes.data, w.size), "fr_mlp_set_weights")


def fr_mlp_get_weights(ctx: Context) -> np.ndarray:
    w = np.zeros(fr_mlp_num_params(), dtype=np.float32)
    _check(ctx.lib.fr_mlp_get_weights(ctx.handle, w.ctypes.data, w.size), "fr_mlp_get_weights")
    return w


def fr_mlp_forward(ctx: Context, x) -> np.ndarray:
    x = _f32(x).reshape(-1, 8)
    p = np.zeros((x.shape[0], 5), dtype=np.float32)
    _check(ctx.lib.fr_mlp_forward(ctx.handle, x.ctypes.data, x.shape[0], p.ctypes.data),
           "fr_mlp_forward")
    return p


def fr_mlp_loss_grad(ctx: Context, x, labels):
    x = _f32(x).reshape(-1, 8)
    y = _i32(labels)
    loss = np.zeros(1, dtype=np.float32)
    g = np.zeros(fr_mlp_num_params(), dtype=np.float32)
    _check(ctx.lib.fr_mlp_loss_grad(ctx.handle, x.ctypes.data, y.ctypes.data, x.shape[0],
                                    loss.ctypes.data, g.ctypes.data), "fr_mlp_loss_grad")
    return float(loss[0]), g


def fr_mlp_train(ctx: Context, x, labels, epochs: int, batch: int, lr: float, seed: int):
    x = _f32(x).reshape(-1, 8)
    y = _i32(labels)
    losses = np.zeros(epochs, dtype=np.float32)
    _check(ctx.lib.fr_mlp_train(ctx.handle, x.ctypes.data, y.ctypes.data, x.shape[0], epochs,
                                batch, lr, seed, losses.ctypes.data), "fr_mlp_train")
    return losses


def fr_mlp_loss_grad_cost(ctx: Context, x, costs):
    """Mean expected cost sum_c p_c costs_c (costs [n, 5]) and its gradient."""
    x = _f32(x).reshape(-1, 8)
    cs = _f32(costs).reshape(-1, 5)
    assert cs.shape[0] == x.shape[0]
    loss = np.zeros(1, dtype=np.float32)
    g = np.zeros(fr_mlp_num_params(), dtype=np.float32)
    _check(ctx.lib.fr_mlp_loss_grad_cost(ctx.handle, x.ctypes.data, cs.ctypes.data, x.shape[0],
                                         loss.ctypes.data, g.ctypes.data), "fr_mlp_loss_grad_cost")
    return float(loss[0]), g


def fr_mlp_train_cost(ctx: Context, x, costs, epochs: int, batch: int, lr: float, seed: int):
    x = _f32(x).reshape(-1, 8)
    cs = _f32(costs).reshape(-1, 5)
    assert cs.shape[0] == x.shape[0]
    losses = np.zeros(epochs, dtype=np.float32)
    _check(ctx.lib.fr_mlp_train_cost(ctx.handle, x.ctypes.data, cs.ctypes.data, x.shape[0],
                                     epochs, batch, lr, seed, losses.ctypes.data),
           "fr_mlp_train_cost")
    return losses


def fr_pair_features(ctx: Context, graph, part, k: int, pairs, eps_ppm: int) -> np.ndarray:
    gs, keep = _graph_arg(graph)
    pr = _i32(pairs).reshape(-1)
    npairs = pr.shape[0] // 2
    f = np.zeros((npairs, 8), dtype=np.float32)
    _check(ctx.lib.fr_pair_features(ctx.handle, ctypes.byref(gs), _part_arg(part, gs.on_device), k,
                                    pr.ctypes.data, npairs, eps_ppm, f.ctypes.data),
           "fr_pair_features")
    return f


def fr_autotune(ctx: Context, graph: DeviceGraph, part, k: int, pairs, prm: FrParams,
                candidates, reps: int = 2):
    """Times each candidate tuning (dicts of FrTuning fields); the fastest is
    kept in the context.  Returns (best index, per-candidate ms)."""
    gs = graph.struct()
    pr = _i32(pairs).reshape(-1)
    cand = (FrTuning * len(candidates))(*[FrTuning(**{"mb_lds": 1, "slice_us": 8000, **c})
                                          for c in candidates])
    ms = (ctypes.c_double * len(candidates))()
    best = i32(-1)
    _check(ctx.lib.fr_autotune(ctx.handle, ctypes.byref(gs), _part_arg(part, True), k,
                               pr.ctypes.data, pr.shape[0] // 2, ctypes.byref(prm), cand,
                               len(candidates), reps, ms, ctypes.byref(best)), "fr_autotune")
    return int(best.value), list(ms)


DEFAULT_CANDIDATES = (
    dict(block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=100, slice_us=8000),
    dict(block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=70, slice_us=8000),
    dict(block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=100, slice_us=0),
    dict(block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=100, slice_us=2000),
    dict(block_threads=1024, blocks_per_cu=2, tpv=8, relabel_period=100, slice_us=16000),
    dict(block_threads=1024, blocks_per_cu=2, tpv=4, relabel_period=200, slice_us=8000),
    dict(block_threads=1024, blocks_per_cu=2, tpv=2, relabel_period=200, slice_us=8000),
    dict(block_threads=512, blocks_per_cu=4, tpv=4, relabel_period=200, slice_us=8000),
    dict(block_threads=256, blocks_per_cu=8, tpv=4, relabel_period=200, slice_us=8000),
)


def tuning_key(arch: str, n: int, narcs: int, npairs: int) -> str:
    """Cache key of a workload: GPU architecture, log2 bucket of the vertex
    count, mean-degree bucket and log2 bucket of the pairs per round."""
    deg = narcs / max(1, n)
    return (f"{arch}|n2^{max(0, int(n).bit_length() - 1)}|deg{int(round(deg))}"
            f"|pairs2^{max(0, int(npairs).bit_length() - 1)}")


def autotune_cached(ctx: Context, graph: "DeviceGraph", part, k: int, pairs, prm: FrParams,
                    cache_path: str | None = None, candidates=DEFAULT_CANDIDATES, reps: int = 2,
                    arch: str | None = None) -> dict:
    """Tuning for this workload from a JSON cache keyed by tuning_key, or
    found by fr_autotune (and stored) on a miss; the tuning is set on the
    context and returned."""
    import json

    if arch is None:
        import torch

        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    if cache_path is None:
        cache_path = os.path.join(os.path.expanduser("~"), ".cache", "flowrefine", "tuning.json")
    key = tuning_key(arch, graph.n, graph.narcs, len(pairs))
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        ctx.set_tuning(**cache[key]["tuning"])
        return cache[key]["tuning"]
    best, ms = fr_autotune(ctx, graph, part, k, pairs, prm, list(candidates), reps)
    tuning = dict(candidates[best])
    cache[key] = {"tuning": tuning, "ms": ms}
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, cache_path)
    return tuning


TRAINED_WEIGHTS = os.path.join(_HERE, "mlp_area_factor.json")


def load_trained_mlp(ctx: Context, path: str = TRAINED_WEIGHTS) -> dict:
    """Loads the committed area-factor weights (written by train_mlp.py) into
    the context; returns the training report."""
    import json

    with open(path) as fh:
        d = json.load(fh)
    fr_mlp_set_weights(ctx, np.asarray(d["weights"], dtype=np.float32))
    return d["report"]

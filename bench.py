"""Benchmark of max-flow min-cut pair refinement on one MI355X.

A step is one full refinement of C5: a 2D random geometric graph (n = 2^24,
mean degree 6, unit weights) cut into k = 256 blocks by recursive coordinate
bisection with 1 % boundary noise, eps = 3 %, swept over the colour classes of
its quotient graph until no pair improves.  Every pair of a class is refined
in one batched round (boundary, bounded BFS corridors, networks, max preflow,
smallest source set, balance check, adaptive factor from the learned start,
write-back).  Inputs are resident in device memory before the timed region;
each step starts from the same partition.

Printed: one JSON line with region edges/s of those steps (corridor edges
summed over the solves the adaptive loops record, divided by wall time), the
roofline of the flow kernel over the same steps (k_flow: relabels,
push/relabel passes, closure; HIP events around each of its launches), the
CPU oracle on the largest round of the same workload, and beside it: the C2
plain pair refinement (2D RGG n = 2^18), batched vs plain on the largest
matching round of C3 (3D RGG n = 2^20, k = 16, autotuned launch) and of C5,
plain vs learned start factor on one sweep of C4 (2D RGG n = 2^22, k = 64),
and the quality leg (most balanced cuts, FM, contracted terminals on C5).

``python bench.py --summarize KIND DIR ...`` turns rocprofv3 output copied
back from the GPU machine into the summaries under profiles/ (see summarize()).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flow-refinement region edges/s + %HBM peak, batched vs plain, bit-exact cut"
HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 512 << 20

# algorithmic bytes per unit of work (4-byte ints; what each phase must read
# or write, not what the caches do)
BYTES = {
    "bnd_verts": 16, "bnd_arcs": 8,        # list + part + xadj pair; neighbour id + its block
    "bfs_items": 16, "bfs_arcs": 12,       # + corridor mark of the neighbour
    "net_verts": 29, "net_arcs": 24,       # two passes (count, fill) over the global arcs
    "sweep_items": 20, "sweep_arcs": 12,   # list, label, excess, offsets; head, residual, label
    "gr_items": 12, "gr_arcs": 16,         # list, offsets; head, reverse arc, its residual, label
    "cl_items": 12, "cl_arcs": 12,         # list, offsets; residual, head, mark
}
CORRIDOR_ARC_BYTES = 36  # reverse-arc search and writes of head / reverse / residual


FLOW_KEYS = ("sweep_items", "sweep_arcs", "gr_items", "gr_arcs", "cl_items", "cl_arcs")


def progress(msg: str):
    """One line on stderr per finished leg (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(stats: dict, region_edges: int) -> int:
    """Bytes the whole solve path must move (every phase)."""
    b = sum(stats[k] * v for k, v in BYTES.items())
    return int(b + CORRIDOR_ARC_BYTES * 2 * region_edges)


def flow_bytes(stats: dict) -> int:
    """Bytes the flow kernel must move: push/relabel sweeps, global relabels,
    residual closure."""
    return int(sum(stats[k] * BYTES[k] for k in FLOW_KEYS))


def kernel_source_hash() -> str:
    """Hash of every source compiled into the library (all of csrc/ and the
    public header), so a counter profile goes stale with any kernel change."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1012_0006_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)
                   if f.endswith((".h", ".hip")))
    files.append(os.path.join(ROOT, "include", "flowrefine.h"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k_flow_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def c2_params(fr, w):
    return fr.params(**{k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max",
                                                  "adaptive", "max_iters", "eps_ppm")})


def run_plain(args, fr, torch, gen):
    w = gen.config("C2")
    ctx = fr.Context()
    ctx.set_validation(False)  # inputs are generated valid
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    dpart = part0.clone()
    prm = c2_params(fr, w)
    for _ in range(args.warmup):
        dpart.copy_(part0)
        fr.flow_refine_pair(ctx, dg, dpart, w.k, 0, 1, prm)
    torch.cuda.synchronize()
    edges, kern_ms, byts, path_ms, path_bytes, launches = 0, 0.0, 0, 0.0, 0, 0
    results = []
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        dpart.copy_(part0)
        res, trace, _ = fr.flow_refine_pair(ctx, dg, dpart, w.k, 0, 1, prm)
        step_s.append(time.perf_counter() - ts)  # the call returns after its stream synchronised
        st = fr.stats_dict(ctx)
        edges += res["region_edges"]
        kern_ms += st["flow_kernel_ms"]
        byts += flow_bytes(st)
        path_ms += st["round_ms"]
        path_bytes += algorithmic_bytes(st, res["region_edges"])
        launches += st["flow_launches"]
        results.append((res, trace))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    final_part = dpart.cpu().numpy()
    ctx.close()
    return dict(w=w, edges=edges, wall=wall, kern_ms=kern_ms, bytes=byts, result=results[-1][0],
                trace=results[-1][1], part=final_part, stats=st, path_ms=path_ms,
                path_bytes=path_bytes, launches=launches,
                step_ms=[t * 1e3 for t in step_s])


def run_cpu_baseline(w):
    import oracle

    t0 = time.perf_counter()
    o = oracle.refine_pair(w.graph, w.part, w.k, 0, 1, w.params, want_side=False)
    dt = time.perf_counter() - t0
    return o, dt


def run_batched(args, fr, torch, gen, cid="C3"):
    """The largest matching round of a workload (C3: 3D RGG n=2^20, mean
    degree 12, k=16 RCB + 2 % noise; C5: 2D RGG n=2^24, k=256): all pairs in
    one batched launch vs the pairs one by one."""
    w = gen.config(cid)
    ctx = fr.Context()
    ctx.set_validation(False)
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges_q, colour = fr.fr_quotient_matchings(ctx, dg, part0, w.k)
    counts = np.bincount(colour)
    c = int(np.argmax(counts))
    pairs = [tuple(e) for e, cc in zip(edges_q.tolist(), colour.tolist()) if cc == c]
    prm = fr.params(**{k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max",
                                                 "adaptive", "max_iters", "eps_ppm")})
    tuning = None
    if cid == "C3":  # the round's launch parameters come from the autotuner
        import tempfile

        with tempfile.TemporaryDirectory() as tmp:
            tuning = fr.autotune_cached(ctx, dg, part0, w.k, pairs, prm,
                                        cache_path=os.path.join(tmp, "tuning.json"), reps=2)
    dpart = part0.clone()
    reps = max(1, args.batch_reps)
    # batched: the median of at least three timed calls (one call is short)
    dpart.copy_(part0)
    fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, prm)  # warm-up
    times_b = []
    for _ in range(max(3, reps)):
        dpart.copy_(part0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_b, _ = fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, prm)
        torch.cuda.synchronize()
        times_b.append(time.perf_counter() - t0)
    t_b = float(np.median(times_b))
    part_b = dpart.cpu().numpy()
    # plain: one pair call after the other on the same partition
    dpart.copy_(part0)
    for a, b in pairs[:1]:
        fr.flow_refine_pair(ctx, dg, dpart, w.k, a, b, prm)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dpart.copy_(part0)
        res_p = [fr.flow_refine_pair(ctx, dg, dpart, w.k, a, b, prm)[0] for a, b in pairs]
    torch.cuda.synchronize()
    t_p = (time.perf_counter() - t0) / reps
    part_p = dpart.cpu().numpy()
    ctx.close()
    e_b = sum(r["region_edges"] for r in res_b)
    e_p = sum(r["region_edges"] for r in res_p)
    same = bool(np.array_equal(part_b, part_p)) and all(
        rb["cut_after"] == rp["cut_after"] for rb, rp in zip(res_b, res_p))
    desc = {"C3": "C3: 3D RGG n=2^20 mean degree 12 unit weights, k=16 RCB + 2% noise",
            "C5": "C5: 2D RGG n=2^24 mean degree 6 unit weights, k=256 RCB + 1% noise"}[cid]
    return {
        "workload": f"{desc}, largest matching round ({len(pairs)} pairs), eps 3%, "
                    "alpha 16 adaptive",
        "pairs": len(pairs),
        "batched_region_edges_per_s": e_b / t_b,
        "plain_region_edges_per_s": e_p / t_p,
        "batched_ms": t_b * 1e3,
        "batched_ms_each": [t * 1e3 for t in times_b],
        "plain_ms": t_p * 1e3,
        "speedup": t_p / t_b,
        "equal_result": same,
        "tuning": tuning,
        "region_edges": e_b,
    }


def run_learned(args, fr, torch, gen):
    """One matching-round sweep of C4 (2D RGG n=2^22, mean degree 8, weights
    1..10, k=64 RCB + 2 % noise): every colour class batched, with the plain
    adaptive search from alpha' = 16, from constant starts 8 and 4, and from
    the learned factor with and without the restart from alpha'."""
    w = gen.config("C4")
    ctx = fr.Context()
    ctx.set_validation(False)
    report = fr.load_trained_mlp(ctx)
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges_q, colour = fr.fr_quotient_matchings(ctx, dg, part0, w.k)
    classes = sorted(set(colour.tolist()))
    out = {}
    runs = {"plain": (0, None, 0), "constant_8": (0, 8, 0), "constant_4": (0, 4, 0),
            "learned": (1, None, 1), "learned_no_restart": (1, None, 0)}
    for name, (use, alpha, restart) in runs.items():
        pc = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                       "max_iters", "eps_ppm")}
        if alpha is not None:
            pc["alpha"] = alpha
        prm = fr.params(**pc, use_mlp=use, mlp_restart=restart)
        dpart = part0.clone()
        solves = edges = restarts = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in classes:
            pairs = [tuple(e) for e, cc in zip(edges_q.tolist(), colour.tolist()) if cc == c]
            res, _ = fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, prm)
            solves += sum(r["iters"] for r in res)
            edges += sum(r["region_edges"] for r in res)
            restarts += fr.stats_dict(ctx)["restarts"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        import oracle  # cut accounting only (sum of cut edge weights)
        out[name] = {
            "seconds": dt, "flow_solves": solves, "region_edges": edges, "restarts": restarts,
            "region_edges_per_s": edges / dt,
            "total_cut": oracle.total_cut(w.graph, dpart.cpu().numpy())}
    ctx.close()
    out["workload"] = ("C4: 2D RGG n=2^22 mean degree 8, weights 1..10, k=64 RCB + 2% noise, "
                       f"one sweep of {len(classes)} matching rounds, eps 3%, alpha' 16 adaptive; "
                       "starts: plain 16, constant 8, constant 4, learned with and without "
                       "the restart from 16")
    out["training"] = {"loss": report.get("loss"), "cost_lambda": report.get("cost_lambda"),
                       "held_out_sweeps": report.get("validation_sweeps")}
    out["speedup"] = out["plain"]["seconds"] / out["learned"]["seconds"]
    out["speedup_vs_constant_8"] = out["constant_8"]["seconds"] / out["learned"]["seconds"]
    return out


C5_WORKLOAD = ("C5: 2D RGG n=2^24 mean degree 6 unit weights, k=256 RCB + 1% noise, eps 3%, "
               "alpha' 16 adaptive with learned start (restarted from 16 where it stops without "
               "improvement), batched rounds over the quotient-graph "
               "colour classes, swept until no pair improves")


def c5_params(fr, w, use_mlp, restart=1):
    return fr.params(**{k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max",
                                                 "adaptive", "max_iters", "eps_ppm")},
                     use_mlp=use_mlp, mlp_restart=restart)


def run_c5_headline(args, fr, torch, gen):
    """C5 refined to convergence per step (learned start factors, every colour
    class one batched round), timed over args.steps steps after args.warmup
    untimed ones; with per-phase timing on, each k_flow launch sits between
    HIP events on the library's stream."""
    import oracle  # cut of the start partition only

    w = gen.config("C5")
    ctx = fr.Context()
    ctx.set_validation(False)  # inputs are generated valid
    ctx.set_timing(True)
    fr.load_trained_mlp(ctx)
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    dpart = part0.clone()
    prm = c5_params(fr, w, 1)
    for _ in range(args.warmup):
        dpart.copy_(part0)
        fr.flow_refine_sweep(ctx, dg, dpart, w.k, prm, args.max_sweeps)
    torch.cuda.synchronize()
    tot = dict(edges=0, kern_ms=0.0, bytes=0, launches=0, solves=0, sweeps=0, corridor_ms=0.0,
               build_ms=0.0, sweeps_pr=0, relabels=0, gr_levels=0)
    step_ms, first, cut = [], None, None
    same = True
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        dpart.copy_(part0)
        cut, stats = fr.flow_refine_sweep(ctx, dg, dpart, w.k, prm, args.max_sweeps)
        step_ms.append((time.perf_counter() - ts) * 1e3)  # the call synchronises its stream
        st = fr.stats_dict(ctx)
        tot["edges"] += int(stats[3])
        tot["solves"] += int(stats[1])
        tot["sweeps"] += int(stats[0])
        tot["kern_ms"] += st["flow_kernel_ms"]
        tot["bytes"] += flow_bytes(st)
        tot["launches"] += st["flow_launches"]
        tot["corridor_ms"] += st["corridor_ms"]
        tot["build_ms"] += st["build_ms"]
        tot["sweeps_pr"] += st["sweeps"]
        tot["relabels"] += st["relabels"]
        tot["gr_levels"] += st["gr_levels"]
        out = dpart.cpu().numpy()
        if first is None:
            first = out
        else:
            same = same and bool(np.array_equal(first, out))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    return dict(w=w, wall=wall, step_ms=step_ms, cut0=int(oracle.total_cut(w.graph, w.part)),
                cut=int(cut), repeatable=same, part=first, **tot)


def run_c5_no_restart(args, fr, torch, w):
    """The headline's sweep once more without the restart of learned starts:
    the learned start's saving and its cut loss on this family."""
    ctx = fr.Context()
    ctx.set_validation(False)
    fr.load_trained_mlp(ctx)
    dg = fr.DeviceGraph.from_host(w.graph)
    dpart = torch.as_tensor(w.part).cuda()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    cut, stats = fr.flow_refine_sweep(ctx, dg, dpart, w.k, c5_params(fr, w, 1, restart=0),
                                      args.max_sweeps)
    out = {"ms": (time.perf_counter() - ts) * 1e3, "cut_after": int(cut), "sweeps": int(stats[0]),
           "flow_solves": int(stats[1]), "region_edges": int(stats[3])}
    ctx.close()
    return out


def run_c5_cpu_baseline(args, fr, torch, w):
    """The oracle on the largest matching round of C5 (the first colour class
    of the start partition), each pair from the start factor the learned
    network gives it on the GPU: over a thread pool of the host cores this
    process may use (at most 16), and on one thread for the first pairs.  The
    GPU's results for the same pairs must be bit-exact."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    ctx = fr.Context()
    ctx.set_validation(False)
    fr.load_trained_mlp(ctx)
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges_q, colour = fr.fr_quotient_matchings(ctx, dg, part0, w.k)
    c = int(np.argmax(np.bincount(colour)))
    pairs = [tuple(e) for e, cc in zip(edges_q.tolist(), colour.tolist()) if cc == c]
    dpart = part0.clone()
    res, trace = fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, c5_params(fr, w, 1))
    gpu_part = dpart.cpu().numpy()
    ctx.close()
    base = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                     "max_iters", "eps_ppm")}

    def one(i):
        a, b = pairs[i]
        return oracle.refine_pair(w.graph, w.part, w.k, a, b,
                                  dict(base, alpha=res[i]["start_alpha"],
                                       restart_alpha=base["alpha"]), want_side=False)

    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, min(16, avail))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        outs = list(pool.map(one, range(len(pairs))))
    dt = time.perf_counter() - t0
    exact = True
    new = w.part.copy()
    for i, o in enumerate(outs):
        exact = exact and o.rc == 0 and o.trace == trace[i] and all(
            o.result[key] == res[i][key] for key in ("flow_value", "cut_after", "weight_a",
                                                     "weight_b", "iters", "region_edges"))
        mine = (w.part == pairs[i][0]) | (w.part == pairs[i][1])
        new[mine] = o.part[mine]
    exact = exact and bool(np.array_equal(new, gpu_part))
    edges = sum(o.result["region_edges"] for o in outs)
    n1 = min(len(pairs), args.cpu_one_thread_pairs)
    t1 = time.perf_counter()
    e1 = sum(one(i).result["region_edges"] for i in range(n1))
    d1 = time.perf_counter() - t1
    return {
        "value": edges / dt, "unit": "region edges/s", "cores": threads, "kind": "oracle",
        "sample": f"the largest matching round of C5 ({len(pairs)} pairs, {edges} region edges), "
                  "each pair the sequential oracle from its learned start factor, spread over "
                  f"{threads} host threads ({os.cpu_count()} logical CPUs visible)",
        "seconds": dt, "host_cpus_visible": os.cpu_count(), "threads": threads,
        "one_thread": {"value": e1 / d1, "unit": "region edges/s", "cores": 1,
                       "sample": f"the first {n1} pairs of that round, one after the other",
                       "seconds": d1},
        "bit_exact_vs_gpu_round": bool(exact),
    }


def run_balanced(args, fr, torch, gen):
    """The widenings of the pair refinement on C5 (2D RGG n=2^24, mean degree
    6, unit weights, k=256 RCB + 1 % noise): most balanced minimum cuts
    (Sec. 4.1.1, 16 sweeps) and 2-way FM with TopGain before the flow
    (Sec. 2.2, stop after 100 moves without improvement), alone and together,
    and together with active block scheduling (Sec. 4.3); the corridor network
    with the blocks' outside parts contracted into s and t instead of the
    pinned border, alone and with all of the above; against the plain flow:
    the largest matching round batched, then whole refinement sweeps until no
    pair improves, for time and the cut reached."""
    import oracle  # cut accounting only

    w = gen.config("C5")
    ctx = fr.Context()
    ctx.set_validation(False)
    dg = fr.DeviceGraph.from_host(w.graph)
    part0 = torch.as_tensor(w.part).cuda()
    edges_q, colour = fr.fr_quotient_matchings(ctx, dg, part0, w.k)
    c = int(np.argmax(np.bincount(colour)))
    pairs = [tuple(e) for e, cc in zip(edges_q.tolist(), colour.tolist()) if cc == c]
    base = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                     "max_iters", "eps_ppm")}
    out = {"workload": f"C5: 2D RGG n=2^24 mean degree 6 unit weights, k=256 RCB + 1% noise, "
                       f"largest matching round ({len(pairs)} pairs) batched, then sweeps "
                       f"until no pair improves; eps 3%, alpha 16 adaptive",
           "pairs": len(pairs)}
    variants = (("smallest_source_set", {}),
                ("most_balanced", {"mb_reps": 16, "mb_seed": 1}),
                ("fm_then_flow", {"fm_limit": 100, "fm_seed": 1}),
                ("fm_then_most_balanced", {"fm_limit": 100, "fm_seed": 1, "mb_reps": 16,
                                           "mb_seed": 1}),
                ("fm_then_most_balanced_active", {"fm_limit": 100, "fm_seed": 1, "mb_reps": 16,
                                                  "mb_seed": 1, "active_blocks": 1}),
                ("contracted_terminals", {"terminals": 1}),
                ("contracted_fm_most_balanced_active", {"terminals": 1, "fm_limit": 100,
                                                        "fm_seed": 1, "mb_reps": 16, "mb_seed": 1,
                                                        "active_blocks": 1}))
    for name, extra in variants:
        prm = fr.params(**base, **extra)
        dpart = part0.clone()
        fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, prm)  # warm-up
        reps = max(1, args.batch_reps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dpart.copy_(part0)
            res, _ = fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, prm)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = fr.stats_dict(ctx)
        edges = sum(r["region_edges"] for r in res)
        rnd = {"round_ms": dt * 1e3, "region_edges_per_s": edges / dt,
               "flow_solves": sum(r["iters"] for r in res),
               "changed_pairs": sum(1 for r in res if r["status"] == fr.FR_ACCEPTED),
               "pair_cut_after": sum(r["cut_after"] for r in res),
               "pair_cut_before": sum(r["cut_before"] for r in res),
               "flow_kernel_ms": st["flow_kernel_ms"], "mb_kernel_ms": st["mb_kernel_ms"],
               "mb_free_vertices": st["mb_free"], "mb_components": st["mb_comp"],
               "mb_device_dag_solves": st["mb_big"], "fm_moves": st["fm_steps"],
               "fm_moves_kept": st["fm_kept"]}
        dpart = part0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cut, stats = fr.flow_refine_sweep(ctx, dg, dpart, w.k, prm, args.max_sweeps)
        torch.cuda.synchronize()
        ds = time.perf_counter() - t0
        newp = dpart.cpu().numpy()
        bw = np.bincount(newp, weights=w.graph.vwgt, minlength=w.k)
        rnd["sweep"] = {"seconds": ds, "sweeps": int(stats[0]), "flow_solves": int(stats[1]),
                        "region_edges_per_s": float(stats[3]) / ds, "cut_after": int(cut),
                        "max_block_weight": int(bw.max())}
        out[name] = rnd
        progress(f"quality leg {name}: round {rnd['round_ms']:.0f} ms, sweeps {ds:.1f} s, "
                 f"cut {int(cut)}")
    ctx.close()
    out["cut_before"] = int(oracle.total_cut(w.graph, w.part))
    ref = out["smallest_source_set"]["sweep"]["cut_after"]
    out["sweep_cut_ratio"] = {name: out[name]["sweep"]["cut_after"] / ref for name, _ in variants}
    return out


def run_multitry(args, fr, torch, gen):
    """Multi-try FM (Sec. 4.2, alpha 10) after the pairwise improvements of the
    largest matching round of C3 and of C5: one batched call with and one
    without it, from the same partition: time, the phase's work and the cut
    reached."""
    import oracle  # cut accounting only

    out = {}
    for cid in args.mt_configs.split(","):
        w = gen.config(cid)
        ctx = fr.Context()
        ctx.set_validation(False)
        dg = fr.DeviceGraph.from_host(w.graph)
        part0 = torch.as_tensor(w.part).cuda()
        edges_q, colour = fr.fr_quotient_matchings(ctx, dg, part0, w.k)
        c = int(np.argmax(np.bincount(colour)))
        pairs = [tuple(e) for e, cc in zip(edges_q.tolist(), colour.tolist()) if cc == c]
        base = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                         "max_iters", "eps_ppm")}
        leg = {"pairs": len(pairs)}
        for name, extra in (("pairwise", {}), ("pairwise_then_multitry",
                                                {"mt_alpha": 10, "mt_seed": 1})):
            dpart = part0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, _ = fr.flow_refine_batch(ctx, dg, dpart, w.k, pairs, fr.params(**base, **extra))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = fr.stats_dict(ctx)
            leg[name] = {"seconds": dt, "total_cut": int(oracle.total_cut(w.graph,
                                                                          dpart.cpu().numpy())),
                         "mt_searches": st["mt_searches"], "mt_moves": st["mt_moves"],
                         "mt_kept": st["mt_kept"]}
        leg["cut_before"] = int(oracle.total_cut(w.graph, w.part))
        leg["multitry_seconds"] = (leg["pairwise_then_multitry"]["seconds"]
                                   - leg["pairwise"]["seconds"])
        out[cid] = leg
        ctx.close()
        progress(f"multi-try {cid}: {leg['multitry_seconds']:.2f} s, "
                 f"cut {leg['pairwise']['total_cut']} -> "
                 f"{leg['pairwise_then_multitry']['total_cut']}")
    return out


def roofline(bytes_total: float, kern_ms: float, launches: int, traffic) -> dict:
    """k_flow against the HBM peak: algorithmic bytes per launch over the
    average launch time from the events (total bytes / total time)."""
    avg_s = kern_ms / 1e3 / max(1, launches)
    per_launch = bytes_total / max(1, launches)
    achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    return {"bound": "hbm", "kernel": "k_flow", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": avg_s * 1e3,
            "launches": launches}


def c2_leg(args, fr, torch, gen):
    plain = run_plain(args, fr, torch, gen)
    progress(f"C2 plain: {plain['wall'] * 1e3 / args.steps:.1f} ms per step")
    out = {
        "workload": "C2: 2D RGG n=2^18 mean degree 8, edge weights 1..10, median-x bisection "
                    "+ 2% boundary noise, eps 3%, alpha 16 adaptive (max 16 solves)",
        "region_edges_per_s": plain["edges"] / plain["wall"],
        "ms_per_step": plain["wall"] * 1e3 / args.steps,
        "ms_per_step_median": float(np.median(plain["step_ms"])),
        "ms_per_step_min": float(np.min(plain["step_ms"])),
        "region_edges_per_step": plain["edges"] // args.steps,
        "solves_per_step": plain["result"]["iters"],
        "sweeps_per_step": plain["stats"]["sweeps"],
        "relabels_per_step": plain["stats"]["relabels"],
        "relabel_bfs_levels_per_step": plain["stats"]["gr_levels"],
        "per_recorded_solve": {
            "push_relabel_sweeps": plain["stats"]["sweeps"] / plain["result"]["iters"],
            "global_relabels": plain["stats"]["relabels"] / plain["result"]["iters"],
            "relabel_bfs_levels": plain["stats"]["gr_levels"] / plain["result"]["iters"]},
        "roofline": roofline(plain["bytes"], plain["kern_ms"], plain["launches"],
                             load_traffic("C2")),
        "whole_path_gb_per_s": plain["path_bytes"] / (plain["path_ms"] / 1e3) / 1e9,
    }
    if not args.no_cpu_baseline:
        o, dt = run_cpu_baseline(plain["w"])
        out["bit_exact_vs_oracle"] = bool(
            o.result["cut_after"] == plain["result"]["cut_after"]
            and o.result["flow_value"] == plain["result"]["flow_value"]
            and o.trace == plain["trace"] and np.array_equal(o.part, plain["part"]))
        out["cpu_baseline"] = {
            "value": o.result["region_edges"] / dt, "unit": "region edges/s", "cores": 1,
            "kind": "oracle", "seconds": dt,
            "sample": "one full adaptive refinement of the same C2 pair "
                      f"({o.result['iters']} flow solves, {o.result['region_edges']} region "
                      "edges), single-threaded sequential Dinic oracle"}
        progress(f"C2 CPU baseline: {dt:.1f} s, bit-exact {out['bit_exact_vs_oracle']}")
    return out


def _csv_rows(root: str, suffix: str):
    import csv

    rows = []
    for dp, _, files in os.walk(root):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(dp, f), newline="") as fh:
                    rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {root}")
    return rows


def _col(row: dict, *names):
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def summarize(argv):
    """Summaries of rocprofv3 output under profiles/ (runs on the host only):
      stats WORKLOAD DIR CMD...  -- the --kernel-trace --stats table of DIR
          -> profiles/k_flow_WORKLOAD_kernel_stats.md
      pmc WORKLOAD FETCH_DIR WRITE_DIR STATS_DIR CMD...  -- two --pmc runs
          (FETCH_SIZE, then WRITE_SIZE) of a command with --copy-probe: the
          mean per k_flow dispatch, each scaled by the ratio of the true byte
          count of the 512 MiB copy to what the same counter read for it; and
          the same for every other kernel, with its mean duration from the
          --kernel-trace --stats run of the same command in STATS_DIR (GB/s
          against the 8 TB/s peak)
          -> profiles/k_flow_WORKLOAD_traffic.{md,json}
    CMD is the command line that produced the output, recorded verbatim."""
    kind, work = argv[0], argv[1]
    out_dir = os.path.join(ROOT, "profiles")
    if kind == "stats":
        src, cmd = argv[2], " ".join(argv[3:])
        rows = _csv_rows(src, "kernel_stats.csv")
        rows.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
        lines = [f"# Kernel time, {work}", "",
                 "Command (from the repository root on the GPU box):", "", "```", cmd, "```", "",
                 "| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
        for r in rows:
            lines.append(f"| {_col(r, 'Name')} | {_col(r, 'Calls')} | "
                         f"{float(_col(r, 'TotalDurationNs')) / 1e6:.3f} | "
                         f"{float(_col(r, 'AverageNs')) / 1e3:.1f} | "
                         f"{float(_col(r, 'Percentage')):.2f} |")
        path = os.path.join(out_dir, f"k_flow_{work}_kernel_stats.md")
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        print(path)
        return
    if kind != "pmc":
        raise SystemExit("summarize: stats or pmc")
    fdir, wdir, sdir, cmd = argv[2], argv[3], argv[4], " ".join(argv[5:])

    def per_dispatch(root, counter):
        vals, names = {}, {}
        for r in _csv_rows(root, "counter_collection.csv"):
            if _col(r, "Counter_Name") != counter:
                continue
            d = _col(r, "Dispatch_Id")
            vals[d] = vals.get(d, 0.0) + float(_col(r, "Counter_Value"))
            names[d] = _col(r, "Kernel_Name")
        return vals, names

    res = {}
    for counter, root in (("FETCH_SIZE", fdir), ("WRITE_SIZE", wdir)):
        vals, names = per_dispatch(root, counter)
        flow = [v for d, v in vals.items() if "k_flow" in names[d]]
        copies = [v for d, v in vals.items() if "copy" in names[d].lower()]
        kname = next(names[d] for d in vals if "k_flow" in names[d])
        res[counter] = (sum(flow) / len(flow), len(flow), max(copies), kname)
    probe_kib = COPY_PROBE_BYTES / 1024
    fscale = probe_kib / res["FETCH_SIZE"][2]
    wscale = probe_kib / res["WRITE_SIZE"][2]
    fk, nl, _, kname = res["FETCH_SIZE"]
    wk = res["WRITE_SIZE"][0]
    hbm = (fk * fscale + wk * wscale) * 1024
    d = {"kernel": kname, "workload": work, "launches": nl, "fetch_kib_per_launch": fk,
         "write_kib_per_launch": wk, "copy_probe_bytes": COPY_PROBE_BYTES,
         "copy_fetch_kib": res["FETCH_SIZE"][2], "copy_write_kib": res["WRITE_SIZE"][2],
         "fetch_scale": fscale, "write_scale": wscale, "hbm_bytes_per_launch": hbm,
         "kernel_source_hash": kernel_source_hash(), "command": cmd}
    # every kernel: scaled HBM bytes per launch, mean duration, bandwidth
    fv, fn = per_dispatch(fdir, "FETCH_SIZE")
    wv, wn = per_dispatch(wdir, "WRITE_SIZE")
    per_k = {}
    for vals, names, scale, slot in ((fv, fn, fscale, 0), (wv, wn, wscale, 1)):
        for dsp, v in vals.items():
            e = per_k.setdefault(names[dsp], [0.0, 0.0, 0, 0])
            e[slot] += v * scale * 1024
            e[2 + slot] += 1
    avg_ns = {_col(r, "Name"): float(_col(r, "AverageNs")) for r in _csv_rows(sdir, "kernel_stats.csv")}
    kernels = []
    for name, (fb, wb, nf, nw) in per_k.items():
        if "copy" in name.lower() or nf == 0:
            continue
        b = fb / nf + (wb / nw if nw else 0.0)
        t = avg_ns.get(name)
        kernels.append({"kernel": name, "launches": nf, "hbm_bytes_per_launch": b,
                        "avg_us": t / 1e3 if t else None,
                        "gb_per_s": b / t if t else None,
                        "frac_of_peak": b / t / 8000.0 if t else None})
    kernels.sort(key=lambda e: -(e["hbm_bytes_per_launch"] * e["launches"]))
    d["kernels"] = kernels
    with open(os.path.join(out_dir, f"k_flow_{work}_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
    md = [f"# HBM traffic of {kname}, {work}", "",
          "Two counter passes, FETCH_SIZE then WRITE_SIZE, each its own run of this command "
          "(from the repository root on the GPU box):", "", "```", cmd, "```", "",
          "Calibration: one 512 MiB device copy in the same run (`--copy-probe`).", "",
          "| | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---:|---:|",
          f"| copy of 512 MiB | {res['FETCH_SIZE'][2]:.1f} | {res['WRITE_SIZE'][2]:.1f} |",
          f"| scale to true bytes | {fscale:.3f} | {wscale:.3f} |",
          f"| {kname}, mean per launch ({nl} launches) | {fk:.1f} | {wk:.1f} |", "",
          f"HBM bytes per launch (scaled): {hbm / 1e6:.2f} MB.", "",
          "Every kernel of the run (scaled FETCH_SIZE + WRITE_SIZE per launch; mean duration from "
          "the `--kernel-trace --stats` run of the same command; the peak is 8 TB/s):", "",
          "| kernel | launches | HBM MB per launch | mean us | GB/s | % of peak |",
          "|---|---:|---:|---:|---:|---:|"]
    for e in kernels:
        md.append(f"| {e['kernel']} | {e['launches']} | {e['hbm_bytes_per_launch'] / 1e6:.2f} | "
                  + (f"{e['avg_us']:.1f} | {e['gb_per_s']:.0f} | {100 * e['frac_of_peak']:.1f} |"
                     if e["avg_us"] else "| | |"))
    md += ["", f"Kernel sources hash: {d['kernel_source_hash']}."]
    with open(os.path.join(out_dir, f"k_flow_{work}_traffic.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(d))


def copy_probe(torch):
    """One device copy of COPY_PROBE_BYTES: the byte counters' calibration."""
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-thread-pairs", type=int, default=8)
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--c2-steps", type=int, default=10)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-balanced", action="store_true")
    ap.add_argument("--no-multitry", action="store_true")
    ap.add_argument("--mt-configs", default="C3")
    ap.add_argument("--max-sweeps", type=int, default=64)
    ap.add_argument("--c2-only", action="store_true",
                    help="only the C2 pair leg, printed as its own JSON line (for profiling it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device copy of 512 MiB (calibrates HBM byte counters)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="stats WORKLOAD DIR CMD... | pmc WORKLOAD FETCH_DIR WRITE_DIR CMD...: "
                         "write the profiles/ summaries from rocprofv3 output (no GPU)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the pairs of a round "
                                   "would shard across GPUs, but no multi-GPU path is built); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    import gen
    import paper_1012_0006_amd as fr

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    fr.load()  # fails loudly when the HIP library is not built

    if args.c2_only:
        c2 = c2_leg(argparse.Namespace(**dict(vars(args), steps=args.c2_steps, warmup=2)), fr,
                    torch, gen)
        if args.copy_probe:
            copy_probe(torch)
        print(json.dumps({"c2_plain": c2}), flush=True)
        return
    h = run_c5_headline(args, fr, torch, gen)
    progress(f"C5 headline: {h['wall'] * 1e3 / args.steps:.0f} ms per step, "
             f"cut {h['cut0']} -> {h['cut']}")
    if args.copy_probe:
        copy_probe(torch)
    line = {
        "metric": METRIC,
        "value": h["edges"] / h["wall"],
        "unit": "region edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["wall"] * 1e3 / args.steps,
        "ms_per_step_median": float(np.median(h["step_ms"])),
        "ms_per_step_min": float(np.min(h["step_ms"])),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": C5_WORKLOAD,
            "region_edges_per_step": h["edges"] // args.steps,
            "flow_solves_per_step": h["solves"] // args.steps,
            "sweeps_per_step": h["sweeps"] // args.steps,
            "cut_before": h["cut0"],
            "cut_after": h["cut"],
            "same_partition_every_step": h["repeatable"],
        },
        "roofline": roofline(h["bytes"], h["kern_ms"], h["launches"], load_traffic("C5")),
        "phase_ms_per_step": {"corridor": h["corridor_ms"] / args.steps,
                              "network_build": h["build_ms"] / args.steps,
                              "flow_kernel": h["kern_ms"] / args.steps},
        "push_relabel_sweeps_per_step": h["sweeps_pr"] // args.steps,
        "global_relabels_per_step": h["relabels"] // args.steps,
        # over the recorded solves; the work of discarded speculative solves
        # is included in the sums
        "per_recorded_solve": {"push_relabel_sweeps": h["sweeps_pr"] / max(1, h["solves"]),
                      "global_relabels": h["relabels"] / max(1, h["solves"]),
                      "relabel_bfs_levels": h["gr_levels"] / max(1, h["solves"])},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = run_c5_cpu_baseline(args, fr, torch, h["w"])
        line["bit_exact_vs_oracle"] = line["cpu_baseline"]["bit_exact_vs_gpu_round"]
        progress(f"C5 CPU baseline: {line['cpu_baseline']['seconds']:.1f} s on "
                 f"{line['cpu_baseline']['cores']} threads, bit-exact {line['bit_exact_vs_oracle']}")
    if not args.no_learned:
        line["c5_learned_without_restart"] = run_c5_no_restart(args, fr, torch, h["w"])
        progress("C5 sweep without restarts done")
    del h
    if not args.no_c2:
        line["c2_plain"] = c2_leg(argparse.Namespace(**dict(vars(args), steps=args.c2_steps,
                                                             warmup=2)), fr, torch, gen)
    if not args.no_batched:
        line["batched"] = run_batched(args, fr, torch, gen)
        progress("C3 batched round done")
        line["batched_c5_round"] = run_batched(
            argparse.Namespace(batch_reps=1, no_cpu_baseline=True), fr, torch, gen, "C5")
        progress("C5 batched round done")
    if not args.no_learned:
        line["learned_factor"] = run_learned(args, fr, torch, gen)
        progress("C4 learned factor done")
    if not args.no_balanced:
        line["balanced"] = run_balanced(args, fr, torch, gen)
    if not args.no_multitry:
        line["multitry"] = run_multitry(args, fr, torch, gen)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

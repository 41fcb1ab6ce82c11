"""flow_refine_pair_static, the pair refinement that allocates no device
memory (its buffers come from the library's static scratch array), against
flow_refine_pair through the C ABI: two calls in a row on one context, the
second on a smaller graph, each bit-exact with the allocating entry point
(result record, trace, partition) and with the oracle; then the input
checks: a graph beyond the scratch, a host graph and unsupported options
are rejected before any device work, with the partition unchanged."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

KEYS = ("status", "iters", "final_alpha", "applied", "iter_cap", "start_alpha", "flow_value",
        "cut_before", "cut_after", "weight_a", "weight_b", "region_vertices", "region_edges")


def _prm(fr, w, **extra):
    p = {k: w.params[k] for k in ("area_mode", "depth", "alpha", "alpha_max", "adaptive",
                                  "max_iters", "eps_ppm")}
    p.update(extra)
    return p, fr.params(**p)


def test_static_entry_matches_pair_refinement(gpu_lib):
    import torch

    fr = gpu_lib
    ctx = fr.Context()
    cases = ((1 << 17, 31, {}), (1 << 13, 32, {}), (1 << 12, 33, {"terminals": 1}))
    for n, seed, extra in cases:  # each call smaller than the one before
        w = gen.config("C2", seed=seed, n_override=n)
        print(f"static entry: C2 recipe n={n} seed={seed} {extra}", flush=True)
        p, prm = _prm(fr, w, **extra)
        dg = fr.DeviceGraph.from_host(w.graph)
        part_a = torch.as_tensor(w.part.copy()).cuda()
        part_b = torch.as_tensor(w.part.copy()).cuda()
        res_a, tr_a, _ = fr.flow_refine_pair(ctx, dg, part_a, w.k, 0, 1, prm)
        res_b, tr_b = fr.flow_refine_pair_static(ctx, dg, part_b, w.k, 0, 1, prm)
        for key in KEYS:
            assert res_b[key] == res_a[key], (n, key, res_b[key], res_a[key])
        assert tr_b == tr_a
        out = part_b.cpu().numpy()
        assert np.array_equal(out, part_a.cpu().numpy())
        o = oracle.refine_pair(w.graph, w.part, w.k, 0, 1, p, want_side=False)
        assert o.trace == tr_b and np.array_equal(o.part, out)
        assert res_b["iters"] >= 1
    ctx.close()


def test_static_entry_rejects_before_device_work(gpu_lib):
    import torch

    fr = gpu_lib
    ctx = fr.Context()
    # 2D RGG n = 2^20, mean degree 8: about 8.4 M arcs, 134 MB of arc records
    w = gen.config("C2", seed=5, n_override=1 << 20)
    p, prm = _prm(fr, w)
    dg = fr.DeviceGraph.from_host(w.graph)
    part = torch.as_tensor(w.part.copy()).cuda()
    with pytest.raises(fr.FlowRefineError) as e:
        fr.flow_refine_pair_static(ctx, dg, part, w.k, 0, 1, prm)
    assert e.value.code == -10
    assert np.array_equal(part.cpu().numpy(), w.part)
    small = gen.config("C2", seed=6, n_override=1 << 12)
    p, prm = _prm(fr, small)
    host_part = small.part.copy()
    with pytest.raises(fr.FlowRefineError) as e:  # host graph
        fr.flow_refine_pair_static(ctx, small.graph, host_part, small.k, 0, 1, prm)
    assert e.value.code == -8 and np.array_equal(host_part, small.part)
    dg = fr.DeviceGraph.from_host(small.graph)
    part = torch.as_tensor(small.part.copy()).cuda()
    for extra in ({"mb_reps": 2}, {"fm_limit": 10}):
        _, prm = _prm(fr, small, **extra)
        with pytest.raises(fr.FlowRefineError) as e:
            fr.flow_refine_pair_static(ctx, dg, part, small.k, 0, 1, prm)
        assert e.value.code == -8
    assert np.array_equal(part.cpu().numpy(), small.part)
    ctx.close()

"""Input checks on graphs with hubs (vertices of more than 16 arcs, checked
through hash tables of their neighbours): a valid graph with hubs refines as
the oracle does; a repeated neighbour of a hub, an asymmetric weight on a
hub's arc, a missing reverse arc into a hub and a self loop at a hub are
each rejected with FR_E_INVALID_GRAPH and leave the partition untouched; the
entry point that allocates nothing rejects them too (it scans the lists)."""
import numpy as np
import pytest

import oracle
from gen import Graph
from tests.helpers import csr_from_edges

pytestmark = pytest.mark.gpu

KEYS = ("status", "iters", "final_alpha", "applied", "flow_value", "cut_before", "cut_after",
        "weight_a", "weight_b", "region_vertices", "region_edges")


def _hub_graph(seed=3, n=600, hubs=(0, 1, 2), deg=150):
    """A ring of 600 vertices plus three hubs joined to 150 random vertices
    each, with random weights; the partition splits the ring in half."""
    rng = np.random.default_rng(seed)
    edges = {(min(u, (u + 1) % n), max(u, (u + 1) % n)) for u in range(n)}
    for h in hubs:
        for v in rng.choice(np.arange(len(hubs), n), deg, replace=False):
            edges.add((min(h, int(v)), max(h, int(v))))
    edges = sorted(edges)
    ws = rng.integers(1, 8, len(edges)).tolist()
    g = csr_from_edges(n, edges, ws)
    part = (np.arange(n) >= n // 2).astype(np.int32)
    return g, part


def _tampered(g, fn):
    xadj, adj, w = g.xadj.copy(), g.adjncy.copy(), g.adjwgt.copy()
    fn(xadj, adj, w)
    return Graph(xadj, adj, w, g.vwgt.copy())


PRM = dict(area_mode=0, depth=0, alpha=4, alpha_max=4, adaptive=1, max_iters=4, eps_ppm=50000)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def test_valid_graph_with_hubs(gpu_lib, ctx):
    import torch

    g, part = _hub_graph()
    assert np.diff(g.xadj).max() > 16
    o = oracle.refine_pair(g, part, 2, 0, 1, PRM)
    dpart = torch.as_tensor(part.copy()).cuda()
    res, tr, _ = gpu_lib.flow_refine_pair(ctx, gpu_lib.DeviceGraph.from_host(g), dpart, 2, 0, 1,
                                          gpu_lib.params(**PRM))
    for key in KEYS:
        assert res[key] == o.result[key], key
    assert tr == o.trace
    assert np.array_equal(dpart.cpu().numpy(), o.part)


def _first_arc(g, u):
    return int(g.xadj[u])


def _cases(g):
    hub = 1
    j = _first_arc(g, hub)
    v = int(g.adjncy[j])

    def repeat(xadj, adj, w):  # the hub's second neighbour becomes a copy of its first
        adj[j + 1] = adj[j]
        w[j + 1] = w[j]

    def asym(xadj, adj, w):  # the hub's arc to v weighs one more than v's arc back
        w[j] += 1

    def missing(xadj, adj, w):  # v's arc back to the hub points elsewhere
        for q in range(int(xadj[v]), int(xadj[v + 1])):
            if adj[q] == hub:
                adj[q] = (hub + 7) if (hub + 7) not in adj[xadj[v]:xadj[v + 1]] else hub + 9
                return

    def selfloop(xadj, adj, w):
        adj[j] = hub

    return {"repeated neighbour": repeat, "asymmetric weight": asym,
            "missing reverse arc": missing, "self loop": selfloop}


@pytest.mark.parametrize("case", ["repeated neighbour", "asymmetric weight",
                                  "missing reverse arc", "self loop"])
@pytest.mark.parametrize("static", [False, True])
def test_malformed_hub_graph_rejected(gpu_lib, ctx, case, static):
    import torch

    g, part = _hub_graph()
    bad = _tampered(g, _cases(g)[case])
    dg = gpu_lib.DeviceGraph.from_host(bad)
    dpart = torch.as_tensor(part.copy()).cuda()
    print(f"malformed hub graph: {case}, static entry point {static}", flush=True)
    with pytest.raises(gpu_lib.FlowRefineError) as e:
        if static:
            gpu_lib.flow_refine_pair_static(ctx, dg, dpart, 2, 0, 1, gpu_lib.params(**PRM))
        else:
            gpu_lib.flow_refine_pair(ctx, dg, dpart, 2, 0, 1, gpu_lib.params(**PRM))
    assert e.value.code == -1
    assert np.array_equal(dpart.cpu().numpy(), part)

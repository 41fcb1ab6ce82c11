"""CPU checks of the C ABI boundary: the shared library loads without a GPU
and exports every function the public header declares; the Python binding's
struct layouts match the header's field lists."""
import ctypes
import os
import re

import pytest

import paper_1012_0006_amd as fr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flowrefine.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("fr_create", "fr_destroy", "flow_refine_pair", "flow_refine_batch",
                 "flow_refine_sweep", "fr_autotune", "fr_mlp_train", "fr_pair_features"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(fr.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(fr.EXPORTS) <= set(_declared_functions())


def _struct_fields(name):
    text = open(HEADER).read()
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", text)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, rest = decl.split(None, 1)
        for part in rest.split(","):
            fields.append((typ, part.strip().lstrip("*")))
    return fields


@pytest.mark.parametrize("cname,pycls", [("fr_params", fr.FrParams), ("fr_result", fr.FrResult),
                                          ("fr_solve", fr.FrSolve), ("fr_tuning", fr.FrTuning)])
def test_binding_struct_layout(cname, pycls):
    fields = _struct_fields(cname)
    assert [f for _, f in fields] == [f for f, _ in pycls._fields_]
    size = {"int32_t": 4, "int64_t": 8}
    for (typ, _), (_, ct) in zip(fields, pycls._fields_):
        assert ctypes.sizeof(ct) == size[typ]


def test_mlp_parameter_count():
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("library not built")
    assert fr.fr_mlp_num_params() == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 5 + 5


def test_tuning_cache_roundtrip(tmp_path, monkeypatch):
    """The JSON tuning cache: a miss runs the autotuner once and stores the
    winner under the workload's key; a hit sets it without timing."""
    import paper_1012_0006_amd as fr

    class FakeCtx:
        def __init__(self):
            self.set = []

        def set_tuning(self, **kw):
            self.set.append(kw)

    class G:
        n, narcs = 1 << 18, 2_097_152

    calls = []

    def fake_autotune(ctx, graph, part, k, pairs, prm, candidates, reps):
        calls.append(len(candidates))
        return 2, [3.0, 2.0, 1.0] + [9.0] * (len(candidates) - 3)

    monkeypatch.setattr(fr, "fr_autotune", fake_autotune)
    path = str(tmp_path / "tune.json")
    ctx = FakeCtx()
    t1 = fr.autotune_cached(ctx, G(), None, 2, [(0, 1)], None, cache_path=path, arch="gfx950")
    assert t1 == fr.DEFAULT_CANDIDATES[2] and calls == [len(fr.DEFAULT_CANDIDATES)]
    t2 = fr.autotune_cached(ctx, G(), None, 2, [(0, 1)], None, cache_path=path, arch="gfx950")
    assert t2 == t1 and len(calls) == 1 and ctx.set == [t1]
    assert fr.tuning_key("gfx950", 1 << 18, 2_097_152, 1) == "gfx950|n2^18|deg8|pairs2^0"
    # another size bucket misses
    fr.autotune_cached(ctx, type("H", (), {"n": 1 << 20, "narcs": 12 << 20})(), None, 16,
                       [(0, 1)] * 8, None, cache_path=path, arch="gfx950")
    assert len(calls) == 2


def test_eps_to_ppm():
    """The double helper of fr_params.eps_ppm (no GPU work): rounding to the
    nearest part per million, and rejection outside [0, 100] and of NaN."""
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("library not built")
    assert fr.eps_to_ppm(0.03) == 30000
    assert fr.eps_to_ppm(0.0) == 0
    assert fr.eps_to_ppm(0.0300004) == 30000 and fr.eps_to_ppm(0.0300006) == 30001
    assert fr.eps_to_ppm(1.0) == 1_000_000
    for bad in (-1e-9, float("nan"), 100.5):
        with pytest.raises(fr.FlowRefineError) as e:
            fr.eps_to_ppm(bad)
        assert e.value.code == -8

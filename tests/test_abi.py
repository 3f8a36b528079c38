"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/henn.h declares, fills defaults, and rejects invalid
arguments before touching a device."""
import ctypes

import pytest

hn = pytest.importorskip("paper_2505_17368_amd.henn")


@pytest.fixture(scope="module")
def lib():
    return hn.load_library()


def test_exports_every_declared_symbol(lib):
    names = hn.header_symbols()
    assert {"henn_build", "henn_search_batch", "henn_free"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header(lib):
    p = hn.default_build_params()
    assert p.struct_size == ctypes.sizeof(hn.BuildParams) == 96
    sp = hn.SearchParams()
    assert lib.henn_default_search_params(ctypes.byref(sp)) == hn.HENN_OK
    assert sp.struct_size == ctypes.sizeof(hn.SearchParams) == 112
    assert ctypes.sizeof(hn.LayerInfo) == 56


def test_defaults(lib):
    p = hn.default_build_params()
    assert (p.metric, p.max_layers, p.m, p.c0, p.num_rings, p.max_attempts, p.degree,
            p.max_degree, p.graph, p.storage, p.seed, p.root_complete_max, p.sampler,
            p.ef_construction, p.insert_shift, p.phi, p.gram) == (
                0, -1, 4, 1.0, 64, 64, 16, 32, 0, 0, 0, 0, 0, 256, 3, 0.5, 0)
    sp = hn.SearchParams()
    lib.henn_default_search_params(ctypes.byref(sp))
    assert (sp.k_all, sp.ef_all, sp.k_max, sp.ef_upper, sp.rerank_factor) == (10, 32, 10, 1, 4)


def test_invalid_arguments_rejected_on_host(lib):
    p = hn.default_build_params()
    h = ctypes.c_void_p()
    assert lib.henn_build(None, 10, 4, ctypes.byref(p), None, ctypes.byref(h)) == hn.HENN_E_INVAL
    assert "null" in hn.last_error()
    fake = ctypes.c_void_p(0x1000)
    assert lib.henn_build(fake, 0, 4, ctypes.byref(p), None, ctypes.byref(h)) == hn.HENN_E_INVAL
    assert lib.henn_build(fake, 10, 0, ctypes.byref(p), None, ctypes.byref(h)) == hn.HENN_E_INVAL
    assert lib.henn_build(fake, 2**31, 4, ctypes.byref(p), None,
                          ctypes.byref(h)) == hn.HENN_E_INVAL
    bad = hn.default_build_params()
    bad.struct_size = 8
    assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None, ctypes.byref(h)) == hn.HENN_E_INVAL
    bad = hn.default_build_params(degree=0)
    assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None, ctypes.byref(h)) == hn.HENN_E_INVAL
    # graph kinds: 0..4; the ones with reverse edges and NSW need degree <= max_degree <= 64
    for graph, maxdeg in ((5, 32), (-1, 32), (3, 8), (3, 65), (1, 65), (4, 8), (4, 65)):
        bad = hn.default_build_params(degree=16, graph=graph, max_degree=maxdeg)
        assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None,
                              ctypes.byref(h)) == hn.HENN_E_INVAL, (graph, maxdeg)
        assert "graph" in hn.last_error() or "max_degree" in hn.last_error()
    assert hn.GRAPH == {"knn": 0, "knn_sym": 1, "pruned": 2, "pruned_sym": 3, "nsw": 4}
    # max_attempts 0 derives the cap from phi, which must then lie in (0, 1)
    for kw in (dict(max_attempts=-1), dict(max_attempts=0, phi=0.0),
               dict(max_attempts=0, phi=1.0)):
        bad = hn.default_build_params(**kw)
        assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None,
                              ctypes.byref(h)) == hn.HENN_E_INVAL, kw
        assert "max_attempts" in hn.last_error()
    # Gram tiles: 0 split BF16, 1 FP32
    for g in (-1, 2):
        bad = hn.default_build_params(gram=g)
        assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None,
                              ctypes.byref(h)) == hn.HENN_E_INVAL
        assert "gram" in hn.last_error()
    for kw in (dict(ef_construction=0), dict(ef_construction=2049), dict(insert_shift=-1),
               dict(insert_shift=63)):
        bad = hn.default_build_params(graph="nsw", **kw)
        assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None,
                              ctypes.byref(h)) == hn.HENN_E_INVAL, kw
    # NSW insertion batch: argument checks happen on the host
    ok = dict(s=100, d=8, metric=0, M=16, lo=10, hi=20, R=8, ef=32)
    for kw in (dict(lo=30), dict(hi=101), dict(lo=-1), dict(R=0), dict(R=33), dict(M=4),
               dict(M=65), dict(ef=0), dict(ef=4096), dict(d=0), dict(d=1025), dict(metric=2),
               dict(s=0)):
        a = {**ok, **kw}
        assert lib.henn_nsw_insert(fake, a["s"], a["d"], a["metric"], fake, a["M"], a["lo"],
                                   a["hi"], a["R"], a["ef"], None) == hn.HENN_E_INVAL, kw
    assert lib.henn_nsw_insert(None, 100, 8, 0, fake, 16, 0, 1, 8, 32, None) == hn.HENN_E_INVAL
    assert lib.henn_insert(None, fake, 10, None) == hn.HENN_E_INVAL
    assert lib.henn_delete(None, fake, 10, None) == hn.HENN_E_INVAL
    assert lib.henn_nsw_insert(fake, 100, 8, 0, fake, 16, 5, 5, 8, 32, None) == hn.HENN_OK
    assert hn.default_build_params(graph="pruned_sym").graph == 3
    # samplers: 0 draws (Alg. 2), 1 halving (Alg. 3)
    for sampler in (2, -1):
        bad = hn.default_build_params(sampler=sampler)
        assert lib.henn_build(fake, 10, 4, ctypes.byref(bad), None,
                              ctypes.byref(h)) == hn.HENN_E_INVAL
        assert "sampler" in hn.last_error()
    assert hn.default_build_params(sampler="halving").sampler == 1
    sp = hn.SearchParams()
    lib.henn_default_search_params(ctypes.byref(sp))
    assert lib.henn_search_batch(None, fake, 1, ctypes.byref(sp), fake, fake,
                                 None) == hn.HENN_E_INVAL
    assert lib.henn_index_shape(None, None, None, None) == hn.HENN_E_INVAL
    lib.henn_free(None)  # no-op


def test_import_validation_on_host(lib):
    import numpy as np
    p = hn.default_build_params()
    fake = ctypes.c_void_p(0x1000)
    h = ctypes.c_void_p()
    adj = np.array([[1, 1], [0, -1], [0, 1]], dtype=np.int32)  # duplicate neighbour in row 0
    sizes = (ctypes.c_int64 * 1)(3)
    ids = (ctypes.c_void_p * 1)(None)
    adjp = (ctypes.c_void_p * 1)(adj.ctypes.data)
    st = lib.henn_import(fake, 3, 4, ctypes.byref(p), 1, sizes, ids, adjp, 2, None,
                         ctypes.byref(h))
    assert st == hn.HENN_E_INVAL and "duplicate" in hn.last_error()
    adj = np.array([[1, 5], [0, -1], [0, 1]], dtype=np.int32)
    adjp = (ctypes.c_void_p * 1)(adj.ctypes.data)
    st = lib.henn_import(fake, 3, 4, ctypes.byref(p), 1, sizes, ids, adjp, 2, None,
                         ctypes.byref(h))
    assert st == hn.HENN_E_INVAL and "range" in hn.last_error()


def test_server_params_and_validation(lib):
    p = hn.ServerParams()
    assert lib.henn_default_server_params(ctypes.byref(p)) == hn.HENN_OK
    assert p.struct_size == ctypes.sizeof(hn.ServerParams) == 48
    assert (p.max_slots, p.steps_per_tick, p.k_max, p.ef_max) == (4096, 16, 10, 128)
    out = ctypes.c_void_p()
    assert lib.henn_server_create(None, ctypes.byref(p), ctypes.byref(out)) == hn.HENN_E_INVAL
    assert lib.henn_server_tick(None, None) == hn.HENN_E_INVAL
    assert lib.henn_server_cancel(None, 1, None) == hn.HENN_E_INVAL
    lib.henn_server_destroy(None)


def test_binding_constants_match_header():
    """Every enumerator and flag the binding mirrors has the header's value."""
    import os
    import re
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    text = (open(os.path.join(inc, "henn.h")).read() +
            open(os.path.join(inc, "henn_testing.h")).read())
    values = {m.group(1): int(m.group(2))
              for m in re.finditer(r"\b(HENN_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    values.update({m.group(1): int(m.group(2))
                   for m in re.finditer(r"#define\s+(HENN_[A-Z0-9_]+)\s+(\d+)u", text)})
    mirrored = [n for n in dir(hn) if n.startswith("HENN_") and isinstance(getattr(hn, n), int)]
    assert len(mirrored) >= 20
    for name in mirrored:
        assert name in values, name
        assert getattr(hn, name) == values[name], name
    for table, prefix in ((hn.GRAPH, "HENN_GRAPH_"), (hn.SAMPLER, "HENN_SAMPLER_")):
        for key, v in table.items():
            assert values[prefix + key.upper()] == v, (prefix, key)
    assert hn.STORAGE == {"f32": values["HENN_F32"], "bf16": values["HENN_BF16"],
                          "fp8": values["HENN_FP8_E4M3"]}

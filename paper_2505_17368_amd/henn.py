"""Python binding of libhenn (include/henn.h): argument marshalling only.

Every step of building and searching runs in the HIP library; this module
only converts torch tensors to device pointers and structs.  The names match
the C ABI: :func:`henn_build`, :func:`henn_search_batch`, :func:`henn_free`,
plus the inspection calls.  Loading fails loudly when ``libhenn.so`` is
missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhenn.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "henn.h")
TESTING_HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "henn_testing.h")

HENN_OK, HENN_E_INVAL, HENN_E_NOMEM, HENN_E_DEVICE, HENN_E_UNSUPPORTED = 0, 1, 2, 3, 4
HENN_W_NOT_VERIFIED = 100
HENN_L2, HENN_IP = 0, 1
HENN_F32, HENN_BF16, HENN_FP8_E4M3 = 0, 1, 2
HENN_GRAPH_KNN, HENN_GRAPH_KNN_SYM, HENN_GRAPH_PRUNED, HENN_GRAPH_PRUNED_SYM = 0, 1, 2, 3
GRAPH = {"knn": 0, "knn_sym": 1, "pruned": 2, "pruned_sym": 3, "nsw": 4}
SAMPLER = {"draws": 0, "halving": 1}
HENN_SEARCH_COUNTERS, HENN_SEARCH_PERSISTENT, HENN_SEARCH_EXACT_VISITED = 1, 2, 64
# test-only flags (include/henn_testing.h)
HENN_SEARCH_NO_ROOT_KERNEL, HENN_SEARCH_ROOT_VALU, HENN_SEARCH_VIS32, HENN_SEARCH_VIS16 = 4, 8, 16, 32
STORAGE = {"f32": HENN_F32, "bf16": HENN_BF16, "fp8": HENN_FP8_E4M3}
METRIC = {"l2": HENN_L2, "ip": HENN_IP}


class BuildParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("metric", ctypes.c_int32),
                ("max_layers", ctypes.c_int32), ("m", ctypes.c_int32), ("c0", ctypes.c_double),
                ("eps_override", ctypes.c_double), ("num_rings", ctypes.c_int32),
                ("max_attempts", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("root_complete_max", ctypes.c_int32), ("sampler", ctypes.c_int32),
                ("ef_construction", ctypes.c_int32), ("insert_shift", ctypes.c_int32),
                ("phi", ctypes.c_double), ("gram", ctypes.c_int32)]


class SearchParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("k", ctypes.c_void_p), ("ef", ctypes.c_void_p), ("k_all", ctypes.c_int32),
                ("ef_all", ctypes.c_int32), ("k_max", ctypes.c_int32), ("ef_max", ctypes.c_int32),
                ("ef_upper", ctypes.c_int32), ("rerank_factor", ctypes.c_int32),
                ("counters", ctypes.c_void_p), ("lanes_per_vec", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("ev_begin", ctypes.c_void_p),
                ("ev_end", ctypes.c_void_p), ("vis_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_int64), ("query_ns", ctypes.c_void_p)]


class LayerInfo(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("draws", ctypes.c_int64), ("eps", ctypes.c_double),
                ("window", ctypes.c_int64), ("attempts", ctypes.c_int32),
                ("hits", ctypes.c_int32), ("status", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("fallback_rows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_slots", ctypes.c_int32),
                ("pool_bytes", ctypes.c_int64), ("steps_per_tick", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("ef_max", ctypes.c_int32),
                ("ef_upper", ctypes.c_int32), ("rerank_factor", ctypes.c_int32),
                ("lanes_per_vec", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("vis_bits", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("pending", "active", "completed", "admitted",
                                              "ticks", "pool_bytes_used", "max_active",
                                              "done_queued", "cancelled")]


STATUS_NAMES = {0: "base", 1: "vacuous", 2: "verified", 3: "not_verified"}

_lib = None


class HennError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"henn status {status}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Loads libhenn.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime with the same soname; loading torch first
    # makes libhenn bind to that one, so the process holds a single runtime
    # (two runtimes in one process do not share the device).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.henn_last_error.restype = ctypes.c_char_p
    lib.henn_default_build_params.argtypes = [P(BuildParams)]
    lib.henn_default_search_params.argtypes = [P(SearchParams)]
    lib.henn_build.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, P(BuildParams), vp, P(vp)]
    lib.henn_search_batch.argtypes = [vp, vp, ctypes.c_int64, P(SearchParams), vp, vp, vp]
    lib.henn_search_batch_noalloc.argtypes = [vp, vp, ctypes.c_int64, P(SearchParams), vp, vp,
                                              vp]
    lib.henn_free.argtypes = [vp]
    lib.henn_free.restype = None
    lib.henn_index_shape.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_int32)]
    lib.henn_layer_info_get.argtypes = [vp, ctypes.c_int32, P(LayerInfo)]
    lib.henn_export_layer.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.henn_autotune.argtypes = [vp, vp, ctypes.c_int64, P(SearchParams), vp, P(SearchParams)]
    lib.henn_search_workspace_size.argtypes = [vp, ctypes.c_int64, P(SearchParams),
                                               P(ctypes.c_int64)]
    lib.henn_search_graph_create.argtypes = [vp, vp, ctypes.c_int64, P(SearchParams), vp, vp,
                                             P(vp)]
    lib.henn_search_graph_launch.argtypes = [vp, vp]
    lib.henn_search_graph_free.argtypes = [vp]
    lib.henn_search_graph_free.restype = None
    lib.henn_default_server_params.argtypes = [P(ServerParams)]
    lib.henn_server_create.argtypes = [vp, P(ServerParams), P(vp)]
    lib.henn_server_submit.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    lib.henn_server_tick.argtypes = [vp, P(ctypes.c_int32)]
    lib.henn_server_submit_batch.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64]
    lib.henn_server_poll.argtypes = [vp, ctypes.c_int32, vp, vp, vp, P(ctypes.c_int32)]
    lib.henn_server_stats.argtypes = [vp, P(ServerStats)]
    lib.henn_server_cancel.argtypes = [vp, ctypes.c_int64, P(ctypes.c_int32)]
    lib.henn_server_destroy.argtypes = [vp]
    lib.henn_server_destroy.restype = None
    lib.henn_import.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, P(BuildParams), ctypes.c_int32,
                                P(ctypes.c_int64), P(vp), P(vp), ctypes.c_int32, vp, P(vp)]
    lib.henn_insert.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.henn_delete.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.henn_nsw_insert.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp,
                                    ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, vp]
    for name in ("henn_default_build_params", "henn_default_search_params", "henn_build",
                 "henn_search_batch", "henn_search_batch_noalloc", "henn_index_shape",
                 "henn_layer_info_get",
                 "henn_export_layer", "henn_import", "henn_autotune",
                 "henn_search_workspace_size", "henn_search_graph_create",
                 "henn_search_graph_launch", "henn_default_server_params", "henn_server_create",
                 "henn_server_submit", "henn_server_submit_batch", "henn_server_tick",
                 "henn_server_poll",
                 "henn_server_stats", "henn_nsw_insert", "henn_insert", "henn_delete",
                 "henn_testing_fail_alloc_after"):
        getattr(lib, name).restype = ctypes.c_int
    lib.henn_testing_fail_alloc_after.argtypes = [ctypes.c_int64]
    _lib = lib
    return lib


def header_symbols(paths=(HEADER_PATH, TESTING_HEADER_PATH)):
    """Function names declared in include/henn.h and include/henn_testing.h."""
    names = set()
    for path in paths:
        txt = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names.update(re.findall(r"\b(henn_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def fail_alloc_after(n: int) -> None:
    """Test-only: the next n device allocations of the library succeed, later
    ones fail as out of memory; n < 0 turns the injector off."""
    _check(load_library().henn_testing_fail_alloc_after(int(n)))


def last_error() -> str:
    return load_library().henn_last_error().decode()


def _check(status: int, allow_warning: bool = False) -> int:
    if status == HENN_OK or (allow_warning and status == HENN_W_NOT_VERIFIED):
        return status
    raise HennError(status, last_error())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be float32 [rows, d]")
    return t.contiguous()


def default_build_params(**kw) -> BuildParams:
    p = BuildParams()
    _check(load_library().henn_default_build_params(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "metric" and isinstance(v, str):
            v = METRIC[v]
        if k == "storage" and isinstance(v, str):
            v = STORAGE[v]
        if k == "graph" and isinstance(v, str):
            v = GRAPH[v]
        if k == "sampler" and isinstance(v, str):
            v = SAMPLER[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class HennIndex:
    """Owns a henn_index* (released by :meth:`free` or garbage collection)."""

    def __init__(self, handle: ctypes.c_void_p, status: int):
        self._h = handle
        self.build_status = status

    @property
    def handle(self):
        if not self._h:
            raise ValueError("index was freed")
        return self._h

    def shape(self):
        nl, n, d = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(load_library().henn_index_shape(self.handle, ctypes.byref(nl), ctypes.byref(n),
                                               ctypes.byref(d)))
        return nl.value, n.value, d.value

    @property
    def num_layers(self) -> int:
        return self.shape()[0]

    def layer_info(self, layer: int) -> dict:
        info = LayerInfo()
        _check(load_library().henn_layer_info_get(self.handle, layer, ctypes.byref(info)))
        out = {f: getattr(info, f) for f, _ in LayerInfo._fields_ if f != "reserved"}
        out["status"] = STATUS_NAMES.get(out["status"], out["status"])
        return out

    def export_layer(self, layer: int):
        info = self.layer_info(layer)
        ids = np.zeros(info["size"], dtype=np.int32)
        adj = np.zeros((info["size"], info["degree"]), dtype=np.int32)
        _check(load_library().henn_export_layer(self.handle, layer, ids.ctypes.data_as(
            ctypes.c_void_p), adj.ctypes.data_as(ctypes.c_void_p)))
        return ids, adj

    def free(self):
        if self._h:
            load_library().henn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def henn_build(X, params: BuildParams | None = None, stream=None, **kw) -> HennIndex:
    """Alg. 1 on the GPU; X is a float32 [n, d] device tensor (copied)."""
    X = _dev_f32(X, "X")
    p = params if params is not None else default_build_params(**kw)
    h = ctypes.c_void_p()
    st = load_library().henn_build(ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1],
                                   ctypes.byref(p), _stream_ptr(stream), ctypes.byref(h))
    _check(st, allow_warning=True)
    return HennIndex(h, st)


def henn_import(X, ids_per_layer, adj_per_layer, params: BuildParams | None = None, stream=None,
                **kw) -> HennIndex:
    """Index from given layers (host arrays): ids ascending, adjacency as
    positions within each layer, -1 padded, equal row width across layers."""
    X = _dev_f32(X, "X")
    p = params if params is not None else default_build_params(**kw)
    L = len(adj_per_layer)
    stride = int(adj_per_layer[0].shape[1])
    ids_keep = [None if (i == 0 and ids_per_layer[0] is None) else
                np.ascontiguousarray(ids_per_layer[i], dtype=np.int32) for i in range(L)]
    adj_keep = []
    for a in adj_per_layer:
        a = np.asarray(a, dtype=np.int32)
        if a.shape[1] < stride:
            a = np.concatenate([a, -np.ones((a.shape[0], stride - a.shape[1]), np.int32)], 1)
        adj_keep.append(np.ascontiguousarray(a[:, :stride]))
    sizes = (ctypes.c_int64 * L)(*[a.shape[0] for a in adj_keep])
    ids_arr = (ctypes.c_void_p * L)(*[None if x is None else x.ctypes.data for x in ids_keep])
    adj_arr = (ctypes.c_void_p * L)(*[x.ctypes.data for x in adj_keep])
    h = ctypes.c_void_p()
    st = load_library().henn_import(ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1],
                                    ctypes.byref(p), L, sizes, ids_arr, adj_arr, stride,
                                    _stream_ptr(stream), ctypes.byref(h))
    _check(st)
    return HennIndex(h, st)


def henn_insert(index: HennIndex, X_new, stream=None) -> None:
    """Insert(x) of the dynamic setting for an NSW-graph index: X_new is a
    float32 [count, d] device tensor; the new points get ids n .. n+count-1."""
    X_new = _dev_f32(X_new, "X_new")
    _check(load_library().henn_insert(index.handle, ctypes.c_void_p(X_new.data_ptr()),
                                      X_new.shape[0], _stream_ptr(stream)))


def henn_delete(index: HennIndex, ids, stream=None) -> None:
    """Delete(x) of the dynamic setting for an NSW-graph index; ids: host ints."""
    arr = np.ascontiguousarray(np.asarray(ids, dtype=np.int32).ravel())
    _check(load_library().henn_delete(index.handle, arr.ctypes.data_as(ctypes.c_void_p),
                                      arr.size, _stream_ptr(stream)))


def henn_nsw_insert(V, adj, lo: int, hi: int, degree: int, ef_construction: int,
                    metric=HENN_L2, stream=None) -> None:
    """One NSW insertion batch on a caller-held graph: V device FP32 [s, d],
    adj device int32 [s, max_degree] (updated in place)."""
    import torch
    V = _dev_f32(V, "V")
    if not (adj.is_cuda and adj.dtype == torch.int32 and adj.is_contiguous()
            and adj.dim() == 2 and adj.shape[0] == V.shape[0]):
        raise ValueError("adj must be a contiguous int32 device tensor [s, max_degree]")
    if isinstance(metric, str):
        metric = METRIC[metric]
    _check(load_library().henn_nsw_insert(
        ctypes.c_void_p(V.data_ptr()), V.shape[0], V.shape[1], metric,
        ctypes.c_void_p(adj.data_ptr()), adj.shape[1], lo, hi, degree, ef_construction,
        _stream_ptr(stream)))


def search_params(k=10, ef=32, k_arr=None, ef_arr=None, k_max=None, ef_max=None, ef_upper=1,
                  rerank_factor=4, counters=None, persistent=False, lanes_per_vec=0,
                  waves_per_block=0, root_kernel=True, events=None,
                  vis_bits=0, vis32=False, vis16=False, workspace=None,
                  exact_visited=False, query_ns=None) -> SearchParams:
    sp = SearchParams()
    _check(load_library().henn_default_search_params(ctypes.byref(sp)))
    sp.k_all = k
    sp.ef_all = ef
    sp.k = k_arr.data_ptr() if k_arr is not None else None
    sp.ef = ef_arr.data_ptr() if ef_arr is not None else None
    sp.k_max = k_max if k_max is not None else k
    sp.ef_max = ef_max if ef_max is not None else ef
    sp.ef_upper = ef_upper
    sp.rerank_factor = rerank_factor
    sp.counters = counters.data_ptr() if counters is not None else None
    sp.query_ns = query_ns.data_ptr() if query_ns is not None else None
    # root_kernel: True (matrix-core scan where available), "valu" (tiled
    # VALU scan) or False (scan inside the search kernel); same results
    if root_kernel not in (True, False, "valu"):
        raise ValueError("root_kernel must be True, False or 'valu'")
    sp.flags = (HENN_SEARCH_PERSISTENT if persistent else 0) | (
        HENN_SEARCH_COUNTERS if counters is not None else 0) | (
        HENN_SEARCH_NO_ROOT_KERNEL if root_kernel is False else 0) | (
        HENN_SEARCH_ROOT_VALU if root_kernel == "valu" else 0) | (
        HENN_SEARCH_VIS32 if vis32 else 0) | (HENN_SEARCH_VIS16 if vis16 else 0) | (
        HENN_SEARCH_EXACT_VISITED if exact_visited else 0)
    sp.lanes_per_vec = lanes_per_vec
    sp.waves_per_block = waves_per_block
    sp.vis_bits = vis_bits
    if events is not None:
        sp.ev_begin = events[0].cuda_event
        sp.ev_end = events[1].cuda_event
    if workspace is not None:
        sp.workspace = workspace.data_ptr()
        sp.workspace_bytes = workspace.numel() * workspace.element_size()
    return sp


def workspace_size(index: HennIndex, nq: int, **kw) -> int:
    """Scratch bytes henn_search_batch needs for nq queries with these
    search arguments (see search_params)."""
    sp = search_params(**kw)
    b = ctypes.c_int64()
    _check(load_library().henn_search_workspace_size(index.handle, nq, ctypes.byref(sp),
                                                     ctypes.byref(b)))
    return b.value


def henn_search_batch(index: HennIndex, Q, k=10, ef=32, k_arr=None, ef_arr=None, k_max=None,
                      ef_max=None, ef_upper=1, rerank_factor=4, with_counters=False,
                      persistent=False, lanes_per_vec=0, waves_per_block=0, root_kernel=True,
                      events=None, vis_bits=0, out_ids=None, out_dist=None, stream=None,
                      vis32=False, vis16=False, noalloc=False, workspace=None,
                      exact_visited=False, with_times=False):
    """Enqueues a batched search; returns (ids, dist[, counters][, query_ns])
    device tensors (query_ns: int64 per-query time in the search kernel).
    ``noalloc``: call henn_search_batch_noalloc (the library's fixed scratch;
    pass out_ids / out_dist to keep the call free of allocations here too).

    ``events``: optional pair of recorded torch.cuda.Event (enable_timing) that
    the library re-records around the main search kernel."""
    import torch
    Q = _dev_f32(Q, "Q")
    nq = Q.shape[0]
    kmax = k_max if k_max is not None else (int(k_arr.max().item()) if k_arr is not None else k)
    if ef_arr is not None and ef_max is None:
        ef_max = int(ef_arr.max().item())
    if out_ids is None:
        out_ids = torch.empty((nq, kmax), dtype=torch.int32, device=Q.device)
    if out_dist is None:
        out_dist = torch.empty((nq, kmax), dtype=torch.float32, device=Q.device)
    counters = torch.zeros((nq, 4), dtype=torch.int32, device=Q.device) if with_counters else None
    times = torch.zeros(nq, dtype=torch.int64, device=Q.device) if with_times else None
    sp = search_params(k, ef, k_arr, ef_arr, kmax, ef_max, ef_upper, rerank_factor, counters,
                       persistent, lanes_per_vec, waves_per_block, root_kernel, events,
                       vis_bits, vis32, vis16, workspace, exact_visited, times)
    entry = load_library().henn_search_batch_noalloc if noalloc else \
        load_library().henn_search_batch
    _check(entry(index.handle, ctypes.c_void_p(Q.data_ptr()), nq, ctypes.byref(sp),
                 ctypes.c_void_p(out_ids.data_ptr()), ctypes.c_void_p(out_dist.data_ptr()),
                 _stream_ptr(stream)))
    out = (out_ids, out_dist) + ((counters,) if with_counters else ()) + (
        (times,) if with_times else ())
    return out


def henn_autotune(index: HennIndex, Q, k=10, ef=32, k_max=None, ef_max=None, ef_upper=1,
                  rerank_factor=4, k_arr=None, ef_arr=None, stream=None) -> dict:
    """Tunes and caches the launch shape for this (storage, beam, k) bucket
    on the calibration queries Q; returns the chosen shape."""
    Q = _dev_f32(Q, "Q")
    kmax = k_max if k_max is not None else k
    sp = search_params(k, ef, k_arr, ef_arr, kmax, ef_max if ef_max is not None else ef,
                       ef_upper, rerank_factor)
    out = SearchParams()
    _check(load_library().henn_autotune(index.handle, ctypes.c_void_p(Q.data_ptr()), Q.shape[0],
                                        ctypes.byref(sp), _stream_ptr(stream),
                                        ctypes.byref(out)))
    return {"lanes_per_vec": out.lanes_per_vec, "waves_per_block": out.waves_per_block,
            "vis_bits": out.vis_bits, "persistent": bool(out.flags & HENN_SEARCH_PERSISTENT)}


class SearchGraph:
    """A batched search captured once in a hipGraph (henn_search_graph_*).

    Q and the outputs are bound at capture; refill ``self.Q`` in place and
    call :meth:`launch` to replay."""

    def __init__(self, index: HennIndex, Q, k=10, ef=32, k_arr=None, ef_arr=None, k_max=None,
                 ef_max=None, ef_upper=1, rerank_factor=4, persistent=True):
        import torch
        self.index = index
        self.Q = _dev_f32(Q, "Q")
        nq = self.Q.shape[0]
        kmax = k_max if k_max is not None else k
        self.k_arr, self.ef_arr = k_arr, ef_arr
        self.ids = torch.empty((nq, kmax), dtype=torch.int32, device=self.Q.device)
        self.dist = torch.empty((nq, kmax), dtype=torch.float32, device=self.Q.device)
        sp = search_params(k, ef, k_arr, ef_arr, kmax, ef_max if ef_max is not None else ef,
                           ef_upper, rerank_factor, persistent=persistent)
        self._g = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(load_library().henn_search_graph_create(
            index.handle, ctypes.c_void_p(self.Q.data_ptr()), nq, ctypes.byref(sp),
            ctypes.c_void_p(self.ids.data_ptr()), ctypes.c_void_p(self.dist.data_ptr()),
            ctypes.byref(self._g)))

    def launch(self, stream=None):
        _check(load_library().henn_search_graph_launch(self._g, _stream_ptr(stream)))
        return self.ids, self.dist

    def free(self):
        if self._g:
            load_library().henn_search_graph_free(self._g)
            self._g = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop on one index (henn_server_*)."""

    def __init__(self, index: HennIndex, **kw):
        lib = load_library()
        p = ServerParams()
        _check(lib.henn_default_server_params(ctypes.byref(p)))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        self.k_max = p.k_max
        self.index = index
        self._s = ctypes.c_void_p()
        _check(lib.henn_server_create(index.handle, ctypes.byref(p), ctypes.byref(self._s)))

    def submit(self, q, k: int, ef: int, tag: int):
        q = np.ascontiguousarray(q, dtype=np.float32)
        _check(load_library().henn_server_submit(self._s, q.ctypes.data_as(ctypes.c_void_p), k,
                                                 ef, tag))

    def submit_batch(self, Q, ks, efs, tags):
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        efs = np.ascontiguousarray(efs, dtype=np.int32)
        tags = np.ascontiguousarray(tags, dtype=np.int64)
        vp = ctypes.c_void_p
        _check(load_library().henn_server_submit_batch(
            self._s, Q.ctypes.data_as(vp), ks.ctypes.data_as(vp), efs.ctypes.data_as(vp),
            tags.ctypes.data_as(vp), Q.shape[0]))

    def cancel(self, tag: int) -> int:
        """henn_server_cancel: 0 not found, 1 removed before admission,
        2 admitted (no result will come), 3 already finished."""
        st = ctypes.c_int32()
        _check(load_library().henn_server_cancel(self._s, int(tag), ctypes.byref(st)))
        return st.value

    def tick(self) -> int:
        n = ctypes.c_int32()
        _check(load_library().henn_server_tick(self._s, ctypes.byref(n)))
        return n.value

    def poll(self, max_results: int | None = None):
        if max_results is None:
            st = ServerStats()
            _check(load_library().henn_server_stats(self._s, ctypes.byref(st)))
            max_results = int(st.done_queued)
        if max_results <= 0:
            return (np.zeros(0, dtype=np.int64), np.zeros((0, self.k_max), dtype=np.int32),
                    np.zeros((0, self.k_max), dtype=np.float32))
        tags = np.empty(max_results, dtype=np.int64)
        ids = np.empty((max_results, self.k_max), dtype=np.int32)
        dist = np.empty((max_results, self.k_max), dtype=np.float32)
        n = ctypes.c_int32()
        _check(load_library().henn_server_poll(self._s, max_results,
                                               tags.ctypes.data_as(ctypes.c_void_p),
                                               ids.ctypes.data_as(ctypes.c_void_p),
                                               dist.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(n)))
        m = n.value
        return tags[:m], ids[:m], dist[:m]

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().henn_server_stats(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._s:
            load_library().henn_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def henn_free(index: HennIndex) -> None:
    index.free()

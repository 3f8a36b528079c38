"""FP64 CPU oracle for HENN (arXiv 2505.17368) -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library
and never imports it.  The heavy loops live in ``henn_oracle.c`` (plain C,
FP64, built with gcc by :func:`build`); this module drives them in the order
of the paper's algorithms:

* :func:`eps_of` -- Eq. (1): eps(s) = c0 * d * log(s) / s * 2^m (natural log).
* :func:`build_index` -- Alg. 1 (BuildHENN): layer i is an eps-net of layer
  i-1 drawn by Alg. 2 (BuildEpsNetSampling, samples with replacement) and
  verified against ``r`` sampled ring ranges (App. B.1 "Practical
  Implementation", App. G.2) -- or, with ``sampler=1``, drawn by Alg. 3's
  halving (:func:`halve`, BuildEpsNetDiscV2) and checked the same way; each
  layer then gets an exact kNN navigable
  graph (App. B.2, App. G.4), or (``graph=4``) the NSW graph of App. B.2
  built by batched incremental insertion (:func:`nsw_graph`).  Layer sizes follow Cor. "layer-size":
  ceil(|L_{i-1}| / 2^m) draws per layer.
* :func:`search` -- Alg. 4 (Query) from the root down, ef=1 greedy on the
  upper layers and a beam of max(ef, k) candidates on layer 0 (Sec. 2.2).
  When the root carries the complete graph (App. B.2: trivially navigable),
  greedy search on it is the exhaustive scan for the root's nearest member.
* :func:`brute_force_knn` -- exact k-NN of the problem setting (Sec. 2).

Readings where the paper is silent (all listed in the design notes):
the entry node is the smallest id of the root layer; rings are the minimal
heavy rings (a uniformly drawn centre in L_{i-1} and a uniformly drawn rank
window of width floor(eps*s)+1); rings are fixed per layer and the sample is
redrawn per attempt; after ``max_attempts`` failures the attempt with the
most hits is kept and the layer is marked not verified; the layer loop stops
before a layer whose draw count would fall below degree+1.
"""
from __future__ import annotations

import copy
import ctypes
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "henn_oracle.c")
_LIB = os.path.join(_HERE, "libhenn_oracle.so")
_lib = None
_lock = threading.Lock()

TAG_SAMPLE, TAG_RING_CENTRE, TAG_RING_START, TAG_HALVE, TAG_INSERT = 1, 2, 3, 4, 5
L2, IP = 0, 1


_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build() -> str:
    """Compile the C oracle with gcc (strict FP64: no contraction, no fast-math)."""
    cmd = ["gcc", *_CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal), for the sanitized run of the oracle's pins; load it
    by setting HENN_ORACLE_LIB to path, with libasan preloaded."""
    cmd = ["gcc", *_CFLAGS, "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", path, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return path


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = os.environ.get("HENN_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        c_i64p, c_i32p, c_f64p, c_f32p = (P(ctypes.c_int64), P(ctypes.c_int32),
                                          P(ctypes.c_double), P(ctypes.c_float))
        lib.ho_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64),
                                         P(ctypes.c_uint64)]
        lib.ho_stream_word.restype = ctypes.c_uint64
        lib.ho_stream_word.argtypes = [ctypes.c_uint64] * 5
        lib.ho_uniform_index.restype = ctypes.c_uint64
        lib.ho_uniform_index.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.ho_draw_indices.argtypes = [ctypes.c_uint64] * 4 + [ctypes.c_int64, ctypes.c_int64,
                                                                c_i64p]
        lib.ho_distance.restype = ctypes.c_double
        lib.ho_distance.argtypes = [c_f32p, c_f32p, ctypes.c_int, ctypes.c_int]
        lib.ho_ring_members.restype = ctypes.c_int
        lib.ho_ring_members.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, c_i64p, c_f64p]
        lib.ho_knn_graph.restype = ctypes.c_int
        lib.ho_knn_graph.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int, c_i32p, c_f64p,
                                     c_f64p, c_f64p]
        lib.ho_search.restype = ctypes.c_int
        lib.ho_search.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, c_i64p,
                                  P(c_i32p), P(c_i32p), c_i32p, P(c_f64p), c_f32p,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, c_i32p, c_f64p, c_f64p, c_f64p,
                                  c_i64p]
        lib.ho_nsw_repair.restype = ctypes.c_int
        lib.ho_nsw_repair.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p, ctypes.c_int64,
                                      c_i32p, ctypes.c_int, P(ctypes.c_uint8), c_f64p]
        lib.ho_nsw_insert.restype = ctypes.c_int
        lib.ho_nsw_insert.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p, ctypes.c_int64,
                                      c_i32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int, c_f64p]
        lib.ho_knn_sym.restype = ctypes.c_int
        lib.ho_knn_sym.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p, ctypes.c_int64,
                                   c_i32p, ctypes.c_int, ctypes.c_int, c_i32p, c_f64p, c_f64p]
        lib.ho_prune.restype = ctypes.c_int
        lib.ho_prune.argtypes = [c_f32p, ctypes.c_int, ctypes.c_int, c_i32p, ctypes.c_int64,
                                 c_i32p, ctypes.c_int, ctypes.c_int, c_i32p, c_f64p]
        lib.ho_brute_knn.restype = ctypes.c_int
        lib.ho_brute_knn.argtypes = [c_f32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, c_f32p,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int, c_i32p, c_f64p]
        _lib = lib
        return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _parallel(nitems: int, fn, threads: int | None = None, min_chunk: int = 1):
    """Run fn(begin, end) over [0, nitems) in contiguous chunks on threads."""
    threads = threads or default_threads()
    if nitems <= 0:
        return
    nch = max(1, min(threads * 4, (nitems + min_chunk - 1) // min_chunk))
    bounds = np.linspace(0, nitems, nch + 1).astype(np.int64)
    if threads == 1 or nch == 1:
        for b, e in zip(bounds[:-1], bounds[1:]):
            fn(int(b), int(e))
        return
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(fn, int(b), int(e)) for b, e in zip(bounds[:-1], bounds[1:]) if e > b]
        for f in futs:
            f.result()


# ---------------------------------------------------------------------------
# Randomness: Philox4x64-10, word q of stream (tag, layer, attempt)
# ---------------------------------------------------------------------------

def philox_block(counter, key):
    lib = _load()
    c = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.ho_philox4x64_10(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64),
                         _ptr(out, ctypes.c_uint64))
    return out


def stream_word(seed, tag, layer, attempt, q) -> int:
    return int(_load().ho_stream_word(seed, tag, layer, attempt, q))


def uniform_index(w: int, s: int) -> int:
    return int(_load().ho_uniform_index(w, s))


def draw_indices(seed, tag, layer, attempt, s, count) -> np.ndarray:
    out = np.zeros(max(count, 0), dtype=np.int64)
    if count > 0:
        _load().ho_draw_indices(seed, tag, layer, attempt, s, count, _ptr(out, ctypes.c_int64))
    return out


# ---------------------------------------------------------------------------
# Eq. (1) and the layer schedule
# ---------------------------------------------------------------------------

def eps_of(s: int, d: int, m: int, c0: float) -> float:
    """Eq. (1): eps(s) = c0 * d * log(s) / s * 2^m, natural logarithm."""
    return c0 * d * math.log(s) / s * (2 ** m)


def window_of(eps: float, s: int) -> int:
    """Fewest points a heavy ring can hold: |R| > eps*s  <=>  |R| >= floor(eps*s)+1."""
    return int(math.floor(eps * s)) + 1


@dataclass
class BuildParams:
    metric: int = L2
    max_layers: int = -1         # upper layers allowed; < 0: until the draw count
                                 # would drop below degree+1
    m: int = 4                   # exponential decay, 2^m = 16
    c0: float = 1.0
    eps_override: float = 0.0
    num_rings: int = 64          # r, the "range size" hyperparameter
    max_attempts: int = 64
    degree: int = 16
    seed: int = 0
    graph: int = 0               # 0: exact kNN; 1: kNN plus reverse edges (kNN_SYM);
                                 # 2: diversity-pruned kNN (PRUNED); 3: PRUNED plus
                                 # reverse edges (PRUNED_SYM); 4: NSW by batched insertion
    ef_construction: int = 256   # NSW: beam width of the insertion searches
    insert_shift: int = 3        # NSW: a batch after lo inserted points holds max(1, lo >> shift)
    max_degree: int = 32         # row cap of the graphs with reverse edges
    root_complete_max: int = 0   # > 0: stop adding layers once a layer holds at most
                                 # this many points and give that root the complete graph
    sampler: int = 0             # 0: Alg. 2 draws with replacement; 1: Alg. 3 halving
    phi: float = 0.5             # Alg. 2: failure probability of one sample (Eq. (3));
                                 # sets the attempt cap when max_attempts is 0


def attempt_cap(p: BuildParams) -> int:
    """Attempts of Alg. 2's repeat loop: max_attempts, or with 0 the smallest t
    with phi^t <= 1e-9 (each attempt fails with probability phi)."""
    if p.max_attempts > 0:
        return p.max_attempts
    return max(1, math.ceil(math.log(1e-9) / math.log(p.phi)))


@dataclass
class LayerInfo:
    size: int
    draws: int
    eps: float
    window: int
    attempts: int
    hits: int
    status: str                  # "base", "vacuous", "verified", "not_verified"
    ring_margin: float = math.inf


@dataclass
class OracleIndex:
    X: np.ndarray
    metric: int
    degree: int
    root_complete: bool = False
    members: list = field(default_factory=list)     # int32 ascending global ids per layer
    adj: list = field(default_factory=list)         # int32 [size, degree] local indices, -1 pad
    adj_dist: list = field(default_factory=list)    # float64 [size, degree]
    adj_margin: list = field(default_factory=list)  # float64 [size] margin at the R / R+1 cut
    order_margin: list = field(default_factory=list)  # float64 [size] min margin in first R+1
    info: list = field(default_factory=list)

    @property
    def num_layers(self) -> int:
        return len(self.members)


def ring_members(X, metric, members, centre_local, a, w):
    """Local indices of ring ranks [a, a+w-1] around L[centre_local] (rank 0 = centre)."""
    lib = _load()
    out = np.zeros(w, dtype=np.int64)
    mg = np.zeros(1, dtype=np.float64)
    rc = lib.ho_ring_members(_ptr(X, ctypes.c_float), X.shape[1], metric,
                             _ptr(members, ctypes.c_int32), len(members), centre_local, a, w,
                             _ptr(out, ctypes.c_int64), _ptr(mg, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"ring_members failed ({rc})")
    return out, float(mg[0])


def halve(seed, layer, attempt, s, m) -> np.ndarray:
    """Alg. 3, BuildEpsNetDiscV2: m halving steps of the positions [0, s).

    Each step matches the current members in pairs -- the paper leaves the
    matching arbitrary; here consecutive members in ascending order -- and
    keeps one member of every pair by a coin; an odd last member has no pair
    and stays.  Pair p of step j (0-based) takes its coin from word p of the
    stream (tag 4 + j, layer, attempt): u(w, 2) = 0 keeps the lower member.
    Returns the ascending survivors."""
    A = np.arange(s, dtype=np.int64)
    for j in range(m):
        a = len(A)
        pairs = a // 2
        coins = draw_indices(seed, TAG_HALVE + j, layer, attempt, 2, pairs)
        kept = A[2 * np.arange(pairs) + coins]       # member 2q or 2q+1 of pair q
        if a % 2 == 1:
            kept = np.append(kept, A[a - 1])
        A = kept
    return A


def _candidate(p: BuildParams, layer, attempt, s, D):
    """One attempt's sample: Alg. 2's D draws (with repeats) or Alg. 3's halving."""
    if p.sampler == 1:
        return halve(p.seed, layer, attempt, s, p.m)
    return draw_indices(p.seed, TAG_SAMPLE, layer, attempt, s, D)


def sample_layer(X, prev, layer, d, p: BuildParams, threads=None):
    """Alg. 2 (or Alg. 3's halving, ``p.sampler == 1``) with the practical
    IsEpsNet of App. B.1 for one layer.

    Returns (local indices of the accepted sample, ascending, distinct), LayerInfo.
    """
    s = len(prev)
    D = -(-s // (2 ** p.m))
    eps = p.eps_override if p.eps_override > 0 else eps_of(s, d, p.m, p.c0)
    w = window_of(eps, s)
    if w > s:
        draws = _candidate(p, layer, 0, s, D)
        return np.unique(draws), LayerInfo(0, D, eps, w, 1, 0, "vacuous")
    r = p.num_rings
    centres = draw_indices(p.seed, TAG_RING_CENTRE, layer, 0, s, r)
    starts = draw_indices(p.seed, TAG_RING_START, layer, 0, s - w + 1, r)
    rings = [None] * r
    margins = np.zeros(r)

    def one(b, e):
        for j in range(b, e):
            rings[j], margins[j] = ring_members(X, p.metric, prev, int(centres[j]),
                                                int(starts[j]), w)
    _parallel(r, one, threads)
    best_t, best_hits, best = -1, -1, None
    cap = attempt_cap(p)
    for t in range(cap):
        draws = _candidate(p, layer, t, s, D)
        sel = np.zeros(s, dtype=bool)
        sel[draws] = True
        hits = int(sum(bool(sel[ring].any()) for ring in rings))
        if hits > best_hits:
            best_t, best_hits, best = t, hits, draws
        if hits == r:
            return np.unique(draws), LayerInfo(0, D, eps, w, t + 1, hits, "verified",
                                               float(margins.min()))
    return np.unique(best), LayerInfo(0, D, eps, w, cap, best_hits, "not_verified",
                                      float(margins.min()))


def knn_graph(X, metric, members, R, threads=None):
    """Exact kNN graph of one layer (App. B.2): local indices, (dist, id) order.

    Returns (adjacency, FP64 distances, cut margin, order margin)."""
    lib = _load()
    s = len(members)
    adj = np.full((s, R), -1, dtype=np.int32)
    ad = np.full((s, R), np.inf)
    cut = np.full(s, np.inf)
    order = np.full(s, np.inf)

    def one(b, e):
        rc = lib.ho_knn_graph(_ptr(X, ctypes.c_float), X.shape[1], metric,
                              _ptr(members, ctypes.c_int32), s, b, e, R,
                              _ptr(adj, ctypes.c_int32), _ptr(ad, ctypes.c_double),
                              _ptr(cut, ctypes.c_double), _ptr(order, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("knn_graph failed")
    _parallel(s, one, threads, min_chunk=16)
    return adj, ad, cut, order


def knn_rows(X, metric, members, rows, R):
    """Exact kNN lists of selected rows of a layer (same definition as
    :func:`knn_graph`): returns (adjacency [len(rows), R], cut margin, order
    margin)."""
    lib = _load()
    s = len(members)
    adj = np.full((s, R), -1, dtype=np.int32)
    cut = np.full(s, np.inf)
    order = np.full(s, np.inf)
    for r in rows:
        rc = lib.ho_knn_graph(_ptr(X, ctypes.c_float), X.shape[1], metric,
                              _ptr(members, ctypes.c_int32), s, int(r), int(r) + 1, R,
                              _ptr(adj, ctypes.c_int32), None, _ptr(cut, ctypes.c_double),
                              _ptr(order, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("knn_graph failed")
    rows = np.asarray(rows)
    return adj[rows], cut[rows], order[rows]


def build_layers(X: np.ndarray, p: BuildParams, threads=None):
    """Alg. 1 layer loop: returns ascending member lists and per-layer info."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n = X.shape[0]
    members = [np.arange(n, dtype=np.int32)]
    infos = [LayerInfo(n, n, 0.0, 0, 0, 0, "base")]
    _extend_layers(X, members, infos, p, threads)
    return members, infos


def _extend_layers(X, members, infos, p: BuildParams, threads=None):
    """Alg. 1's layer loop on top of the given layers, in place."""
    d = X.shape[1]
    i = len(members)
    while True:
        s = len(members[-1])
        D = -(-s // (2 ** p.m))
        if D < p.degree + 1 or (p.max_layers >= 0 and i > p.max_layers):
            break
        if p.root_complete_max > 0 and s <= p.root_complete_max:
            break
        local, info = sample_layer(X, members[-1], i, d, p, threads)
        members.append(members[-1][local].astype(np.int32))
        info.size = len(local)
        infos.append(info)
        i += 1


def build_index(X: np.ndarray, p: BuildParams | None = None, threads=None) -> OracleIndex:
    """Alg. 1 (BuildHENN) with exact kNN graphs per layer."""
    p = p or BuildParams()
    X = np.ascontiguousarray(X, dtype=np.float32)
    members, infos = build_layers(X, p, threads)
    root_complete = p.root_complete_max > 0 and len(members) >= 2
    idx = OracleIndex(X=X, metric=p.metric, degree=p.degree, members=members, info=infos,
                      root_complete=root_complete)
    for mb in members:
        if p.graph in (2, 3):
            cands = prune_candidates(p.degree)
            a, ad, cut, order = knn_graph(X, p.metric, mb, cands, threads)
            a, pm = prune(X, p.metric, mb, a, p.degree)
            # a row's list now also rests on its pruning comparisons
            order = np.minimum(np.minimum(order, cut), pm)
            cut = order.copy()
            ad = None
            if p.graph == 3:
                a, cut2, order2 = knn_sym(X, p.metric, mb, a, p.max_degree)
                cut, order = np.minimum(cut, cut2), np.minimum(order, order2)
        elif p.graph == 4:
            a, order = nsw_graph(X, p.metric, mb, p.degree, p.max_degree, p.ef_construction,
                                 p.insert_shift)
            ad, cut = None, order.copy()
        else:
            a, ad, cut, order = knn_graph(X, p.metric, mb, p.degree, threads)
        if p.graph == 1:
            a, cut, order = knn_sym(X, p.metric, mb, a, p.max_degree)
            ad = None
        idx.adj.append(a)
        idx.adj_dist.append(ad)
        idx.adj_margin.append(cut)
        idx.order_margin.append(order)
    if root_complete:
        # the root's decisions are the exhaustive scan's, not its list's
        idx.adj_margin[-1] = np.full(len(members[-1]), np.inf)
    return idx


def prune_candidates(degree: int) -> int:
    """Candidates scanned by the pruned graphs: the exact top min(2R, 32)."""
    return min(2 * degree, 32)


def prune(X, metric, members, adj_in, keep):
    """Diversity pruning of candidate lists (ho_prune): returns (adjacency
    [s, keep], smallest relative margin of each row's comparisons)."""
    lib = _load()
    s = len(members)
    adj_in = np.ascontiguousarray(adj_in, dtype=np.int32)
    out = np.full((s, keep), -1, dtype=np.int32)
    pm = np.full(s, np.inf)
    rc = lib.ho_prune(_ptr(X, ctypes.c_float), X.shape[1], metric,
                      _ptr(members, ctypes.c_int32), s, _ptr(adj_in, ctypes.c_int32),
                      adj_in.shape[1], keep, _ptr(out, ctypes.c_int32), _ptr(pm, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("prune failed")
    return out, pm


def nsw_batches(s: int, shift: int):
    """Insertion batches of the NSW graph: [lo, lo + max(1, lo >> shift)), from lo = 0."""
    lo = 0
    while lo < s:
        hi = min(s, lo + max(1, lo >> shift))
        yield lo, hi
        lo = hi


def nsw_insert(X, metric, members, adj, margin, lo, hi, R, ef):
    """One NSW insertion batch (ho_nsw_insert), in place on adj [s, M] and margin [s]."""
    lib = _load()
    assert adj.dtype == np.int32 and adj.flags.c_contiguous and margin.dtype == np.float64
    rc = lib.ho_nsw_insert(_ptr(X, ctypes.c_float), X.shape[1], metric,
                           _ptr(members, ctypes.c_int32), len(members),
                           _ptr(adj, ctypes.c_int32), adj.shape[1], lo, hi, R, ef,
                           _ptr(margin, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"nsw_insert failed ({rc})")


def nsw_graph(X, metric, members, R, M, ef, shift):
    """App. B.2's NSW graph of one layer: the members join in ascending id
    order, in the batches of :func:`nsw_batches`.  Returns (adjacency [s, M]
    local positions in (distance, id) order, -1 padded; min decision margin per row)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    members = np.ascontiguousarray(members, dtype=np.int32)
    s = len(members)
    adj = np.full((s, M), -1, dtype=np.int32)
    margin = np.full(s, np.inf)
    for lo, hi in nsw_batches(s, shift):
        nsw_insert(X, metric, members, adj, margin, lo, hi, R, ef)
    return adj, margin


def insert(idx: OracleIndex, X_new: np.ndarray, p: BuildParams) -> OracleIndex:
    """Insert(x) of the dynamic setting (App. C) for an index with NSW graphs.

    The new points get ids n, n+1, ...  Each layer is kept a random sample of
    the one below: a new member g of layer i-1 joins layer i when
    u(word g of stream (tag 5, layer i, attempt 0), 2^m) = 0 (probability
    2^-m).  New ids are the largest, so they extend every member list in order,
    and each layer graph takes its new members by NSW insertion, continuing the
    batch schedule of :func:`nsw_batches` from the layer's old size."""
    X_new = np.ascontiguousarray(X_new, dtype=np.float32)
    n_old = idx.X.shape[0]
    X = np.ascontiguousarray(np.concatenate([idx.X, X_new]), dtype=np.float32)
    new = np.arange(n_old, n_old + len(X_new), dtype=np.int32)
    out = OracleIndex(X=X, metric=idx.metric, degree=idx.degree,
                      root_complete=idx.root_complete, info=list(idx.info))
    for i in range(idx.num_layers):
        if i > 0:
            new = np.array([g for g in new.tolist()
                            if uniform_index(stream_word(p.seed, TAG_INSERT, i, 0, g),
                                             2 ** p.m) == 0], dtype=np.int32)
        old = idx.members[i]
        mb = np.concatenate([old, new]).astype(np.int32)
        M = idx.adj[i].shape[1]
        adj = np.full((len(mb), M), -1, dtype=np.int32)
        adj[:len(old)] = idx.adj[i]
        margin = np.full(len(mb), np.inf)
        margin[:len(old)] = idx.order_margin[i]
        lo = len(old)
        while lo < len(mb):
            hi = min(len(mb), lo + max(1, lo >> p.insert_shift))
            nsw_insert(X, idx.metric, mb, adj, margin, lo, hi, p.degree, p.ef_construction)
            lo = hi
        out.members.append(mb)
        out.adj.append(adj)
        out.adj_dist.append(None)
        out.adj_margin.append(margin.copy())
        out.order_margin.append(margin)
    if out.root_complete:
        out.adj_margin[-1] = np.full(len(out.members[-1]), np.inf)
    return out


def delete(idx: OracleIndex, ids, p: BuildParams) -> OracleIndex:
    """Delete(x) of the dynamic setting (App. C) for an index with NSW graphs.

    Every deleted point leaves every layer.  In each layer, the live rows that
    linked to deleted members are repaired (``ho_nsw_repair``), then the
    deleted members are dropped and positions renumbered in id order.  When a
    layer i >= 1 falls below half of ceil(|L_{i-1}| / 2^m), layers i and up are
    drawn again from L_{i-1} (Alg. 1's loop, same streams) and given new NSW
    graphs.  The rows of deleted points stay in X, unreachable."""
    lib = _load()
    X = idx.X
    D = np.unique(np.asarray(ids, dtype=np.int64))
    members, adjs, margins = [], [], []
    for i in range(idx.num_layers):
        mb = idx.members[i]
        pos = np.searchsorted(mb, D)
        pos = pos[(pos < len(mb)) & (mb[np.minimum(pos, len(mb) - 1)] == D)]
        adj = np.ascontiguousarray(idx.adj[i], dtype=np.int32).copy()
        margin = np.ascontiguousarray(idx.order_margin[i], dtype=np.float64).copy()
        if len(pos):
            dflag = np.zeros(len(mb), dtype=np.uint8)
            dflag[pos] = 1
            rc = lib.ho_nsw_repair(_ptr(X, ctypes.c_float), X.shape[1], idx.metric,
                                   _ptr(mb, ctypes.c_int32), len(mb), _ptr(adj, ctypes.c_int32),
                                   adj.shape[1], _ptr(dflag, ctypes.c_uint8),
                                   _ptr(margin, ctypes.c_double))
            if rc != 0:
                raise RuntimeError("nsw_repair failed")
            keep = dflag == 0
            newpos = np.cumsum(keep) - 1
            newpos[~keep] = -1
            adj = adj[keep]
            adj = np.where(adj >= 0, newpos[np.maximum(adj, 0)], -1).astype(np.int32)
            mb, margin = mb[keep], margin[keep]
        members.append(mb.astype(np.int32))
        adjs.append(adj)
        margins.append(margin)
    infos = [copy.copy(x) for x in idx.info]
    for i in range(1, len(members)):
        if 2 * len(members[i]) < -(-len(members[i - 1]) // 2 ** p.m):
            del members[i:], adjs[i:], margins[i:], infos[i:]
            _extend_layers(X, members, infos, p)
            for mb in members[i:]:
                a, mg = nsw_graph(X, idx.metric, mb, p.degree, p.max_degree, p.ef_construction,
                                  p.insert_shift)
                adjs.append(a)
                margins.append(mg)
            break
    for i, mb in enumerate(members):
        infos[i].size = len(mb)
    root_complete = p.root_complete_max > 0 and len(members) >= 2
    out = OracleIndex(X=X, metric=idx.metric, degree=idx.degree, root_complete=root_complete,
                      members=members, adj=adjs, adj_dist=[None] * len(members),
                      adj_margin=[m.copy() for m in margins], order_margin=margins, info=infos)
    if root_complete:
        out.adj_margin[-1] = np.full(len(members[-1]), np.inf)
    return out


def knn_sym(X, metric, members, adj_knn, max_deg):
    """kNN plus reverse edges: first max_deg of the deduplicated union of
    out- and in-neighbours in (distance, id) order (cut / order margins)."""
    lib = _load()
    s = len(members)
    adj_knn = np.ascontiguousarray(adj_knn, dtype=np.int32)
    out = np.full((s, max_deg), -1, dtype=np.int32)
    cut = np.full(s, np.inf)
    order = np.full(s, np.inf)
    rc = lib.ho_knn_sym(_ptr(X, ctypes.c_float), X.shape[1], metric,
                        _ptr(members, ctypes.c_int32), s, _ptr(adj_knn, ctypes.c_int32),
                        adj_knn.shape[1], max_deg, _ptr(out, ctypes.c_int32),
                        _ptr(cut, ctypes.c_double), _ptr(order, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("knn_sym failed")
    return out, cut, order


def index_from_arrays(X, metric, members, adj, degree=None, root_complete=False) -> OracleIndex:
    """Wrap an index given as data (e.g. exported by another builder)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    members = [np.ascontiguousarray(m, dtype=np.int32) for m in members]
    adj = [np.ascontiguousarray(a, dtype=np.int32) for a in adj]
    deg = degree if degree is not None else adj[0].shape[1]
    return OracleIndex(X=X, metric=metric, degree=deg, members=members, adj=adj,
                       root_complete=bool(root_complete) and len(members) >= 2)


@dataclass
class SearchResult:
    ids: np.ndarray          # int32 [nq, k]
    dist: np.ndarray         # float64 [nq, k]
    margin: np.ndarray       # float64 [nq] min decision margin over the trace
    adj_margin: np.ndarray   # float64 [nq] min adjacency margin of expanded nodes
    counters: np.ndarray     # int64 [nq, 4]: expansions, evals (all layers), (layer 0)


def search(idx: OracleIndex, Q: np.ndarray, k: int, ef: int, ef_upper: int = 1,
           threads=None, q_range=None) -> SearchResult:
    """Alg. 4 Query with the Sec. 2.2 candidate set; see module docstring."""
    lib = _load()
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    X = idx.X
    nq = Q.shape[0]
    L = idx.num_layers
    sizes = np.array([len(m) for m in idx.members], dtype=np.int64)
    degs = np.array([a.shape[1] for a in idx.adj], dtype=np.int32)
    P32 = ctypes.POINTER(ctypes.c_int32)
    PF64 = ctypes.POINTER(ctypes.c_double)
    mem_arr = (P32 * L)(*[_ptr(m, ctypes.c_int32) for m in idx.members])
    adj_arr = (P32 * L)(*[_ptr(a, ctypes.c_int32) for a in idx.adj])
    if idx.adj_margin:
        am_arr = (PF64 * L)(*[_ptr(a, ctypes.c_double) for a in idx.adj_margin])
    else:
        am_arr = None
    ids = np.full((nq, k), -1, dtype=np.int32)
    dist = np.full((nq, k), np.inf)
    margin = np.full(nq, np.inf)
    amargin = np.full(nq, np.inf)
    counters = np.zeros((nq, 4), dtype=np.int64)
    b0, e0 = (0, nq) if q_range is None else q_range

    def one(b, e):
        rc = lib.ho_search(_ptr(X, ctypes.c_float), X.shape[1], idx.metric, L,
                           _ptr(sizes, ctypes.c_int64), mem_arr, adj_arr,
                           _ptr(degs, ctypes.c_int32), am_arr, _ptr(Q, ctypes.c_float),
                           b0 + b, b0 + e, k, ef, ef_upper, int(idx.root_complete),
                           _ptr(ids, ctypes.c_int32),
                           _ptr(dist, ctypes.c_double), _ptr(margin, ctypes.c_double),
                           _ptr(amargin, ctypes.c_double), _ptr(counters, ctypes.c_int64))
        if rc != 0:
            raise RuntimeError(f"search failed ({rc})")
    _parallel(e0 - b0, one, threads, min_chunk=4)
    return SearchResult(ids, dist, margin, amargin, counters)


def brute_force_knn(X: np.ndarray, Q: np.ndarray, k: int, metric: int = L2, threads=None):
    """Exact k-NN by FP64 brute force, ties by id (Sec. 2 problem setting)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    nq = Q.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int32)
    dist = np.full((nq, k), np.inf)

    def one(b, e):
        rc = lib.ho_brute_knn(_ptr(X, ctypes.c_float), X.shape[0], X.shape[1], metric,
                              _ptr(Q, ctypes.c_float), b, e, k, _ptr(ids, ctypes.c_int32),
                              _ptr(dist, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("brute_knn failed")
    _parallel(nq, one, threads)
    return ids, dist


def _seq_dist(Xc: np.ndarray, q: np.ndarray, metric: int) -> np.ndarray:
    """FP64 distances of rows Xc [m, d] to q, each summed in coordinate order
    (the same sums as the C oracle's, vectorised over the rows)."""
    Xc = Xc.astype(np.float64)
    q = q.astype(np.float64)
    acc = np.zeros(Xc.shape[0])
    for j in range(Xc.shape[1]):
        if metric == L2:
            t = Xc[:, j] - q[j]
            acc += t * t
        else:
            acc += Xc[:, j] * q[j]
    return acc if metric == L2 else -acc


def brute_force_knn_gram(X: np.ndarray, Q: np.ndarray, k: int, metric: int = L2,
                         threads=None, chunk: int = 256):
    """Exact k-NN (Sec. 2 problem setting) for large inputs, through an FP64
    matrix product as a step (the same result as :func:`brute_force_knn`):

    1. g(x) = |x|^2 - 2 <q, x> (L2; the squared distance minus |q|^2) or
       -<q, x> (IP) for every point, by one FP64 matrix product per block of
       queries (torch on the CPU);
    2. the m = 2k + 8 points of smallest g per query (torch.topk);
    3. their exact FP64 distances (:func:`_seq_dist`, coordinate order), sorted
       by (distance, id); the first k are the answer
    4. provided the shortlist provably holds them: every point left out has
       g >= the m-th g, and |g + |q|^2 - dist| <= delta with
       delta = 2 (d + 2) 2^-53 (|q| + max|x|)^2 (the rounding of the dot
       product and of the norms), so when the exact k-th distance is below
       (m-th g) + |q|^2 - 2 delta no left-out point can enter the top k.
       Queries that fail the test are answered by :func:`brute_force_knn`.
    Returns (ids int32 [nq, k], FP64 distances [nq, k])."""
    import torch
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    n, d = X.shape
    nq = Q.shape[0]
    m = min(n, 2 * k + 8)
    old = torch.get_num_threads()
    torch.set_num_threads(threads or default_threads())
    try:
        Xt = torch.from_numpy(X).to(torch.float64)
        xn = (Xt * Xt).sum(1)
        xmax = float(xn.max().sqrt())
        ids = np.full((nq, k), -1, dtype=np.int32)
        dist = np.full((nq, k), np.inf)
        redo = []
        for b in range(0, nq, chunk):
            Qc = torch.from_numpy(Q[b:b + chunk]).to(torch.float64)
            if metric == L2:
                g = torch.addmm(xn.unsqueeze(0).expand(Qc.shape[0], -1), Qc, Xt.T, alpha=-2.0)
            else:
                g = -(Qc @ Xt.T)
            gv, gi = torch.topk(g, m, dim=1, largest=False, sorted=True)
            gv, gi = gv.numpy(), gi.numpy()
            del g
            for r in range(Qc.shape[0]):
                qi = b + r
                cand = gi[r]
                dd = _seq_dist(X[cand], Q[qi], metric)
                order = np.lexsort((cand, dd))[:k]
                ids[qi, :len(order)] = cand[order]
                dist[qi, :len(order)] = dd[order]
                if m < n:
                    qn = float(np.linalg.norm(Q[qi].astype(np.float64)))
                    delta = 2.0 * (d + 2) * 2.0 ** -53 * (qn + xmax) ** 2
                    bound = gv[r, m - 1] + (qn * qn if metric == L2 else 0.0) - 2 * delta
                    if not dist[qi, k - 1] < bound:
                        redo.append(qi)
        if redo:
            ri, rd = brute_force_knn(X, Q[redo], k, metric, threads)
            ids[redo], dist[redo] = ri, rd
    finally:
        torch.set_num_threads(old)
    return ids, dist


def distance(a: np.ndarray, b: np.ndarray, metric: int = L2) -> float:
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return float(_load().ho_distance(_ptr(a, ctypes.c_float), _ptr(b, ctypes.c_float),
                                     a.shape[0], metric))


def recall_at_k(found_ids: np.ndarray, true_dist: np.ndarray, X: np.ndarray, Q: np.ndarray,
                metric: int = L2) -> float:
    """Tie-tolerant Recall@k (Sec. 2): a returned id counts when its exact FP64
    distance is at most the true k-th distance."""
    nq, k = found_ids.shape
    hits = 0
    for i in range(nq):
        kth = true_dist[i, k - 1]
        for j in range(k):
            u = int(found_ids[i, j])
            if u < 0:
                continue
            if distance(Q[i], X[u], metric) <= kth:
                hits += 1
    return hits / float(nq * k)


def near_tie(res: SearchResult, tol: float = 1e-5) -> np.ndarray:
    """Queries whose trace holds a decision with relative margin <= tol, or
    that expanded a node whose R-th / (R+1)-th neighbour are that close (a
    near tie inside a list cannot matter: the order of neighbours within one
    expansion does not change the result)."""
    return (res.margin <= tol) | (res.adj_margin <= tol)

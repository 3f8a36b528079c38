"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

The plain FP32 path must return the oracle's ids bit-exactly, position by
position, for every query whose oracle trace holds no decision within the
FP32 error bound (exempt_tol(d), below the specification's 1e-5), with
distances within 1e-5 relative.  Each test caps the exempt fraction near 1.5x
the oracle's own rate on its inputs (printed).  Sizes span
several tiles / waves and ragged tails; edge cases cover tiny and padded
inputs.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import (assert_results_valid, assert_search_parity, exempt_mask, exempt_tol,
                      to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hn():
    import paper_2505_17368_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def ho():
    from oracle import henn_oracle
    return henn_oracle


@pytest.fixture(scope="module")
def cfg1(ho):
    """The parity workload: 10,000 x 32 uniform points, 1,000 queries."""
    X, Q = wl.make("uniform_10k_d32")
    oidx = ho.build_index(X, ho.BuildParams(degree=16))
    return X, Q, oidx


def _sync():
    import torch
    torch.cuda.synchronize()


def _import(hn, X, oidx, **kw):
    if oidx.root_complete:
        kw.setdefault("root_complete_max", len(oidx.members[-1]))
    return hn.henn_import(to_dev(X), oidx.members, oidx.adj, degree=oidx.degree,
                          metric=oidx.metric, **kw)


def test_search_parity_on_oracle_index_cfg1(hn, ho, cfg1):
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32)
    _sync()
    ores = ho.search(oidx, Q, 10, 32)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, max_exempt=0.041)
    assert_results_valid(gi.cpu().numpy()[:100], gd.cpu().numpy()[:100], X, Q[:100])
    idx.free()


# caps: 1.5x the oracle's exempt rate on these 300 queries (0, 0, 10.7%, 43.3%,
# 2.0%, 11.7%), at least 1%
@pytest.mark.parametrize("k,ef,ef_upper,cap", [(1, 1, 1, 0.01), (10, 10, 1, 0.01),
                                               (10, 64, 1, 0.161), (5, 200, 1, 0.65),
                                               (10, 32, 4, 0.03), (64, 64, 1, 0.176)])
def test_search_parity_beam_widths(hn, ho, cfg1, k, ef, ef_upper, cap):
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    Qs = Q[:300]
    gi, gd = hn.henn_search_batch(idx, to_dev(Qs), k=k, ef=ef, ef_upper=ef_upper)
    _sync()
    ores = ho.search(oidx, Qs, k, ef, ef_upper)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Qs, max_exempt=cap)
    idx.free()


# caps: 1.5x the oracle's exempt rate (1.6%, 3.9%, 6.2%, 8.6% of 257 queries)
@pytest.mark.parametrize("metric,d,cap", [(0, 20, 0.024), (1, 24, 0.059), (0, 100, 0.094),
                                          (1, 128, 0.129)])
def test_search_parity_metrics_and_ragged_dims(hn, ho, metric, d, cap):
    X = wl.uniform(3001, d, 21) - 0.5
    Q = wl.uniform(257, d, 22) - 0.5
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    oidx = ho.build_index(X, ho.BuildParams(degree=12, metric=metric))
    idx = _import(hn, X, oidx)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=7, ef=40)
    _sync()
    ores = ho.search(oidx, Q, 7, 40)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, metric=metric,
                         max_exempt=cap)
    idx.free()


def test_launch_shapes_give_identical_results(hn, cfg1):
    """Canonical reduction: any lanes-per-vector / waves-per-block / persistent
    launch returns bit-identical ids and distances."""
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    Qd = to_dev(Q)
    ref_i, ref_d = hn.henn_search_batch(idx, Qd, k=10, ef=48)
    _sync()
    ref_i, ref_d = ref_i.cpu().numpy(), ref_d.cpu().numpy()
    for lpn in (2, 4):  # both lane shapes that exist for d = 32
        for wpb in (1, 2, 4, 8):
            for pers in (False, True):
                gi, gd = hn.henn_search_batch(idx, Qd, k=10, ef=48, lanes_per_vec=lpn,
                                              waves_per_block=wpb, persistent=pers)
                _sync()
                assert np.array_equal(gi.cpu().numpy(), ref_i), (lpn, wpb, pers)
                assert np.array_equal(gd.cpu().numpy().view(np.uint32),
                                      ref_d.view(np.uint32)), (lpn, wpb, pers)
    idx.free()


def test_concurrent_persistent_searches_on_two_streams(hn, cfg1):
    """Persistent searches each take their own work counter: one large search
    on one stream while 80 small ones run on another (more than any shared
    pool of counters would hold) all equal the same searches run alone."""
    import torch
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    Qd = to_dev(Q)
    big_ref = hn.henn_search_batch(idx, Qd, k=10, ef=64, persistent=True)
    small_ref = [hn.henn_search_batch(idx, Qd[j * 8:(j + 1) * 8], k=10, ef=32, persistent=True)
                 for j in range(80)]
    _sync()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        big = hn.henn_search_batch(idx, Qd, k=10, ef=64, persistent=True, stream=sa)
    with torch.cuda.stream(sb):
        small = [hn.henn_search_batch(idx, Qd[j * 8:(j + 1) * 8], k=10, ef=32, persistent=True,
                                      stream=sb) for j in range(80)]
    torch.cuda.synchronize()
    assert torch.equal(big[0], big_ref[0]) and torch.equal(big[1], big_ref[1])
    for j in range(80):
        assert torch.equal(small[j][0], small_ref[j][0]), j
        assert torch.equal(small[j][1], small_ref[j][1]), j
    idx.free()


def test_query_alone_equals_query_in_batch(hn, cfg1):
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    full_i, full_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32)
    _sync()
    for qi in (0, 17, 999):
        one_i, one_d = hn.henn_search_batch(idx, to_dev(Q[qi:qi + 1]), k=10, ef=32)
        _sync()
        assert np.array_equal(one_i.cpu().numpy()[0], full_i.cpu().numpy()[qi])
        assert np.array_equal(one_d.cpu().numpy()[0], full_d.cpu().numpy()[qi])
    idx.free()


def test_mixed_k_ef_per_query_matches_uniform_calls(hn, ho, cfg1):
    import torch
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    Qs = Q[:240]
    ks = np.array([1, 10, 5, 3] * 60, dtype=np.int32)
    efs = np.array([8, 32, 16, 64, 12, 40] * 40, dtype=np.int32)
    gi, gd = hn.henn_search_batch(idx, to_dev(Qs), k_arr=to_dev(ks), ef_arr=to_dev(efs),
                                  k_max=10, ef_max=64)
    _sync()
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    exempt = 0
    for kk, ee in {(int(a), int(b)) for a, b in zip(ks, efs)}:
        sel = np.where((ks == kk) & (efs == ee))[0]
        ores = ho.search(oidx, Qs[sel], kk, ee)
        exempt += int(assert_search_parity(gi[sel, :kk], gd[sel, :kk], ores, X, Qs[sel]).sum())
        assert (gi[sel, kk:] == -1).all() and np.isinf(gd[sel, kk:]).all()
    # the oracle exempts 2 of these 240 queries
    print(f"exempt {exempt} of 240")
    assert exempt <= 3
    del torch
    idx.free()


def test_counters_match_oracle_on_exact_queries(hn, ho, cfg1):
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx)
    gi, gd, cnt = hn.henn_search_batch(idx, to_dev(Q[:200]), k=10, ef=32, with_counters=True)
    _sync()
    ores = ho.search(oidx, Q[:200], 10, 32)
    ok = ~exempt_mask(ores, X.shape[1])
    c = cnt.cpu().numpy()
    # expansions are exactly the oracle's; evaluations never fewer (the
    # visited table may forget) and equal when nothing was forgotten
    assert np.array_equal(c[ok, 0], ores.counters[ok, 0])
    assert np.array_equal(c[ok, 2], ores.counters[ok, 2])
    assert (c[ok, 1] >= ores.counters[ok, 1]).all()
    idx.free()


@pytest.mark.parametrize("storage,persistent", [(0, False), (2, True)])
def test_exact_visited_counts_equal_oracle_and_keeps_results(hn, ho, cfg1, storage, persistent):
    """With the exact visited set every node is evaluated once per layer, as
    the method does: all four counters equal the oracle's on the queries whose
    traversal decisions are not near ties, and the results are those of the
    default table bit for bit."""
    X, Q, oidx = cfg1
    idx = _import(hn, X, oidx, storage=storage)
    Qd = to_dev(Q[:300])
    ei, ed, ec = hn.henn_search_batch(idx, Qd, k=10, ef=32, with_counters=True,
                                      exact_visited=True, persistent=persistent)
    di, dd, dc = hn.henn_search_batch(idx, Qd, k=10, ef=32, with_counters=True,
                                      persistent=persistent)
    _sync()
    assert np.array_equal(ei.cpu().numpy(), di.cpu().numpy())
    assert np.array_equal(ed.cpu().numpy().view(np.uint32), dd.cpu().numpy().view(np.uint32))
    ec, dc = ec.cpu().numpy(), dc.cpu().numpy()
    assert (dc[:, 1] >= ec[:, 1]).all() and np.array_equal(dc[:, 0], ec[:, 0])
    if storage == 0:
        ores = ho.search(oidx, Q[:300], 10, 32)
        ok = ~exempt_mask(ores, X.shape[1])
        print(f"exact-visited counters compared on {ok.sum()} of {len(ok)} queries; "
              f"the table re-evaluated {int((dc[:, 1] - ec[:, 1]).sum())} rows")
        assert ok.sum() >= 250
        assert np.array_equal(ec[ok], ores.counters[ok])
    idx.free()


def test_edge_cases(hn, ho):
    # one point; fewer points than k; empty batch
    X = wl.uniform(5, 8, 30)
    Q = wl.uniform(3, 8, 31)
    oidx = ho.build_index(X, ho.BuildParams(degree=4))
    idx = _import(hn, X, oidx)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=8, ef=8)
    _sync()
    ores = ho.search(oidx, Q, 8, 8)
    assert np.array_equal(gi.cpu().numpy(), ores.ids)
    assert (gi.cpu().numpy()[:, 5:] == -1).all() and np.isinf(gd.cpu().numpy()[:, 5:]).all()
    empty = to_dev(np.zeros((0, 8), np.float32))
    ei, ed = hn.henn_search_batch(idx, empty, k=3, ef=3)
    assert ei.shape == (0, 3)
    idx.free()
    X1 = wl.uniform(1, 3, 1)
    idx1 = hn.henn_build(to_dev(X1))
    gi, gd = hn.henn_search_batch(idx1, to_dev(X1), k=2, ef=2)
    _sync()
    assert gi.cpu().numpy().tolist() == [[0, -1]] and gd.cpu().numpy()[0, 0] == 0.0
    idx1.free()


# ----------------------------------------------------------- GPU build ----

def _gpu_layers(idx):
    return [idx.export_layer(i) for i in range(idx.num_layers)]


def test_build_layers_match_oracle_cfg1(hn, ho, cfg1):
    X, Q, oidx = cfg1
    idx = hn.henn_build(to_dev(X), degree=16)
    layers = _gpu_layers(idx)
    assert len(layers) == oidx.num_layers
    for i, (ids, _) in enumerate(layers):
        assert np.array_equal(ids, oidx.members[i]), f"layer {i}"
        gi = idx.layer_info(i)
        oi = oidx.info[i]
        if i > 0:
            assert gi["status"] == oi.status and gi["attempts"] == oi.attempts
            assert gi["window"] == oi.window and gi["draws"] == oi.draws
            assert gi["eps"] == pytest.approx(oi.eps, rel=1e-15)
    idx.free()


@pytest.mark.parametrize("seed,eps", [(3, 0.031), (7, 0.02), (11, 0.05)])
def test_build_las_vegas_repeats_match_oracle(hn, ho, seed, eps):
    X = wl.uniform(4000, 6, seed)
    p = dict(degree=8, seed=seed, eps_override=eps, max_layers=2)
    olayers, oinfo = ho.build_layers(X, ho.BuildParams(**p))
    idx = hn.henn_build(to_dev(X), **p)
    layers = _gpu_layers(idx)
    assert len(layers) == len(olayers)
    for i in range(1, len(olayers)):
        gi = idx.layer_info(i)
        assert (gi["status"], gi["attempts"], gi["hits"]) == (
            oinfo[i].status, oinfo[i].attempts, oinfo[i].hits), f"layer {i}"
        assert np.array_equal(layers[i][0], olayers[i])
    idx.free()


@pytest.mark.parametrize("n,d,seed,eps,attempts", [
    (4000, 6, 3, 0.015, 64),       # Las-Vegas repeats (layer 1 kept at attempt 6)
    (4000, 6, 7, 0.006, 4),        # attempt cap: best attempt kept
    (10_000, 32, 5, 0.0, 64),      # Eq. (1) schedule (vacuous layers)
    (1_000_003, 4, 9, 2.0, 1),     # one large odd layer, no ring check
])
def test_halving_layers_match_oracle(hn, ho, n, d, seed, eps, attempts):
    """Alg. 3's halving sampler: member lists bit-exact, same Las-Vegas outcome."""
    X = wl.uniform(n, d, seed)
    p = dict(degree=8, seed=seed, eps_override=eps, max_attempts=attempts, sampler=1,
             max_layers=1 if n > 100_000 else -1)
    olayers, oinfo = ho.build_layers(X, ho.BuildParams(**p))
    idx = hn.henn_build(to_dev(X), **p)
    layers = _gpu_layers(idx)
    assert len(layers) == len(olayers)
    for i in range(1, len(olayers)):
        gi = idx.layer_info(i)
        assert (gi["status"], gi["attempts"], gi["hits"]) == (
            oinfo[i].status, oinfo[i].attempts, oinfo[i].hits), f"layer {i}"
        assert len(layers[i][0]) == -(-len(olayers[i - 1]) // 16)
        assert np.array_equal(layers[i][0], olayers[i]), f"layer {i}"
    idx.free()


def _ring_outcomes(ho, X, prev, layer, p, window, attempts, d):
    """Per attempt and ring: 1 when the sample certainly hits the ring under
    any FP32 ordering of the distances, 0 when it certainly misses, -1 when a
    sample point near a window end leaves it open.  A point's rank among the
    ring centre's distances is bounded by the points certainly below it (FP64
    distance below its own by more than both FP32 errors) and those possibly
    below it."""
    s = len(prev)
    Xl = X[prev].astype(np.float64)
    E = exempt_tol(d) / 2.0                       # one distance's relative error, with allowance
    lo_f, hi_f = (1 - E) / (1 + E), (1 + E) / (1 - E)
    D = -(-s // 2 ** p.m)
    cen = ho.draw_indices(p.seed, ho.TAG_RING_CENTRE, layer, 0, s, p.num_rings)
    st = ho.draw_indices(p.seed, ho.TAG_RING_START, layer, 0, s - window + 1, p.num_rings)
    samples = [np.unique(ho.draw_indices(p.seed, ho.TAG_SAMPLE, layer, t, s, D))
               for t in range(attempts)]
    out = np.zeros((attempts, p.num_rings), np.int8)
    for j in range(p.num_rings):
        dd = ((Xl - Xl[cen[j]]) ** 2).sum(1)
        srt = np.sort(dd)
        a = int(st[j])
        for t, S in enumerate(samples):
            certainly_below = np.searchsorted(srt, dd[S] * lo_f, side="left")
            possibly_below = np.searchsorted(srt, dd[S] * hi_f, side="right") - 1
            inside = (certainly_below >= a) & (possibly_below <= a + window - 1)
            outside = (possibly_below < a) | (certainly_below > a + window - 1)
            out[t, j] = 1 if inside.any() else (0 if outside.all() else -1)
    return out


@pytest.mark.parametrize("seed,status,attempts,cap", [(4, "verified", 3, dict(max_attempts=3)),
                                                       (6, "not_verified", 3, dict(max_attempts=3)),
                                                       (6, "not_verified", 3,
                                                        dict(max_attempts=0, phi=5e-4))])
def test_ring_check_at_400k_points_matches_oracle(hn, ho, seed, status, attempts, cap):
    """Layer 1 of 400,000 points: the ring check ranks 400,000 keys per ring
    (the radix histogram's grid-stride loop runs more than once) with windows
    of 49 points, so samples are redrawn (Alg. 2's repeat) or the attempt cap
    keeps the best one.  Every attempt's outcome on every ring is first shown
    to be independent of FP32 rounding at the window ends; then the GPU's
    status, attempts, hits and member list equal the oracle's."""
    n, d = 400_000, 8
    X = wl.uniform(n, d, 90)
    kw = dict(degree=8, seed=seed, eps_override=1.2e-4, max_layers=1, **cap)
    p = ho.BuildParams(**kw)
    olayers, oinfo = ho.build_layers(X, p)
    info = oinfo[1]
    assert (info.status, info.attempts) == (status, attempts)
    rings = _ring_outcomes(ho, X, olayers[0], 1, p, info.window, info.attempts, d)
    print(f"ring outcomes open to rounding: {int((rings < 0).sum())}; window margin "
          f"{info.ring_margin:.3g}; hits per attempt {(rings == 1).sum(1).tolist()}")
    assert (rings >= 0).all()
    idx = hn.henn_build(to_dev(X), **kw)
    gi = idx.layer_info(1)
    assert (gi["status"], gi["attempts"], gi["hits"], gi["window"]) == (
        info.status, info.attempts, info.hits, info.window)
    assert np.array_equal(idx.export_layer(1)[0], olayers[1])
    idx.free()


def test_build_graph_matches_oracle(hn, ho, cfg1):
    X, Q, oidx = cfg1
    idx = hn.henn_build(to_dev(X), degree=16)
    for i, (ids, adj) in enumerate(_gpu_layers(idx)):
        oadj = oidx.adj[i]
        same = (adj == oadj).all(1)
        tie = oidx.order_margin[i] <= exempt_tol(X.shape[1])
        assert (same | tie).all(), f"layer {i}: {np.where(~same & ~tie)[0][:5]}"
        # near-tie rows still hold the same neighbour set unless the R / R+1 cut is tied
        cut_tie = oidx.adj_margin[i] <= exempt_tol(X.shape[1])
        for r in np.where(~same & ~cut_tie)[0]:
            assert set(adj[r].tolist()) == set(oadj[r].tolist())
    idx.free()


def test_end_to_end_cfg1(hn, ho, cfg1):
    X, Q, oidx = cfg1
    idx = hn.henn_build(to_dev(X), degree=16)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32)
    _sync()
    ores = ho.search(oidx, Q, 10, 32)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, max_exempt=0.041,
                         graph_margins=True)
    idx.free()


@pytest.mark.parametrize("n,d,metric", [(20000, 128, 0), (6000, 96, 0), (5000, 64, 1),
                                         (5000, 200, 0), (4000, 768, 1), (3000, 136, 1)])
def test_build_graph_matches_oracle_rows_larger(hn, ho, n, d, metric):
    """Several MFMA row blocks and a ragged tail: sampled layer-0 rows against
    the oracle's exact kNN rows (order may differ only at near ties)."""
    X = wl.gauss_mix(n, d, 20, 0.3, 40)
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    idx = hn.henn_build(to_dev(X), degree=16, metric=metric, max_layers=0)
    _, adj = idx.export_layer(0)
    rows = np.sort(np.random.default_rng(0).choice(n, 200, replace=False))
    rows = np.concatenate([rows, [n - 1]])
    oadj, cut, order = ho.knn_rows(X, metric, np.arange(n, dtype=np.int32), rows, 16)
    for j, r in enumerate(rows):
        if np.array_equal(adj[r], oadj[j]):
            continue
        assert order[j] <= exempt_tol(d), f"row {r}: {adj[r]} vs {oadj[j]}"
        if cut[j] > exempt_tol(d):
            assert set(adj[r].tolist()) == set(oadj[j].tolist())
    info = idx.layer_info(0)
    print(f"fallback rows {info['fallback_rows']}")
    idx.free()


@pytest.mark.parametrize("kind,n,d,metric", [
    ("gauss", 20000, 128, 0), ("gauss", 6000, 96, 0), ("gauss", 5000, 64, 1),
    ("gauss", 3000, 36, 0), ("gauss", 2500, 8, 0), ("spectral", 4000, 120, 1),
    ("curve", 8000, 96, 0), ("expskew", 6000, 32, 0)])
def test_split_bf16_and_fp32_gram_give_the_same_graph(hn, ho, kind, n, d, metric):
    """The kNN graph from split-BF16 Gram tiles (the default) and from FP32
    tiles: both shortlists are proven (or re-solved exactly) against the
    canonical distance, so the graphs are identical, row for row, including
    inputs with many near ties (the curve) where rows fall back."""
    if kind == "gauss":
        X = wl.gauss_mix(n, d, 20, 0.3, 40)
        if metric == 1:
            X /= np.linalg.norm(X, axis=1, keepdims=True)
    elif kind == "spectral":
        X = wl.spectral(n, d, 41)
    elif kind == "curve":
        X = wl.curve(n, d, 42)
    else:
        X = wl.expskew(n, d, 32.0, seed=43)
    Xd = to_dev(X)
    out = []
    for gram in (0, 1):
        idx = hn.henn_build(Xd, degree=16, metric=metric, max_layers=0, gram=gram)
        out.append((idx.export_layer(0)[1], idx.layer_info(0)["fallback_rows"]))
        idx.free()
    print(f"{kind} {n} x {d}: fallback rows split {out[0][1]}, fp32 {out[1][1]}")
    assert np.array_equal(out[0][0], out[1][0])
    # and both are the exact kNN rows (sampled rows against the oracle)
    adj = out[0][0]
    rows = np.sort(np.random.default_rng(1).choice(n, 100, replace=False))
    oadj, cut, order = ho.knn_rows(X, metric, np.arange(n, dtype=np.int32), rows, 16)
    for j, r in enumerate(rows):
        if np.array_equal(adj[r], oadj[j]):
            continue
        assert order[j] <= exempt_tol(d), f"row {r}: {adj[r]} vs {oadj[j]}"
        if cut[j] > exempt_tol(d):
            assert set(adj[r].tolist()) == set(oadj[j].tolist())


@pytest.mark.parametrize("n,d,metric", [(17, 64, 0), (33, 128, 0), (95, 40, 1), (130, 8, 0)])
def test_split_gram_on_layers_of_one_or_a_few_tiles(hn, ho, n, d, metric):
    """Layers of one partial tile up to a few tiles (the split-BF16 kernel
    pads its rows and tile norms to whole 32-row tiles): the graph equals
    the FP32 tiles' and the oracle's exact kNN rows."""
    X = wl.gauss_mix(n, d, 4, 0.3, 44)
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    Xd = to_dev(X)
    out = []
    for gram in (0, 1):
        idx = hn.henn_build(Xd, degree=16, metric=metric, max_layers=0, gram=gram)
        out.append(idx.export_layer(0)[1])
        idx.free()
    assert np.array_equal(out[0], out[1])
    rows = np.arange(n, dtype=np.int64)
    oadj, cut, order = ho.knn_rows(X, metric, np.arange(n, dtype=np.int32), rows, 16)
    for r in range(n):
        if not np.array_equal(out[0][r], oadj[r]):
            assert order[r] <= exempt_tol(d), f"row {r}: {out[0][r]} vs {oadj[r]}"
            if cut[r] > exempt_tol(d):
                assert set(out[0][r].tolist()) == set(oadj[r].tolist())


@pytest.mark.parametrize("d,metric", [(200, 0), (768, 1)])
def test_wide_rows_end_to_end(hn, ho, d, metric):
    """Rows wider than 128 coordinates (K-sliced Gram build, 16-lane gathers):
    the GPU hierarchy searched by the oracle and by the kernel agree."""
    if metric == 0:
        X = wl.gauss_mix(3000, d, 10, 0.3, 41)
        Q = wl.gauss_mix(200, d, 10, 0.3, 42)
    else:
        # unit vectors with a power-law spectrum (the retrieval workload's
        # distribution); normalised tight clusters would put most traces
        # through a near tie of the inner products
        X = wl.spectral(3000, d, 41)
        Q = wl.spectral(200, d, 42)
    idx = hn.henn_build(to_dev(X), degree=16, metric=metric)
    layers = _gpu_layers(idx)
    oidx = ho.index_from_arrays(X, metric, [l[0] for l in layers], [l[1] for l in layers])
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=48)
    _sync()
    ores = ho.search(oidx, Q, 10, 48)
    # the oracle exempts 14.5% (d = 200) / 13.5% (d = 768) of these 200 queries
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, metric=metric,
                         max_exempt=0.22 if d == 200 else 0.21)
    idx.free()


# ------------------------------------------- complete root, kNN_SYM ------

@pytest.fixture(scope="module")
def cfg1_sym_root(ho):
    X, Q = wl.make("uniform_10k_d32")
    p = ho.BuildParams(degree=16, graph=1, max_degree=32, root_complete_max=1000)
    return X, Q, ho.build_index(X, p)


def test_search_parity_complete_root_and_sym_graph(hn, ho, cfg1_sym_root):
    X, Q, oidx = cfg1_sym_root
    assert oidx.root_complete and oidx.num_layers == 2
    idx = _import(hn, X, oidx)
    gi, gd, cnt = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32, with_counters=True)
    _sync()
    ores = ho.search(oidx, Q, 10, 32)
    ex = assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, max_exempt=0.051)
    c = cnt.cpu().numpy()
    ok = ~ex
    assert np.array_equal(c[ok, 0], ores.counters[ok, 0])
    assert (c[ok, 1] >= ores.counters[ok, 1]).all()
    idx.free()


@pytest.mark.parametrize("storage", [1, 2])
def test_complete_root_precision_forms_run(hn, ho, cfg1_sym_root, storage):
    X, Q, oidx = cfg1_sym_root
    idx = _import(hn, X, oidx, storage=storage)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q[:200]), k=10, ef=64)
    _sync()
    assert_results_valid(gi.cpu().numpy(), gd.cpu().numpy(), X, Q[:200])
    idx.free()


def test_build_sym_graph_matches_oracle(hn, ho, cfg1_sym_root):
    X, Q, oidx = cfg1_sym_root
    idx = hn.henn_build(to_dev(X), degree=16, graph=1, max_degree=32, root_complete_max=1000)
    assert idx.num_layers == oidx.num_layers
    for i in range(idx.num_layers):
        ids, adj = idx.export_layer(i)
        assert np.array_equal(ids, oidx.members[i])
        same = (adj == oidx.adj[i]).all(1)
        tie = oidx.order_margin[i] <= exempt_tol(X.shape[1])
        # a row may also move when a kNN row feeding it has a near tie at its cut
        kadj, _, kcut, _ = ho.knn_graph(X, 0, oidx.members[i], 16)
        knn_tie_rows = np.where(kcut <= exempt_tol(X.shape[1]))[0]
        touched = set(knn_tie_rows.tolist())
        for r in knn_tie_rows:
            touched |= set(kadj[r].tolist())
        bad = [r for r in np.where(~same & ~tie)[0] if r not in touched]
        assert not bad, f"layer {i}: rows {bad[:5]}"
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32)
    _sync()
    ores = ho.search(oidx, Q, 10, 32)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, max_exempt=0.051,
                         graph_margins=True)
    idx.free()


@pytest.mark.parametrize("metric", [0, 1])
def test_fp8_rows_of_exact_codes_traverse_like_fp32(hn, metric):
    """Rows of integers in [-7, 7] with +-7 in every row quantise with scale
    7 / 448 = 2^-6 to exact E4M3 codes (64 x), and with integer queries every
    traversal distance is an exact integer in all three forms: the FP32 and
    BF16 forms' canonical sums and the FP8 form's f16 differences (the
    converter applying the row scale) with FP32 dot-product accumulation.  So
    the three forms must return the same ids and distances bit for bit; this
    pins the packed FP8 converter's format, byte order and scale operand."""
    rng = np.random.default_rng(77)
    n, d = 4000, 64
    X = rng.integers(-7, 8, size=(n, d)).astype(np.float32)
    X[np.arange(n), rng.integers(0, d, size=n)] = np.where(rng.random(n) < 0.5, 7.0, -7.0)
    Q = rng.integers(-20, 21, size=(300, d)).astype(np.float32)
    base = hn.henn_build(to_dev(X), degree=12, metric=metric, graph=1, max_degree=24,
                         root_complete_max=300)
    ex = [base.export_layer(i) for i in range(base.num_layers)]
    res = {}
    for storage in (0, 1, 2):
        idx = hn.henn_import(to_dev(X), [e[0] for e in ex], [e[1] for e in ex], storage=storage,
                             degree=12, metric=metric, graph=1, max_degree=24,
                             root_complete_max=300)
        for mode in (True, False):
            gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=32, root_kernel=mode)
            _sync()
            res[(storage, mode)] = (gi.cpu().numpy(), gd.cpu().numpy().view(np.uint32))
        idx.free()
    base.free()
    ref = res[(0, True)]
    for key, (ids, dist) in res.items():
        assert np.array_equal(ids, ref[0]), key
        assert np.array_equal(dist, ref[1]), key


@pytest.mark.parametrize("storage,metric,d", [(0, 0, 32), (1, 0, 96), (2, 0, 128), (0, 1, 64),
                                              (2, 1, 40)])
def test_root_scan_kernel_matches_in_kernel_scan(hn, ho, storage, metric, d):
    """The matrix-core root scan (Gram shortlist + exact check), the tiled
    VALU scan and the in-kernel scan find the same root member, so the
    searches agree bit for bit."""
    X = wl.uniform(6000, d, 50) - 0.5
    Q = wl.uniform(700, d, 51) - 0.5
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    idx = hn.henn_build(to_dev(X), degree=12, metric=metric, storage=storage, graph=1,
                        max_degree=24, root_complete_max=700)
    assert idx.num_layers >= 2
    a_i, a_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40)
    for mode in (False, "valu"):
        b_i, b_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40, root_kernel=mode)
        _sync()
        assert np.array_equal(a_i.cpu().numpy(), b_i.cpu().numpy()), mode
        assert np.array_equal(a_d.cpu().numpy().view(np.uint32),
                              b_d.cpu().numpy().view(np.uint32)), mode
    idx.free()


@pytest.mark.parametrize("nq", [1, 3, 9])
def test_root_check_with_a_half_filled_last_wave(hn, nq):
    """The exact check takes two queries a wave and eight a block: batches of
    1, 3 and 9 queries leave half waves and whole waves without a query.  The
    results must equal the in-kernel scan's, bit for bit."""
    X = wl.uniform(5000, 64, 52) - 0.5
    Q = wl.uniform(nq, 64, 53) - 0.5
    idx = hn.henn_build(to_dev(X), degree=12, metric=0, storage=2, graph=1, max_degree=24,
                        root_complete_max=700)
    assert idx.num_layers >= 2
    a_i, a_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40)
    b_i, b_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40, root_kernel=False)
    _sync()
    assert np.array_equal(a_i.cpu().numpy(), b_i.cpu().numpy())
    assert np.array_equal(a_d.cpu().numpy().view(np.uint32), b_d.cpu().numpy().view(np.uint32))
    idx.free()


@pytest.mark.parametrize("storage", [0, 2])
def test_root_shortlist_overflow_matches_in_kernel_scan(hn, ho, storage):
    """A third of the points are copies of one point, so the root holds many
    rows with equal Gram values: queries near that point list more rows than
    a shortlist holds, and the check falls back to scanning the root.  The
    results must still equal the in-kernel scan's, bit for bit."""
    rng = np.random.default_rng(91)
    X = (wl.uniform(3000, 48, 60) - 0.5).astype(np.float32)
    X[:1000] = X[1000]
    Q = np.concatenate([X[1000] + 1e-3 * rng.standard_normal((200, 48)),
                        wl.uniform(200, 48, 61) - 0.5]).astype(np.float32)
    idx = hn.henn_build(to_dev(X), degree=12, metric=0, storage=storage, graph=1,
                        max_degree=24, root_complete_max=1000)
    assert idx.num_layers >= 2
    root = idx.export_layer(idx.num_layers - 1)[0]
    assert np.sum(root < 1001) > 40, "the root should hold many copies"
    a_i, a_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40)
    b_i, b_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40, root_kernel=False)
    _sync()
    assert np.array_equal(a_i.cpu().numpy(), b_i.cpu().numpy())
    assert np.array_equal(a_d.cpu().numpy().view(np.uint32), b_d.cpu().numpy().view(np.uint32))
    idx.free()


def _knn_positions(X, R):
    """Positions of each row's R nearest other rows (exact, FP64)."""
    X = X.astype(np.float64)
    sq = (X * X).sum(1)
    D = sq[:, None] + sq[None, :] - 2.0 * (X @ X.T)
    np.fill_diagonal(D, np.inf)
    return np.argsort(D, axis=1, kind="stable")[:, :R].astype(np.int32)


@pytest.mark.parametrize("storage", [0, 2])
def test_root_rows_past_a_lanes_room_match_in_kernel_scan(hn, storage):
    """Groups of near copies in a complete root of 1,000 rows (24 in one
    tile, one group split over two tiles) give a query more rows within the
    shortlist margin than one lane of the Gram pass keeps in registers, while
    the list itself does not overflow.  The results must equal the in-kernel
    scan's and the tiled scan's, bit for bit."""
    rng = np.random.default_rng(93)
    n, d, s, R = 3000, 48, 1000, 12
    X = (wl.uniform(n, d, 62) - 0.5).astype(np.float32)
    groups = [list(range(0, 3)) + list(range(96, 102)), list(range(32, 38)),
              list(range(64, 88)), list(range(200, 205))]
    centres = []
    for rows in groups:
        base = X[rows[0]].copy()
        X[rows] = base + 1e-5 * rng.standard_normal((len(rows), d)).astype(np.float32)
        centres.append(base)
    Q = np.concatenate([c + 1e-3 * rng.standard_normal((20, d)) for c in centres] +
                       [wl.uniform(100, d, 63) - 0.5]).astype(np.float32)
    adj0 = _knn_positions(X, R)
    adj1 = _knn_positions(X[:s], R)
    idx = hn.henn_import(to_dev(X), [None, np.arange(s, dtype=np.int32)], [adj0, adj1],
                         storage=storage, degree=R, metric=0, graph=1, max_degree=R,
                         root_complete_max=s)
    a_i, a_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40)
    for mode in (False, "valu"):
        b_i, b_d = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=40, root_kernel=mode)
        _sync()
        assert np.array_equal(a_i.cpu().numpy(), b_i.cpu().numpy()), mode
        assert np.array_equal(a_d.cpu().numpy().view(np.uint32),
                              b_d.cpu().numpy().view(np.uint32)), mode
    idx.free()


def test_autotune_caches_a_shape_and_keeps_results(hn, cfg1_sym_root):
    X, Q, oidx = cfg1_sym_root
    idx = _import(hn, X, oidx, storage=1)
    Qd = to_dev(Q)
    ref_i, ref_d = hn.henn_search_batch(idx, Qd, k=10, ef=64, lanes_per_vec=4, waves_per_block=4,
                                        vis_bits=10)
    _sync()
    shape = hn.henn_autotune(idx, Qd, k=10, ef=64)
    assert shape["lanes_per_vec"] in (1, 2, 4) and 8 <= shape["vis_bits"] <= 12  # the swept range
    gi, gd = hn.henn_search_batch(idx, Qd, k=10, ef=64)  # uses the cached shape
    _sync()
    assert np.array_equal(gi.cpu().numpy(), ref_i.cpu().numpy())
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), ref_d.cpu().numpy().view(np.uint32))
    idx.free()


@pytest.mark.parametrize("mixed", [False, True])
def test_search_graph_replays_match_eager(hn, cfg1_sym_root, mixed):
    """hipGraph form: every replay (new queries copied into the bound buffer,
    eager work and synchronisation in between) equals the eager search."""
    import torch
    X, Q, oidx = cfg1_sym_root
    idx = _import(hn, X, oidx, storage=2)
    n = 400
    kw = dict(k=10, ef=64)
    if mixed:
        ks = to_dev(np.array([1, 10, 5, 10] * (n // 4), dtype=np.int32))
        efs = to_dev(np.array([32, 64, 16, 48, 64] * (n // 5), dtype=np.int32))
        kw = dict(k=10, ef=64, k_arr=ks, ef_arr=efs, k_max=10, ef_max=64)
    g = hn.SearchGraph(idx, to_dev(Q[:n]).clone(), persistent=True, **kw)
    for rep in range(4):
        qs = np.roll(Q, -137 * rep, axis=0)[:n].copy()
        g.Q.copy_(to_dev(qs))
        gi, gd = g.launch()
        torch.cuda.synchronize()
        gi, gd = gi.cpu().numpy().copy(), gd.cpu().numpy().copy()
        ei, ed = hn.henn_search_batch(idx, to_dev(qs), **kw)
        torch.cuda.synchronize()
        assert np.array_equal(gi, ei.cpu().numpy()), rep
        assert np.array_equal(gd.view(np.uint32), ed.cpu().numpy().view(np.uint32)), rep
    g.free()
    idx.free()


# ------------------------------------------------- pruned navigable graphs ---

@pytest.mark.parametrize("graph,metric", [(2, 0), (3, 0), (3, 1)])
def test_pruned_graphs_match_oracle(hn, ho, graph, metric):
    """Diversity-pruned graphs (with and without reverse edges) against the
    oracle's, layer by layer.  Rows whose candidate order, candidate cut or
    pruning comparisons hold a near tie are exempt; with reverse edges, so
    are the rows such a node may point to."""
    X = wl.uniform(6000, 24, 60) - 0.5
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    p = ho.BuildParams(degree=12, graph=graph, max_degree=28, metric=metric)
    oidx = ho.build_index(X, p)
    idx = hn.henn_build(to_dev(X), degree=12, graph=graph, max_degree=28, metric=metric)
    layers = _gpu_layers(idx)
    assert len(layers) == oidx.num_layers
    C = ho.prune_candidates(12)
    checked = 0
    for i, (ids, adj) in enumerate(layers):
        assert np.array_equal(ids, oidx.members[i])
        mb = oidx.members[i]
        cand, _, cut, order = ho.knn_graph(X, metric, mb, C)
        _, pm = ho.prune(X, metric, mb, cand, 12)
        tie = np.minimum(np.minimum(cut, order), pm) <= exempt_tol(X.shape[1])
        if graph == 3:
            spread = tie.copy()
            for u in np.where(tie)[0]:
                spread[cand[u][cand[u] >= 0]] = True
            tie = spread
        same = (adj == oidx.adj[i]).all(1)
        assert (same | tie).all(), f"layer {i}: rows {np.where(~same & ~tie)[0][:5]}"
        checked += int((~tie).sum())
    assert checked > 0.75 * sum(len(m) for m in oidx.members)
    idx.free()


def test_pruned_sym_search_parity(hn, ho):
    """Search on a GPU-built PRUNED_SYM hierarchy against the oracle searching
    the same exported hierarchy."""
    X, Q = wl.make("uniform_10k_d32")
    idx = hn.henn_build(to_dev(X), degree=16, graph=3, max_degree=32, root_complete_max=1000)
    layers = _gpu_layers(idx)
    oidx = ho.index_from_arrays(X, 0, [l[0] for l in layers], [l[1] for l in layers],
                                root_complete=True)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=48)
    _sync()
    ores = ho.search(oidx, Q, 10, 48)
    assert_search_parity(gi.cpu().numpy(), gd.cpu().numpy(), ores, X, Q, max_exempt=0.087)
    idx.free()


@pytest.mark.parametrize("storage", [0, 2])
def test_visited_tags_and_ids_give_the_same_results(hn, cfg1_sym_root, storage):
    """The visited table may hold 8- or 16-bit tags (slot = low id bits) or
    full ids (multiplicative hash); it only decides what is re-evaluated, so
    the results are identical, also for a table small enough to evict often
    (10,000 points: 8-bit tags are exact for every table size here)."""
    X, Q, oidx = cfg1_sym_root
    idx = _import(hn, X, oidx, storage=storage)
    Qd = to_dev(Q)
    for vb in (8, 10, 12):
        a_i, a_d = hn.henn_search_batch(idx, Qd, k=10, ef=64, vis_bits=vb)
        for kw in (dict(vis16=True), dict(vis32=True)):
            b_i, b_d = hn.henn_search_batch(idx, Qd, k=10, ef=64, vis_bits=vb, **kw)
            _sync()
            assert np.array_equal(a_i.cpu().numpy(), b_i.cpu().numpy()), (vb, kw)
            assert np.array_equal(a_d.cpu().numpy().view(np.uint32),
                                  b_d.cpu().numpy().view(np.uint32)), (vb, kw)
    idx.free()


# ---------------------------------------------------------------- NSW graphs

def _explained_rows(got, ref, margin, lo, hi, tol):
    """Rows of one NSW insertion batch that may differ between the GPU (got)
    and the oracle (ref): a row decided by a near tie (its own search or merge,
    margin <= tol), and a row that a near-tie new point links to in either
    graph (its merge then takes or misses that point)."""
    tie = margin <= tol
    linked = np.zeros(len(margin), bool)
    for p in np.where(tie[lo:hi])[0] + lo:
        for row in (got[p], ref[p]):
            linked[row[row >= 0]] = True
    return tie | linked


@pytest.mark.parametrize("metric,d", [(0, 16), (1, 20)])
def test_nsw_insert_batch_matches_oracle(hn, ho, metric, d):
    """Every NSW insertion batch of a layer, run on the GPU from the oracle's
    graph state before it, against the oracle's batch: each differing row is
    one the oracle recorded a near tie for, or linked to such a new point."""
    import torch
    s, R, M, ef = 3000, 8, 16, 32
    X = np.ascontiguousarray(wl.uniform(s, d, 31) - (0.5 if metric else 0.0), dtype=np.float32)
    mb = np.arange(s, dtype=np.int32)
    adj = np.full((s, M), -1, np.int32)
    Vd = to_dev(X)
    tol = exempt_tol(d)
    tied = differ = 0
    batches = list(ho.nsw_batches(s, 3))
    for lo, hi in batches:
        g = torch.from_numpy(adj.copy()).to("cuda:0")
        hn.henn_nsw_insert(Vd, g, lo, hi, R, ef, metric=metric)
        got = g.cpu().numpy()
        bm = np.full(s, np.inf)
        ho.nsw_insert(X, metric, mb, adj, bm, lo, hi, R, ef)
        diff = np.any(got != adj, axis=1)
        ok = _explained_rows(got, adj, bm, lo, hi, tol)
        assert not np.any(diff & ~ok), (lo, hi, np.where(diff & ~ok)[0][:5])
        assert np.all(got[hi:] == -1)
        tied += int((bm <= tol).sum())
        differ += int(diff.sum())
    print(f"{len(batches)} batches: {tied} near-tie rows, {differ} rows differ")
    assert tied < 0.05 * s


@pytest.mark.parametrize("metric", [0, 1])
def test_nsw_build_matches_oracle(hn, ho, metric):
    """Whole NSW builds: same layers, nearly all rows identical (a near tie in
    one batch can move later rows), and the same search quality."""
    X = np.ascontiguousarray(wl.uniform(6000, 24, 41) - (0.5 if metric else 0.0),
                             dtype=np.float32)
    Q = np.ascontiguousarray(wl.uniform(300, 24, 42) - (0.5 if metric else 0.0),
                             dtype=np.float32)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=5, metric=metric)
    oidx = ho.build_index(X, ho.BuildParams(**p))
    idx = hn.henn_build(to_dev(X), **p)
    layers = _gpu_layers(idx)
    assert len(layers) == oidx.num_layers
    for i, (ids, adj) in enumerate(layers):
        assert np.array_equal(ids, oidx.members[i])
        same = (adj == oidx.adj[i]).all(1).mean()
        print(f"layer {i}: {same:.4f} of {len(ids)} rows identical")
        assert same >= 0.98, (i, same)
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=48)
    ores = ho.search(oidx, Q, k=10, ef=48)
    _, gt_d = ho.brute_force_knn(X, Q, 10, metric)
    rg = ho.recall_at_k(gi.cpu().numpy(), gt_d, X, Q, metric)
    ro = ho.recall_at_k(ores.ids, gt_d, X, Q, metric)
    assert rg > 0.8 and abs(rg - ro) < 0.02, (rg, ro)      # 24-d uniform data, ef 48
    idx.free()


# --------------------------------------------------- Insert(x) (App. C) ----

@pytest.mark.parametrize("metric,root_max", [(0, 0), (1, 0), (0, 400)])
def test_insert_matches_oracle(hn, ho, metric, root_max):
    """Insert(x) into an NSW index on the GPU against the oracle's insertion:
    same members per layer, nearly all rows identical, same search quality."""
    sh = 0.5 if metric else 0.0
    X = np.ascontiguousarray(wl.uniform(6000, 24, 51) - sh, dtype=np.float32)
    Xn = np.ascontiguousarray(wl.uniform(3000, 24, 52) - sh, dtype=np.float32)
    Q = np.ascontiguousarray(wl.uniform(300, 24, 53) - sh, dtype=np.float32)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=6, metric=metric,
             root_complete_max=root_max)
    bp = ho.BuildParams(**p)
    grown = ho.insert(ho.build_index(X, bp), Xn, bp)
    idx = hn.henn_build(to_dev(X), **p)
    hn.henn_insert(idx, to_dev(Xn))
    assert idx.shape()[1] == 9000
    layers = _gpu_layers(idx)
    assert len(layers) == grown.num_layers
    for i, (ids, adj) in enumerate(layers):
        assert np.array_equal(ids, grown.members[i]), f"layer {i}"
        same = (adj == grown.adj[i]).all(1).mean()
        print(f"layer {i}: {same:.4f} of {len(ids)} rows identical")
        assert same >= 0.98, (i, same)
    Xa = np.concatenate([X, Xn])
    gi, gd = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=48)
    ores = ho.search(grown, Q, k=10, ef=48)
    _, gt_d = ho.brute_force_knn(Xa, Q, 10, metric)
    rg = ho.recall_at_k(gi.cpu().numpy(), gt_d, Xa, Q, metric)
    ro = ho.recall_at_k(ores.ids, gt_d, Xa, Q, metric)
    assert rg > 0.8 and abs(rg - ro) < 0.02, (rg, ro)
    idx.free()


@pytest.mark.parametrize("metric", [0, 1])
def test_insert_rows_attributed_on_imported_index(hn, ho, metric):
    """Insert(x) into the oracle's own NSW hierarchy, imported into the library:
    with insert_shift 0 each layer takes its new points in one insertion
    batch, so every row that differs from the oracle's insertion is decided by
    a near tie of that batch or linked to such a new point."""
    sh = 0.5 if metric else 0.0
    X = np.ascontiguousarray(wl.uniform(5000, 24, 54) - sh, dtype=np.float32)
    Xn = np.ascontiguousarray(wl.uniform(800, 24, 55) - sh, dtype=np.float32)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=6, metric=metric,
             insert_shift=0)
    bp = ho.BuildParams(**p)
    built = ho.build_index(X, bp)
    base = ho.index_from_arrays(X, metric, built.members, built.adj)
    base.order_margin = [np.full(len(m), np.inf) for m in built.members]
    base.info = built.info
    grown = ho.insert(base, Xn, bp)
    idx = hn.henn_import(to_dev(X), built.members, built.adj, **p)
    hn.henn_insert(idx, to_dev(Xn))
    tol = exempt_tol(24)
    for i, (ids, adj) in enumerate(_gpu_layers(idx)):
        assert np.array_equal(ids, grown.members[i]), f"layer {i}"
        lo, hi = len(built.members[i]), len(ids)
        assert hi - lo <= max(1, lo), "one batch per layer"
        diff = np.any(adj != grown.adj[i], axis=1)
        ok = _explained_rows(adj, grown.adj[i], grown.order_margin[i], lo, hi, tol)
        assert not np.any(diff & ~ok), (i, np.where(diff & ~ok)[0][:5])
        print(f"layer {i}: {hi - lo} new, {int(diff.sum())} rows differ, "
              f"{int((grown.order_margin[i] <= tol).sum())} near-tie rows")
    idx.free()


@pytest.mark.parametrize("storage", [1, 2])
def test_insert_precision_forms(hn, storage):
    """Insert(x) rebuilds the BF16 / FP8 copies: the grown index searches like
    its FP32 twin (same graphs) up to the precision forms' usual recall gap."""
    X = wl.uniform(5000, 32, 61)
    Xn = wl.uniform(5000, 32, 62)
    Q = to_dev(wl.uniform(200, 32, 63))
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=3)
    a = hn.henn_build(to_dev(X), storage=0, **p)
    b = hn.henn_build(to_dev(X), storage=storage, **p)
    for ix in (a, b):
        hn.henn_insert(ix, to_dev(Xn))
    for i in range(a.num_layers):
        assert np.array_equal(a.export_layer(i)[1], b.export_layer(i)[1])
    ia, _ = hn.henn_search_batch(a, Q, k=10, ef=64)
    ib, db = hn.henn_search_batch(b, Q, k=10, ef=64)
    ia, ib = ia.cpu().numpy(), ib.cpu().numpy()
    overlap = np.mean([len(set(x) & set(y)) / 10 for x, y in zip(ia, ib)])
    assert overlap > 0.9 and (ib >= 5000).any()
    assert np.all(np.diff(db.cpu().numpy(), axis=1) >= 0)
    a.free()
    b.free()


def test_insert_rejects_other_graphs(hn):
    idx = hn.henn_build(to_dev(wl.uniform(2000, 8, 1)), degree=8)
    with pytest.raises(hn.HennError):
        hn.henn_insert(idx, to_dev(wl.uniform(10, 8, 2)))
    idx.free()


# --------------------------------------------------- Delete(x) (App. C) ----

def _delete_case(hn, ho, X, Q, p, gone, then_insert=None):
    bp = ho.BuildParams(**p)
    oidx = ho.delete(ho.build_index(X, bp), gone, bp)
    idx = hn.henn_build(to_dev(X), **p)
    hn.henn_delete(idx, gone)
    Xa = X
    if then_insert is not None:
        oidx = ho.insert(oidx, then_insert, bp)
        hn.henn_insert(idx, to_dev(then_insert))
        Xa = np.concatenate([X, then_insert])
    layers = _gpu_layers(idx)
    assert len(layers) == oidx.num_layers
    for i, (ids, adj) in enumerate(layers):
        assert np.array_equal(ids, oidx.members[i]), f"layer {i}"
        same = (adj == oidx.adj[i]).all(1).mean()
        print(f"layer {i}: {same:.4f} of {len(ids)} rows identical")
        assert same >= 0.98, (i, same)
    gi, _ = hn.henn_search_batch(idx, to_dev(Q), k=10, ef=48)
    gi = gi.cpu().numpy()
    assert not np.isin(gi, gone).any()
    ores = ho.search(oidx, Q, k=10, ef=48)
    live = oidx.members[0]
    _, gt_d = ho.brute_force_knn(Xa[live], Q, 10, p.get("metric", 0))
    rg = ho.recall_at_k(gi, gt_d, Xa, Q, p.get("metric", 0))
    ro = ho.recall_at_k(ores.ids, gt_d, Xa, Q, p.get("metric", 0))
    assert rg > 0.8 and abs(rg - ro) < 0.02, (rg, ro)
    return idx


@pytest.mark.parametrize("metric,root_max", [(0, 0), (1, 0), (0, 400)])
def test_delete_matches_oracle(hn, ho, metric, root_max):
    """Delete(x) on the GPU against the oracle's: same layers, repaired rows
    identical (near ties aside), no deleted id returned, same recall."""
    sh = 0.5 if metric else 0.0
    X = np.ascontiguousarray(wl.uniform(6000, 24, 71) - sh, dtype=np.float32)
    Q = np.ascontiguousarray(wl.uniform(300, 24, 72) - sh, dtype=np.float32)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=2, metric=metric,
             root_complete_max=root_max)
    gone = np.random.default_rng(9).choice(6000, 1500, replace=False).astype(np.int32)
    idx = _delete_case(hn, ho, X, Q, p, gone)
    assert idx.shape()[1] == 4500
    idx.free()


def test_delete_redraws_thinned_layers_and_insert_continues(hn, ho):
    """Deleting most of layer 1 redraws it and the layers above (bit-exact
    samples); a later Insert(x) continues after the largest id."""
    X = wl.uniform(6000, 16, 73)
    Q = wl.uniform(300, 16, 74)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=3)
    ref = ho.build_index(X, ho.BuildParams(**p))
    gone = ref.members[1][: int(0.7 * len(ref.members[1]))].astype(np.int32)
    idx = _delete_case(hn, ho, X, Q, p, gone, then_insert=wl.uniform(2000, 16, 75))
    ids0 = idx.export_layer(0)[0]
    assert ids0[-1] == 7999 and len(ids0) == 8000 - len(gone)
    idx.free()


@pytest.mark.parametrize("metric", [0, 1])
def test_delete_rows_attributed_on_imported_index(hn, ho, metric):
    """Delete(x) on the oracle's own NSW hierarchy, imported into the library:
    the repair reads the same graph on both sides, so every repaired row equals
    the oracle's unless the oracle recorded a near tie in its sorted list."""
    sh = 0.5 if metric else 0.0
    X = np.ascontiguousarray(wl.uniform(6000, 24, 81) - sh, dtype=np.float32)
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=2, metric=metric)
    bp = ho.BuildParams(**p)
    built = ho.build_index(X, bp)
    base = ho.index_from_arrays(X, metric, built.members, built.adj)
    base.order_margin = [np.full(len(m), np.inf) for m in built.members]
    base.info = built.info
    gone = np.random.default_rng(10).choice(6000, 1500, replace=False).astype(np.int32)
    out = ho.delete(base, gone, bp)
    idx = hn.henn_import(to_dev(X), built.members, built.adj, **p)
    hn.henn_delete(idx, gone)
    layers = _gpu_layers(idx)
    assert len(layers) == out.num_layers == built.num_layers   # no layer is redrawn here
    tol = exempt_tol(24)
    for i, (ids, adj) in enumerate(layers):
        assert np.array_equal(ids, out.members[i]), f"layer {i}"
        diff = np.any(adj != out.adj[i], axis=1)
        tie = out.order_margin[i] <= tol
        assert not np.any(diff & ~tie), (i, np.where(diff & ~tie)[0][:5])
        print(f"layer {i}: {int(diff.sum())} rows differ, {int(tie.sum())} near-tie rows")
    idx.free()


@pytest.mark.parametrize("storage", [1, 2])
def test_delete_precision_forms(hn, storage):
    X = wl.uniform(5000, 32, 76)
    Q = to_dev(wl.uniform(200, 32, 77))
    p = dict(degree=8, max_degree=16, graph=4, ef_construction=48, seed=4)
    gone = np.arange(0, 5000, 3, dtype=np.int32)
    a = hn.henn_build(to_dev(X), storage=0, **p)
    b = hn.henn_build(to_dev(X), storage=storage, **p)
    for ix in (a, b):
        hn.henn_delete(ix, gone)
    ia, _ = hn.henn_search_batch(a, Q, k=10, ef=64)
    ib, db = hn.henn_search_batch(b, Q, k=10, ef=64)
    ia, ib = ia.cpu().numpy(), ib.cpu().numpy()
    assert not np.isin(ib, gone).any() and not np.isin(ia, gone).any()
    overlap = np.mean([len(set(x) & set(y)) / 10 for x, y in zip(ia, ib)])
    assert overlap > 0.9
    assert np.all(np.diff(db.cpu().numpy(), axis=1) >= 0)
    a.free()
    b.free()


def test_delete_argument_errors(hn):
    idx = hn.henn_build(to_dev(wl.uniform(2000, 8, 78)), degree=8, max_degree=16, graph=4)
    with pytest.raises(hn.HennError):
        hn.henn_delete(idx, [2000])                 # not in the index
    with pytest.raises(hn.HennError):
        hn.henn_delete(idx, np.arange(2000))        # would empty the index
    hn.henn_delete(idx, [5, 5, 7])                  # repeats are fine
    assert idx.shape()[1] == 1998
    with pytest.raises(hn.HennError):
        hn.henn_delete(idx, [5])                    # already gone
    idx.free()
    knn = hn.henn_build(to_dev(wl.uniform(2000, 8, 79)), degree=8)
    with pytest.raises(hn.HennError):
        hn.henn_delete(knn, [1])
    knn.free()

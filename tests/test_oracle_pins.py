"""Pins of the FP64 oracle against things other than itself.

Each test ties one oracle function to the paper's definitions, a closed form,
an independent library routine or a brute-force recomputation:

* Philox4x64-10 against NumPy's ``numpy.random.Philox`` (an independent
  implementation of Salmon et al., SC'11; NumPy increments its counter before
  the first block, so block B(x) is NumPy's first output for counter x-1).
* Eq. (1) against hand-computed values.
* Alg. 2 layer samples against ``np.unique`` of NumPy-Philox draws.
* Alg. 3 halving: sizes ceil(s / 2^m), one survivor per dyadic block, fair
  and independent coins, and a backward walk with NumPy-Philox coins.
* NSW graphs (App. B.2): with a beam as wide as the layer the insertion
  equals exact k-NN over the inserted prefix (brute force); row invariants.
* Insert(x) (App. C): growing a one-layer index from a batch boundary equals
  building it whole; upper-layer membership against NumPy-Philox coins,
  nesting and the 2^-m rate.
* Delete(x) (App. C): the repair rule written out with NumPy keys; the
  closed form on the complete graph (the complete graph on the survivors);
  rows without deleted neighbours unchanged; no deleted point left in layers
  or results; a thinned layer is drawn again.
* Ring ranges (Def. Ring Ranges) and the hit test against a NumPy lexsort.
* The exact kNN graph (App. B.2) against NumPy all-pairs + lexsort.
* Search: complete graph => exact k-NN (App. B.2: the complete graph is
  trivially navigable); ef >= reachable set => exact k-NN over that set;
  ef = 1 => Alg. 4 GreedySearch written out separately; the equivalences the
  GPU kernel relies on (flagged result list, any neighbour order, a lossy
  visited table) against a separate implementation.
* Brute-force k-NN and the tie-tolerant Recall@k (Sec. 2).
"""
import math

import numpy as np
import pytest

import workloads as wl

MASK64 = (1 << 64) - 1


def numpy_block(counter, key):
    x = sum(int(c) << (64 * i) for i, c in enumerate(counter))
    x = (x - 1) % (1 << 256)
    c = np.array([(x >> (64 * i)) & MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=c)
    return [int(v) for v in bg.random_raw(4)]


def numpy_stream(seed, tag, layer, attempt, count):
    """Words 0..count-1 of stream (tag, layer, attempt) from NumPy's Philox."""
    x = (0 + (layer << 64) + (attempt << 128) + (tag << 192) - 1) % (1 << 256)
    c = np.array([(x >> (64 * i)) & MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64), counter=c)
    nblk = (count + 3) // 4
    return [int(v) for v in bg.random_raw(4 * nblk)[:count]]


def numpy_uindex(words, s):
    return np.array([(w * s) >> 64 for w in words], dtype=np.int64)


def d64_seq(a, b, metric=0):
    """FP64 distance summed in coordinate order (same rounding as the C loop)."""
    acc = 0.0
    if metric == 0:
        for x, y in zip(a.tolist(), b.tolist()):
            t = float(x) - float(y)
            acc += t * t
        return acc
    for x, y in zip(a.tolist(), b.tolist()):
        acc += float(x) * float(y)
    return -acc


# ---------------------------------------------------------------- Philox ---

@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [5, 0]),
    ([0, 3, 7, 1], [123456789, 0]),
    ([MASK64, MASK64, 2, 3], [2**63 + 11, 0]),
    ([17, 0, 0, 2], [MASK64, 0]),
])
def test_philox_block_matches_numpy(oracle, counter, key):
    got = [int(v) for v in oracle.philox_block(counter, key)]
    assert got == numpy_block(counter, key)


def test_stream_words_and_uniform_index(oracle):
    for seed, tag, layer, attempt in [(0, 1, 1, 0), (7, 2, 3, 0), (99, 1, 2, 5)]:
        ref = numpy_stream(seed, tag, layer, attempt, 23)
        got = [oracle.stream_word(seed, tag, layer, attempt, q) for q in range(23)]
        assert got == ref
        for s in (1, 2, 17, 10_000, 2**31 - 1, 2**40 + 3):
            got_u = oracle.draw_indices(seed, tag, layer, attempt, s, 23)
            assert np.array_equal(got_u, numpy_uindex(ref, s))
            assert got_u.min() >= 0 and got_u.max() < s


def test_uniform_index_closed_form(oracle):
    assert oracle.uniform_index(0, 10) == 0
    assert oracle.uniform_index(MASK64, 10) == 9
    assert oracle.uniform_index(1 << 63, 10) == 5
    assert oracle.uniform_index(MASK64, 1) == 0


# ---------------------------------------------------------------- Eq. (1) --

def test_eps_schedule_values(oracle):
    # eps(s) = c0 * d * ln(s) / s * 2^m
    assert oracle.eps_of(10_000, 32, 4, 1.0) == pytest.approx(32 * math.log(1e4) / 1e4 * 16)
    assert oracle.eps_of(10_000, 32, 4, 1.0) == pytest.approx(0.471569, abs=1e-6)
    assert oracle.window_of(oracle.eps_of(10_000, 32, 4, 1.0), 10_000) == 4716
    assert oracle.eps_of(1_000_000, 128, 4, 1.0) == pytest.approx(0.0282942, abs=1e-6)
    # a heavy ring holds more than eps*s points
    assert oracle.window_of(0.5, 10) == 6
    assert oracle.window_of(0.05, 100) == 6


# ------------------------------------------------------- Alg. 2 sampling --

def _brute_rings(X, members, centres, starts, w, metric=0):
    rings = []
    for c, a in zip(centres, starts):
        dc = np.array([d64_seq(X[members[c]], X[members[j]], metric)
                       for j in range(len(members))])
        order = np.lexsort((members, dc))
        rings.append(set(order[a:a + w].tolist()))
    return rings


def test_layer_sample_vacuous_matches_numpy_unique(oracle):
    X = wl.uniform(3000, 32, 0)
    p = oracle.BuildParams(degree=8, seed=11)
    members, infos = oracle.build_layers(X, p)
    assert len(members) >= 2
    for i in range(1, len(members)):
        s = len(members[i - 1])
        D = -(-s // 16)
        assert infos[i].status == "vacuous"      # c0 = 1 makes eps >= 1 at this size
        draws = numpy_uindex(numpy_stream(11, 1, i, 0, D), s)
        assert np.array_equal(members[i], members[i - 1][np.unique(draws)])
        assert np.all(np.diff(members[i]) > 0)
        assert np.isin(members[i], members[i - 1]).all()     # nesting L_i in L_{i-1}


def test_layer_sample_verified_las_vegas(oracle):
    """With a small eps the Las-Vegas loop repeats; the accepted attempt is the
    first whose sample hits every sampled ring (checked by brute force)."""
    X = wl.uniform(2000, 3, 0)
    s, D = 2000, 125
    p = oracle.BuildParams(degree=8, seed=3, eps_override=0.031, num_rings=64,
                           max_layers=1)
    members, infos = oracle.build_layers(X, p)
    info = infos[1]
    w = oracle.window_of(0.031, s)
    assert info.window == w == 63
    r = 64
    centres = numpy_uindex(numpy_stream(3, 2, 1, 0, r), s)
    starts = numpy_uindex(numpy_stream(3, 3, 1, 0, r), s - w + 1)
    rings = _brute_rings(X, members[0], centres, starts, w)
    accepted = None
    for t in range(p.max_attempts):
        draws = set(numpy_uindex(numpy_stream(3, 1, 1, t, D), s).tolist())
        hits = sum(1 for ring in rings if ring & draws)
        if hits == r:
            accepted = t
            break
    assert accepted is not None and accepted >= 1, "fixture must exercise a repeat"
    assert info.status == "verified" and info.attempts == accepted + 1
    draws = numpy_uindex(numpy_stream(3, 1, 1, accepted, D), s)
    assert np.array_equal(members[1], np.unique(draws).astype(np.int32))


def test_attempt_cap_from_phi(oracle):
    """max_attempts 0: the cap is the smallest t with phi^t <= 1e-9, the
    point where a layer that keeps failing at rate phi has had its chance."""
    for phi, cap in ((0.5, 30), (0.2, 13), (5e-4, 3), (1e-9, 1), (0.999, 20713)):
        p = oracle.BuildParams(max_attempts=0, phi=phi)
        assert oracle.attempt_cap(p) == cap, phi
        assert phi ** cap <= 1e-9 and (cap == 1 or phi ** (cap - 1) > 1e-9)
    assert oracle.attempt_cap(oracle.BuildParams(max_attempts=7, phi=0.5)) == 7


def test_layer_sample_not_verified_keeps_best(oracle):
    X = wl.uniform(800, 2, 0)
    p = oracle.BuildParams(degree=8, seed=5, eps_override=0.002, num_rings=64,
                           max_attempts=4, max_layers=1)
    members, infos = oracle.build_layers(X, p)
    s, D = 800, 50
    w = infos[1].window
    centres = numpy_uindex(numpy_stream(5, 2, 1, 0, 64), s)
    starts = numpy_uindex(numpy_stream(5, 3, 1, 0, 64), s - w + 1)
    rings = _brute_rings(X, members[0], centres, starts, w)
    hits = []
    for t in range(4):
        draws = set(numpy_uindex(numpy_stream(5, 1, 1, t, D), s).tolist())
        hits.append(sum(1 for ring in rings if ring & draws))
    assert max(hits) < 64
    best = int(np.argmax(hits))      # lowest attempt with the most hits
    assert infos[1].status == "not_verified" and infos[1].hits == hits[best]
    draws = numpy_uindex(numpy_stream(5, 1, 1, best, D), s)
    assert np.array_equal(members[1], np.unique(draws).astype(np.int32))


# ------------------------------------------------------- Alg. 3 halving --

def _numpy_halving_walk(seed, layer, attempt, s, m):
    """Alg. 3's halving written backwards, with NumPy's Philox: with pairs of
    consecutive members the survivor of pair p lands at position p of the next
    step, so a final position is traced back through the m steps."""
    sizes = [s]
    for _ in range(m):
        sizes.append((sizes[-1] + 1) // 2)
    coins = [numpy_uindex(numpy_stream(seed, 4 + j, layer, attempt, sizes[j] // 2), 2)
             for j in range(m)]
    out = []
    for p in range(sizes[m]):
        pos = p
        for j in range(m - 1, -1, -1):
            pos = sizes[j] - 1 if pos == sizes[j] // 2 else 2 * pos + int(coins[j][pos])
        out.append(pos)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("s", [0, 1, 2, 3, 5, 16, 17, 31, 32, 33, 100, 1023, 4096])
@pytest.mark.parametrize("m", [1, 2, 4])
def test_halving_size_order_and_dyadic_blocks(oracle, s, m):
    got = oracle.halve(9, 2, 1, s, m)
    assert len(got) == -(-s // 2 ** m)                  # Cor. layer-size: ceil(s / 2^m)
    assert np.all(np.diff(got) > 0) and (len(got) == 0 or (got[0] >= 0 and got[-1] < s))
    if s % 2 ** m == 0:
        # consecutive pairs compose into dyadic blocks: one survivor per block
        assert np.array_equal(got // 2 ** m, np.arange(s // 2 ** m))
    if s % 2 == 1 and m == 1:
        assert got[-1] == s - 1                          # the unpaired last member stays


def test_halving_tiny_case_by_hand(oracle):
    # s = 5, m = 2: step 0 keeps one of {0,1}, one of {2,3} and 4; step 1
    # keeps one of the first two survivors and 4 again
    for t in range(50):
        got = oracle.halve(1, 1, t, 5, 2)
        assert len(got) == 2 and got[1] == 4 and 0 <= got[0] <= 3


@pytest.mark.parametrize("s,m", [(37, 1), (64, 3), (1000, 4), (77, 5)])
def test_halving_matches_backward_walk_with_numpy_philox(oracle, s, m):
    for seed, layer, attempt in [(0, 1, 0), (5, 3, 7)]:
        assert np.array_equal(oracle.halve(seed, layer, attempt, s, m),
                              _numpy_halving_walk(seed, layer, attempt, s, m))


def test_halving_coins_are_fair_and_independent(oracle):
    """Each halving keeps either member of a pair with probability 1/2, so
    with s = 16 and m = 2 every point survives with probability 1/4, and the
    choices in the four blocks are independent."""
    T = 4000
    picks = np.array([oracle.halve(13, 1, t, 16, 2) for t in range(T)])   # [T, 4]
    freq = np.bincount(picks.ravel(), minlength=16) / T
    assert np.all(np.abs(freq - 0.25) < 0.035), freq
    joint = np.bincount((picks[:, 0] % 4) * 4 + picks[:, 1] % 4, minlength=16) / T
    assert np.all(np.abs(joint - 1 / 16) < 0.025), joint


def test_halving_layer_las_vegas(oracle):
    """Alg. 3's sample goes through the same ring check: the kept attempt is
    the first halving that hits every sampled ring (brute force)."""
    X = wl.uniform(2000, 3, 0)
    s, r = 2000, 64
    p = oracle.BuildParams(degree=8, seed=3, eps_override=0.025, num_rings=r, max_layers=1,
                           sampler=1)
    members, infos = oracle.build_layers(X, p)
    w = oracle.window_of(0.025, s)
    centres = numpy_uindex(numpy_stream(3, 2, 1, 0, r), s)
    starts = numpy_uindex(numpy_stream(3, 3, 1, 0, r), s - w + 1)
    rings = _brute_rings(X, members[0], centres, starts, w)
    accepted = None
    for t in range(p.max_attempts):
        kept = set(_numpy_halving_walk(3, 1, t, s, 4).tolist())
        if all(ring & kept for ring in rings):
            accepted = t
            break
    assert accepted is not None and accepted >= 1, "fixture must exercise a repeat"
    assert infos[1].status == "verified" and infos[1].attempts == accepted + 1
    assert len(members[1]) == 125
    assert np.array_equal(members[1], _numpy_halving_walk(3, 1, accepted, s, 4))


# ---------------------------------------------------- NSW (App. B.2) -------

def test_nsw_batch_schedule(oracle):
    for s, shift in [(1, 3), (17, 3), (1000, 3), (1000, 0), (300, 62)]:
        b = list(oracle.nsw_batches(s, shift))
        assert b[0] == (0, 1) and b[-1][1] == s
        assert all(b[i][1] == b[i + 1][0] for i in range(len(b) - 1))
        assert all(hi - lo == min(s - lo, max(1, lo >> shift)) for lo, hi in b)
        if shift == 62:
            assert len(b) == s            # one point at a time: plain sequential insertion


def _nsw_by_exact_prefix_knn(X, metric, R, M, shift):
    """The NSW rule with every insertion search replaced by an exact k-NN
    over the points inserted before the batch (what a beam as wide as the
    layer finds on a connected graph).  Also reports whether a row ever
    overflowed M (a dropped reverse edge could disconnect the graph)."""
    s = len(X)
    D = np.array([[d64_seq(X[i], X[j], metric) for j in range(s)] for i in range(s)])
    rows = [[] for _ in range(s)]
    overflow = False
    lo = 0
    while lo < s:
        hi = min(s, lo + max(1, lo >> shift))
        new = {}
        for p in range(lo, hi):
            order = np.lexsort((np.arange(lo), D[p, :lo]))
            new[p] = order[:R].tolist()
        chosen = {}
        for p in range(lo, hi):
            rows[p] = list(new[p])
            for v in new[p]:
                chosen.setdefault(v, []).append(p)
        for v, ps in chosen.items():
            cand = rows[v] + ps
            overflow |= len(cand) > M
            cand.sort(key=lambda u: (D[v, u], u))
            rows[v] = cand[:M]
        lo = hi
    adj = np.full((s, M), -1, dtype=np.int32)
    for v in range(s):
        adj[v, :len(rows[v])] = rows[v]
    return adj, overflow


@pytest.mark.parametrize("metric,shift", [(0, 62), (0, 2), (1, 3)])
def test_nsw_with_exhaustive_beam_is_prefix_knn(oracle, metric, shift):
    X = wl.uniform(150, 4, 21) - (0.5 if metric == 1 else 0.0)
    X = np.ascontiguousarray(X, dtype=np.float32)
    mb = np.arange(150, dtype=np.int32)
    ref, overflow = _nsw_by_exact_prefix_knn(X, metric, 4, 64, shift)
    assert not overflow, "fixture must keep every reverse edge"
    got, _ = oracle.nsw_graph(X, metric, mb, 4, 64, 150, shift)
    assert np.array_equal(got, ref)


def test_nsw_graph_invariants(oracle):
    X = wl.uniform(2000, 8, 4)
    mb = np.arange(2000, dtype=np.int32)
    R, M = 8, 16
    adj, _ = oracle.nsw_graph(X, 0, mb, R, M, 32, 3)
    X64 = X.astype(np.float64)
    for v in range(2000):
        row = adj[v][adj[v] >= 0]
        assert np.all(adj[v][len(row):] == -1)            # padding only at the end
        assert len(set(row.tolist())) == len(row) and v not in row
        if v > 0:
            assert len(row) >= 1
        d = ((X64[row] - X64[v]) ** 2).sum(1)
        assert np.all(np.diff(d) >= -1e-12)              # (distance, id) order
    # the graph is navigable from the entry in practice: BFS from position 0
    seen = np.zeros(2000, bool)
    seen[0] = True
    frontier = [0]
    while frontier:
        nxt = [u for v in frontier for u in adj[v] if u >= 0 and not seen[u]]
        for u in nxt:
            seen[u] = True
        frontier = list(set(nxt))
    assert seen.mean() > 0.99


def test_nsw_index_search_quality(oracle):
    X = wl.uniform(4000, 8, 6)
    Q = wl.uniform(200, 8, 7)
    idx = oracle.build_index(X, oracle.BuildParams(degree=8, max_degree=16, graph=4,
                                                   ef_construction=32, seed=2))
    res = oracle.search(idx, Q, k=10, ef=48)
    _, gt_d = oracle.brute_force_knn(X, Q, 10, 0)
    assert oracle.recall_at_k(res.ids, gt_d, X, Q) > 0.95


# ------------------------------------------ Insert(x), App. C (NSW index) --

def test_insert_into_layer0_continues_the_build(oracle):
    """A single-layer NSW index built on a prefix that ends at a batch boundary
    and then given the rest by Insert(x) is the index built on all points."""
    X = wl.uniform(3000, 8, 12)
    starts = [lo for lo, _ in oracle.nsw_batches(3000, 3)]
    n0 = [lo for lo in starts if lo >= 1800][0]
    p = oracle.BuildParams(degree=8, max_degree=16, graph=4, ef_construction=32, max_layers=0)
    full = oracle.build_index(X, p)
    grown = oracle.insert(oracle.build_index(X[:n0], p), X[n0:], p)
    assert grown.num_layers == 1 and np.array_equal(grown.members[0], full.members[0])
    assert np.array_equal(grown.adj[0], full.adj[0])


def test_insert_membership_coins_and_nesting(oracle):
    X = wl.uniform(6000, 8, 13)
    Xn = wl.uniform(4000, 8, 14)
    p = oracle.BuildParams(degree=8, max_degree=16, graph=4, ef_construction=32, seed=9)
    idx = oracle.build_index(X, p)
    grown = oracle.insert(idx, Xn, p)
    new = np.arange(6000, 10000)
    for i in range(1, idx.num_layers):
        coins = numpy_uindex(numpy_stream(9, 5, i, 0, 10000), 16)
        new = new[coins[new] == 0]
        assert np.array_equal(grown.members[i], np.concatenate([idx.members[i], new]))
        assert np.isin(grown.members[i], grown.members[i - 1]).all()      # nesting
    k1 = len(grown.members[1]) - len(idx.members[1])
    assert abs(k1 - 4000 / 16) < 4 * math.sqrt(4000 / 16)       # probability 2^-m
    for i in range(grown.num_layers):
        a = grown.adj[i]
        assert a.shape == (len(grown.members[i]), 16)
        assert a.max() < len(grown.members[i]) and np.all((a >= 0).sum(1)[1:] >= 1)


def test_insert_keeps_search_quality(oracle):
    X = wl.uniform(5000, 8, 15)
    Xn = wl.uniform(3000, 8, 16)
    Q = wl.uniform(200, 8, 17)
    p = oracle.BuildParams(degree=8, max_degree=16, graph=4, ef_construction=32, seed=4)
    grown = oracle.insert(oracle.build_index(X, p), Xn, p)
    Xa = np.concatenate([X, Xn])
    res = oracle.search(grown, Q, k=10, ef=48)
    _, gt_d = oracle.brute_force_knn(Xa, Q, 10, 0)
    assert oracle.recall_at_k(res.ids, gt_d, Xa, Q) > 0.95
    assert (res.ids >= 5000).any()            # inserted points are found


# ------------------------------------------ Delete(x), App. C (NSW index) --

def _repair_by_definition(X, metric, members, adj, dflag):
    """The repair rule written out with NumPy keys: each live row that links to
    a deleted member takes the first M live points among its row and its
    deleted neighbours' rows (itself and repeats out), in (distance, id) order."""
    M = adj.shape[1]
    out = adj.copy()
    for v in range(len(members)):
        row = [u for u in adj[v] if u >= 0]
        if dflag[v] or not any(dflag[u] for u in row):
            continue
        cand = {u for u in row if not dflag[u]}
        for u in row:
            if dflag[u]:
                cand |= {w for w in adj[u] if w >= 0 and not dflag[w] and w != v}
        cand = sorted(cand, key=lambda u: (d64_seq(X[members[v]], X[members[u]], metric),
                                           members[u]))[:M]
        out[v] = cand + [-1] * (M - len(cand))
    return out


@pytest.mark.parametrize("metric", [0, 1])
def test_delete_repairs_rows_by_definition(oracle, metric):
    X = np.ascontiguousarray(wl.uniform(600, 4, 22) - (0.5 if metric else 0.0), dtype=np.float32)
    p = oracle.BuildParams(degree=6, max_degree=12, graph=4, ef_construction=24, max_layers=0,
                           metric=metric)
    idx = oracle.build_index(X, p)
    gone = np.random.default_rng(3).choice(600, 150, replace=False)
    dflag = np.zeros(600, bool)
    dflag[gone] = True
    ref = _repair_by_definition(X, metric, idx.members[0], idx.adj[0], dflag)
    keep = ~dflag
    newpos = np.cumsum(keep) - 1
    ref = np.where(ref[keep] >= 0, newpos[np.maximum(ref[keep], 0)], -1)
    out = oracle.delete(idx, gone, p)
    assert np.array_equal(out.members[0], np.flatnonzero(keep))
    assert np.array_equal(out.adj[0], ref)


@pytest.mark.parametrize("metric", [0, 1])
def test_delete_repair_of_the_complete_graph_is_complete_on_survivors(oracle, metric):
    """Closed form: when every row lists all other points in (distance, id)
    order (the complete graph, row capacity s - 1), every live row links to a
    deleted point, and its repaired row must be the complete graph on the live
    points: all other survivors, (distance, id) order, -1 padded."""
    s = 40
    X = np.ascontiguousarray(wl.uniform(s, 5, 26) - (0.5 if metric else 0.0), dtype=np.float32)
    Xd = X.astype(np.float64)
    D = ((Xd[:, None, :] - Xd[None, :, :]) ** 2).sum(-1) if metric == 0 else -(Xd @ Xd.T)
    ids = np.arange(s)
    adj = np.full((s, s - 1), -1, np.int32)
    for v in range(s):
        order = [u for u in np.lexsort((ids, D[v])) if u != v]
        adj[v] = order
    idx = oracle.index_from_arrays(X, metric, [ids.astype(np.int32)], [adj])
    idx.order_margin = [np.full(s, np.inf)]
    idx.info = [oracle.LayerInfo(s, s, 0.0, 0, 0, 0, "base")]
    p = oracle.BuildParams(degree=4, max_degree=s - 1, graph=4, max_layers=0, metric=metric)
    gone = np.array([0, 3, 4, 17, 18, 30, 39])
    out = oracle.delete(idx, gone, p)
    live = np.setdiff1d(ids, gone)
    assert np.array_equal(out.members[0], live)
    for j, v in enumerate(live):
        others = [u for u in live[np.lexsort((live, D[v, live]))] if u != v]
        want = np.searchsorted(live, others).tolist() + [-1] * (s - 1 - len(others))
        assert out.adj[0][j].tolist() == want, v


def test_delete_leaves_rows_without_deleted_neighbours_alone(oracle):
    """Rows that link to no deleted member keep their neighbours (renumbered)."""
    X = wl.uniform(800, 4, 27)
    p = oracle.BuildParams(degree=6, max_degree=12, graph=4, ef_construction=24, max_layers=0)
    idx = oracle.build_index(X, p)
    gone = np.random.default_rng(4).choice(800, 40, replace=False)
    out = oracle.delete(idx, gone, p)
    live = np.setdiff1d(np.arange(800), gone)
    untouched = 0
    for j, v in enumerate(live):
        row = [u for u in idx.adj[0][v] if u >= 0]
        if np.isin(row, gone).any():
            continue
        untouched += 1
        got = [int(live[u]) for u in out.adj[0][j] if u >= 0]
        assert got == row
    assert untouched > 400


def test_delete_search_returns_only_live_points(oracle):
    X = wl.uniform(4000, 8, 23)
    Q = wl.uniform(200, 8, 24)
    p = oracle.BuildParams(degree=8, max_degree=16, graph=4, ef_construction=32, seed=7)
    idx = oracle.build_index(X, p)
    gone = np.random.default_rng(5).choice(4000, 1000, replace=False)
    out = oracle.delete(idx, gone, p)
    for i in range(out.num_layers):
        assert not np.isin(out.members[i], gone).any()
        if i:
            assert np.isin(out.members[i], out.members[i - 1]).all()
    res = oracle.search(out, Q, k=10, ef=48)
    assert not np.isin(res.ids, gone).any()
    live = np.setdiff1d(np.arange(4000), gone)
    gt_ids, gt_d = oracle.brute_force_knn(X[live], Q, 10, 0)
    assert oracle.recall_at_k(res.ids, gt_d, X, Q) > 0.95


def test_delete_redraws_a_thinned_layer(oracle):
    """Deleting most of layer 1 leaves it below half its expected size, so it
    and the layers above are drawn again from the remaining layer 0."""
    X = wl.uniform(6000, 8, 25)
    p = oracle.BuildParams(degree=8, max_degree=16, graph=4, ef_construction=32, seed=8)
    idx = oracle.build_index(X, p)
    gone = idx.members[1][: int(0.7 * len(idx.members[1]))]
    out = oracle.delete(idx, gone, p)
    s0 = len(out.members[0])
    assert s0 == 6000 - len(gone)
    ref = oracle.build_layers(X, p)      # the layer loop on the remaining points
    members = [out.members[0]]
    infos = [ref[1][0]]
    oracle._extend_layers(X, members, infos, p)
    assert len(members) == out.num_layers
    for a, b in zip(members[1:], out.members[1:]):
        assert np.array_equal(a, b)
    assert 2 * len(out.members[1]) >= -(-s0 // 16)


def test_ring_members_brute_force(oracle):
    X = wl.uniform(500, 5, 3)
    members = np.arange(0, 500, 2, dtype=np.int32)      # a layer = every other point
    for c, a, w in [(0, 0, 10), (17, 5, 40), (249, 200, 50), (3, 0, 250)]:
        got, _ = oracle.ring_members(X, 0, members, c, a, w)
        ref = _brute_rings(X, members, [c], [a], w)[0]
        assert set(got.tolist()) == ref
        if a == 0:
            assert got[0] == c        # rank 0 is the centre itself


def test_eps_net_property_exhaustive_on_tiny_input(oracle):
    """When every point-centred minimal heavy ring is checked, an accepted
    sample is an eps-net for those rings (Def. eps-net, App. B.1)."""
    X = wl.uniform(160, 2, 9)
    s = 160
    eps = 0.2
    w = oracle.window_of(eps, s)
    # exhaustive verification: one ring per (centre, start)
    members = np.arange(s, dtype=np.int32)
    rings = [set(oracle.ring_members(X, 0, members, c, a, w)[0].tolist())
             for c in range(s) for a in range(0, s - w + 1)]
    D = 60
    for t in range(64):
        draws = set(oracle.draw_indices(1, 1, 1, t, s, D).tolist())
        if all(r & draws for r in rings):
            break
    else:
        pytest.fail("no attempt verified")
    # the accepted sample hits every heavy ring whose centre is a data point
    # and whose size exceeds eps*s (bigger rings contain a minimal one)
    for c in range(0, s, 7):
        dc = np.array([d64_seq(X[c], X[j]) for j in range(s)])
        order = np.lexsort((np.arange(s), dc))
        for a in range(0, s - w, 9):
            for extra in (0, 5):
                if a + w + extra <= s:
                    assert set(order[a:a + w + extra].tolist()) & draws


# --------------------------------------------------------- kNN graph -------

@pytest.mark.parametrize("metric", [0, 1])
def test_knn_graph_matches_numpy(oracle, metric):
    X = wl.uniform(300, 8, 4) - 0.5
    members = np.arange(0, 300, 1, dtype=np.int32)[::3].copy()
    R = 6
    adj, ad, cut, order = oracle.knn_graph(X, metric, members, R)
    Y = X[members].astype(np.float64)
    if metric == 0:
        D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    else:
        D = -(Y @ Y.T)
    for v in range(len(members)):
        dv = D[v].copy()
        dv[v] = np.inf
        ref = np.lexsort((np.arange(len(members)), dv))[:R]
        assert np.array_equal(adj[v], ref)
        assert np.allclose(ad[v], dv[ref], rtol=1e-12, atol=1e-12)


def test_knn_graph_small_layer_pads(oracle):
    X = wl.uniform(5, 3, 1)
    adj, _, _, _ = oracle.knn_graph(X, 0, np.arange(5, dtype=np.int32), 6)
    assert (adj[:, 4:] == -1).all() and (adj[:, :4] >= 0).all()


# --------------------------------------------------------- search ----------

def _one_layer_index(oracle, X, R, metric=0):
    p = oracle.BuildParams(degree=R, max_layers=0, metric=metric)
    return oracle.build_index(X, p)


@pytest.mark.parametrize("metric", [0, 1])
def test_complete_graph_gives_exact_knn(oracle, metric):
    X = wl.uniform(60, 6, 2) - 0.3
    Q = wl.uniform(25, 6, 3) - 0.3
    idx = _one_layer_index(oracle, X, 59, metric)
    assert idx.num_layers == 1
    res = oracle.search(idx, Q, k=10, ef=10)
    for i in range(len(Q)):
        dq = np.array([d64_seq(Q[i], X[j], metric) for j in range(60)])
        ref = np.lexsort((np.arange(60), dq))[:10]
        assert np.array_equal(res.ids[i], ref)
        assert np.array_equal(res.dist[i], dq[ref])


def test_large_ef_gives_exact_knn_over_reachable_set(oracle):
    X = wl.uniform(150, 5, 5)
    Q = wl.uniform(20, 5, 6)
    idx = _one_layer_index(oracle, X, 3)
    adj = idx.adj[0]
    seen, stack = {0}, [0]
    while stack:
        v = stack.pop()
        for u in adj[v]:
            if u >= 0 and u not in seen:
                seen.add(int(u))
                stack.append(int(u))
    reach = np.array(sorted(seen))
    res = oracle.search(idx, Q, k=8, ef=200)
    for i in range(len(Q)):
        dq = np.array([d64_seq(Q[i], X[j]) for j in reach])
        ref = reach[np.lexsort((reach, dq))][:8]
        assert np.array_equal(res.ids[i, :len(ref)], ref)
        if len(ref) < 8:
            assert (res.ids[i, len(ref):] == -1).all()


def _greedy_alg4(X, members, adj, q, v_global):
    """Alg. 4 GreedySearch on one layer under the (dist, id) order."""
    pos = {int(g): i for i, g in enumerate(members)}
    nxt = v_global
    while True:
        cur = nxt
        key_cur = (d64_seq(q, X[cur]), cur)
        nbrs = [int(members[u]) for u in adj[pos[cur]] if u >= 0]
        if not nbrs:
            return cur
        nxt = min(nbrs, key=lambda u: (d64_seq(q, X[u]), u))
        if (d64_seq(q, X[nxt]), nxt) >= key_cur:
            return cur


def test_ef1_is_alg4_greedy_search(oracle):
    X = wl.uniform(4000, 4, 7)
    Q = wl.uniform(40, 4, 8)
    idx = oracle.build_index(X, oracle.BuildParams(degree=8, seed=1))
    assert idx.num_layers >= 3
    res = oracle.search(idx, Q, k=1, ef=1, ef_upper=1)
    for i in range(len(Q)):
        v = int(idx.members[-1][0])          # smallest id of the root layer
        for lay in range(idx.num_layers - 1, -1, -1):
            v = _greedy_alg4(X, idx.members[lay], idx.adj[lay], Q[i], v)
        assert res.ids[i, 0] == v


def _flagged_w_search(X, members, adj, q, entry_local, ef, perm_rng, vis_slots):
    """Single-layer beam search in the form the GPU kernel uses: one sorted
    result list W with an 'expanded' flag per entry, a lossy direct-mapped
    visited table, duplicate check against W, neighbours in random order."""
    def key(l):
        return (d64_seq(q, X[members[l]]), int(members[l]))
    table = [-1] * vis_slots
    W = [(key(entry_local), entry_local, False)]
    table[entry_local % vis_slots] = entry_local
    while True:
        pos = next((i for i, w in enumerate(W) if not w[2]), None)
        if pos is None:
            break
        kc, c, _ = W[pos]
        W[pos] = (kc, c, True)
        nb = [int(u) for u in adj[c] if u >= 0]
        perm_rng.shuffle(nb)
        for u in nb:
            if table[(u * 2654435761) % vis_slots] == u:
                continue
            table[(u * 2654435761) % vis_slots] = u
            ku = key(u)
            if any(w[1] == u for w in W):
                continue
            if len(W) < ef or ku < W[-1][0]:
                W.append((ku, u, False))
                W.sort(key=lambda t: t[0])
                del W[ef:]
    return W


@pytest.mark.parametrize("vis_slots", [4096, 7])
def test_flagged_list_and_lossy_visited_equivalence(oracle, vis_slots):
    X = wl.uniform(250, 4, 10)
    Q = wl.uniform(15, 4, 11)
    idx = _one_layer_index(oracle, X, 5)
    res = oracle.search(idx, Q, k=6, ef=12)
    rng = np.random.default_rng(0)
    for i in range(len(Q)):
        W = _flagged_w_search(X, idx.members[0], idx.adj[0], Q[i], 0, 12, rng, vis_slots)
        got = [int(idx.members[0][w[1]]) for w in W[:6]]
        assert got == res.ids[i].tolist()


def test_counters_and_margins(oracle):
    X = wl.uniform(500, 4, 12)
    X[7] = X[3]          # an exact duplicate forces a zero-margin decision
    Q = np.repeat(X[3:4] + 1e-3, 4, axis=0)
    idx = oracle.build_index(X, oracle.BuildParams(degree=8))
    res = oracle.search(idx, Q, k=5, ef=16)
    assert oracle.near_tie(res).all()
    assert (res.counters[:, 0] >= 1).all()
    assert (res.counters[:, 1] >= res.counters[:, 0]).all()
    assert (res.counters[:, 2] <= res.counters[:, 0]).all()


# ------------------------------------------------- brute force, recall ----

@pytest.mark.parametrize("metric", [0, 1])
def test_brute_force_knn_matches_numpy(oracle, metric):
    X = wl.uniform(400, 7, 13) - 0.5
    Q = wl.uniform(30, 7, 14) - 0.5
    ids, dist = oracle.brute_force_knn(X, Q, 12, metric)
    Xd, Qd = X.astype(np.float64), Q.astype(np.float64)
    D = ((Qd[:, None, :] - Xd[None, :, :]) ** 2).sum(-1) if metric == 0 else -(Qd @ Xd.T)
    for i in range(len(Q)):
        ref = np.lexsort((np.arange(400), D[i]))[:12]
        assert np.array_equal(ids[i], ref)
        assert np.allclose(dist[i], D[i][ref], rtol=1e-12, atol=1e-12)


def test_brute_force_pads_when_k_exceeds_n(oracle):
    X = wl.uniform(3, 2, 1)
    ids, dist = oracle.brute_force_knn(X, X[:1], 5)
    assert ids[0, 0] == 0 and (ids[0, 3:] == -1).all() and np.isinf(dist[0, 3:]).all()


def test_recall_tie_tolerant(oracle):
    X = np.array([[0, 0], [1, 0], [0, 1], [3, 3]], dtype=np.float32)
    Q = np.array([[0, 0]], dtype=np.float32)
    _, td = oracle.brute_force_knn(X, Q, 2)
    # ids 1 and 2 tie at distance 1: either one completes the top-2
    assert oracle.recall_at_k(np.array([[0, 2]]), td, X, Q) == 1.0
    assert oracle.recall_at_k(np.array([[0, 1]]), td, X, Q) == 1.0
    assert oracle.recall_at_k(np.array([[0, 3]]), td, X, Q) == 0.5
    assert oracle.recall_at_k(np.array([[-1, 3]]), td, X, Q) == 0.0


# ------------------------------------------- kNN_SYM and complete root ----

@pytest.mark.parametrize("metric", [0, 1])
def test_knn_sym_matches_numpy(oracle, metric):
    X = wl.uniform(240, 6, 15) - 0.5
    members = np.arange(240, dtype=np.int32)[::2].copy()
    R, M = 5, 9
    Y = X[members].astype(np.float64)
    D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1) if metric == 0 else -(Y @ Y.T)
    s = len(members)
    knn = []
    for v in range(s):
        dv = D[v].copy()
        dv[v] = np.inf
        knn.append(np.lexsort((np.arange(s), dv))[:R])
    adj, _, _, _ = oracle.knn_graph(X, metric, members, R)
    assert np.array_equal(adj, np.array(knn))
    sym, cut, order = oracle.knn_sym(X, metric, members, adj, M)
    for v in range(s):
        cand = set(knn[v].tolist()) | {u for u in range(s) if v in knn[u]}
        cand = np.array(sorted(cand))
        ref = cand[np.lexsort((cand, D[v][cand]))][:M]
        row = sym[v][sym[v] >= 0]
        assert np.array_equal(row, ref), v
        assert (sym[v][len(ref):] == -1).all()


def test_complete_root_hands_down_exact_root_nn(oracle):
    """With the complete graph on the root, greedy search there returns the
    root member nearest to q; the descent continues from it (Alg. 4)."""
    X = wl.uniform(5000, 4, 16)
    Q = wl.uniform(30, 4, 17)
    p = oracle.BuildParams(degree=8, root_complete_max=400)
    idx = oracle.build_index(X, p)
    assert idx.root_complete and len(idx.members[-1]) <= 400
    assert len(idx.members[-2]) > 400
    res = oracle.search(idx, Q, k=1, ef=1, ef_upper=1)
    top = idx.members[-1]
    for i in range(len(Q)):
        dq = np.array([d64_seq(Q[i], X[u]) for u in top])
        v = int(top[np.lexsort((top, dq))[0]])
        for lay in range(idx.num_layers - 2, -1, -1):
            v = _greedy_alg4(X, idx.members[lay], idx.adj[lay], Q[i], v)
        assert res.ids[i, 0] == v
    # counters: the root scan evaluates every root member
    assert (res.counters[:, 1] >= len(top)).all()


def test_root_complete_stops_layer_loop(oracle):
    X = wl.uniform(3000, 32, 0)
    members, _ = oracle.build_layers(X, oracle.BuildParams(degree=8, root_complete_max=5000))
    assert len(members) == 1
    members, _ = oracle.build_layers(X, oracle.BuildParams(degree=8, root_complete_max=200))
    assert len(members[-1]) <= 200 and len(members[-2]) > 200


# ---------------------------------------------------------------- pruning ---

def _line_points(n, d, seed):
    """n distinct points on a line in R^d with irregular gaps."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.uniform(0.5, 2.0, size=n))
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    return (t[:, None] * u[None, :]).astype(np.float32), t


def test_prune_on_a_line_keeps_the_nearest_on_each_side(oracle):
    """On a line a farther candidate on the same side as a kept one is closer
    to that kept point than to v, so exactly the two nearest neighbours (one
    per side; one at the ends) survive."""
    X, t = _line_points(60, 8, 3)
    members = np.arange(60, dtype=np.int32)
    cand, _, _, _ = oracle.knn_graph(X, oracle.L2, members, 16)
    out, pm = oracle.prune(X, oracle.L2, members, cand, 16)
    order = np.argsort(t)
    rank = np.empty(60, dtype=int)
    rank[order] = np.arange(60)
    for v in range(60):
        r = rank[v]
        expect = set()
        if r > 0:
            expect.add(int(order[r - 1]))
        if r < 59:
            expect.add(int(order[r + 1]))
        got = [int(x) for x in out[v] if x >= 0]
        assert set(got) == expect, (v, got, expect)
        assert got[0] == cand[v][0]  # the nearest candidate is always kept
    assert np.all(pm > 1e-6)


def test_prune_keeps_orthogonal_candidates(oracle):
    """Candidates on distinct orthogonal axes around v are farther from each
    other than from v (r_i^2 + r_j^2 > r_i^2), so none is dropped."""
    d = 12
    radii = np.linspace(1.0, 2.1, d)
    pts = [np.zeros(d)]
    for i in range(d):
        e = np.zeros(d)
        e[i] = radii[i]
        pts.append(e)
    X = np.array(pts, dtype=np.float32)
    members = np.arange(d + 1, dtype=np.int32)
    cand, _, _, _ = oracle.knn_graph(X, oracle.L2, members, d)
    out, _ = oracle.prune(X, oracle.L2, members, cand, d)
    assert np.array_equal(out[0], cand[0])
    out4, _ = oracle.prune(X, oracle.L2, members, cand, 4)
    assert np.array_equal(out4[0], cand[0][:4])  # the cap keeps the first four


@pytest.mark.parametrize("metric", [0, 1])
def test_pruned_graph_invariants(oracle, metric):
    """Pruned rows are ordered subsequences of the candidate lists, start with
    the nearest candidate, never repeat or list the row itself, and every
    dropped candidate has a kept one strictly closer to it than the row is
    (checked in FP64 with NumPy)."""
    X = wl.uniform(400, 6, 11) - 0.5
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    members = np.arange(400, dtype=np.int32)
    C = oracle.prune_candidates(8)
    cand, _, _, _ = oracle.knn_graph(X, metric, members, C)
    out, pm = oracle.prune(X, metric, members, cand, 8)
    X64 = X.astype(np.float64)

    def dist(a, b):
        return float(((X64[a] - X64[b]) ** 2).sum()) if metric == 0 else -float(X64[a] @ X64[b])

    for v in range(400):
        kept = [int(x) for x in out[v] if x >= 0]
        cl = [int(x) for x in cand[v] if x >= 0]
        assert kept[0] == cl[0] and v not in kept and len(set(kept)) == len(kept)
        pos = [cl.index(k) for k in kept]
        assert pos == sorted(pos)
        last = pos[-1] if len(kept) == 8 else len(cl) - 1
        for j in range(last + 1):
            c = cl[j]
            if c in kept:
                continue
            earlier = [k for k in kept if cl.index(k) < j]
            assert any(dist(c, k) < dist(c, v) for k in earlier), (v, c)


def test_pruned_sym_rows_are_out_plus_in_neighbours(oracle):
    """PRUNED_SYM rows: the pruned out-list plus only nodes whose pruned list
    holds the row, deduplicated, sorted by (distance, id), at most max_degree."""
    X = wl.uniform(500, 5, 12)
    members = np.arange(500, dtype=np.int32)
    cand, _, _, _ = oracle.knn_graph(X, oracle.L2, members, oracle.prune_candidates(6))
    pr, _ = oracle.prune(X, oracle.L2, members, cand, 6)
    sym, _, _ = oracle.knn_sym(X, oracle.L2, members, pr, 20)
    X64 = X.astype(np.float64)
    ins = {v: set() for v in range(500)}
    for u in range(500):
        for x in pr[u]:
            if x >= 0:
                ins[int(x)].add(u)
    for v in range(500):
        row = [int(x) for x in sym[v] if x >= 0]
        out = {int(x) for x in pr[v] if x >= 0}
        assert len(row) == len(set(row)) <= 20
        assert set(row) <= out | ins[v]
        if len(out | ins[v]) <= 20:
            assert set(row) == out | ins[v]
        dd = [float(((X64[v] - X64[u]) ** 2).sum()) for u in row]
        assert all(dd[i] <= dd[i + 1] for i in range(len(dd) - 1))
    idx = oracle.build_index(X, oracle.BuildParams(degree=6, graph=3, max_degree=20))
    assert np.array_equal(idx.adj[0], sym)


@pytest.mark.parametrize("metric,n,d,k", [(0, 3000, 16, 10), (1, 2500, 24, 7), (0, 40, 8, 30)])
def test_gram_brute_force_equals_plain_brute_force(oracle, metric, n, d, k):
    """The matrix-product route to exact k-NN returns the plain brute force's
    ids and distances (bit for bit: both sum each distance in coordinate
    order), also when k exceeds half the points (no shortlist)."""
    X = wl.gauss_mix(n, d, 8, 0.3, 28)
    Q = wl.gauss_mix(60, d, 8, 0.3, 29)
    if metric == 1:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    a_i, a_d = oracle.brute_force_knn(X, Q, k, metric)
    b_i, b_d = oracle.brute_force_knn_gram(X, Q, k, metric, chunk=16)
    assert np.array_equal(a_i, b_i)
    assert np.array_equal(a_d, b_d)

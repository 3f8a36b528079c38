"""Pins of the oracle's near-tie recorder, one per decisive comparison.

The parity rule exempts a query from the id check when its oracle trace holds
a decision between two distinct ids whose distances lie within a small
relative margin (the FP32 error bound).  These tests plant exactly one such
near tie at one kind of decision in a hand-built trace and check that the
recorded margin is that pair's margin, computed here from the definition
(|d_a - d_b| / max(|d_a|, |d_b|) for L2; |d_a - d_b| / (|q| max(|a|, |b|))
for inner product), and that a planted tie no decision compares is not
recorded.  The decisions (the beam of Sec. 2.2 as HNSW's SEARCH-LAYER, and
Alg. 4 above it):

* admission: a candidate against the worst entry of a full list;
* eviction: the evicted entry against the new worst;
* next expansion: the expanded candidate against the one that follows it;
* the stop test: the expanded candidate against the worst entry;
* the complete-graph root (App. B.2): its best member against the second;
* the returned list: adjacent entries of the top k and the k / k+1 cut.

Each trace is a one-dimensional layer with query 0, so every distance is the
exact square of a float32 coordinate and every comparison is known in
advance.  A tie is planted by moving a coordinate by a few ulps.
"""
import numpy as np
import pytest

TOL = 3e-6          # the exemption threshold the GPU parity tests use
DX = 2.0 ** -22     # planted offset: a relative distance gap of ~1e-6 near x = 0.3 .. 0.5


def _l2(x):
    x = float(np.float32(x))
    return x * x


def _margin_l2(xa, xb):
    a, b = _l2(xa), _l2(xb)
    return abs(a - b) / max(abs(a), abs(b), 1e-30)


def _run(oracle, xs, nbrs, k, ef, root=None, metric=0, q=0.0, adj_margin=None):
    """Search a hand-built layer (adjacency lists by position) with one query."""
    X = np.array(xs, dtype=np.float32).reshape(-1, 1)
    n = len(xs)
    deg = 4
    adj = np.full((n, deg), -1, np.int32)
    for v, row in nbrs.items():
        adj[v, :len(row)] = row
    members, adjs = [np.arange(n, dtype=np.int32)], [adj]
    if root is not None:
        members.append(np.array(sorted(root), dtype=np.int32))
        adjs.append(np.full((len(root), deg), -1, np.int32))
    idx = oracle.index_from_arrays(X, metric, members, adjs, root_complete=root is not None)
    if adj_margin is not None:
        idx.adj_margin = [np.asarray(adj_margin, dtype=np.float64)] + \
            [np.full(len(m), np.inf) for m in members[1:]]
    return oracle.search(idx, np.array([[q]], np.float32), k, ef)


def test_admission_against_the_worst_of_a_full_list(oracle):
    # e (0.5) expands to a (0.2), which fills the list (ef = 2), then t (0.5 + dx),
    # which only the admission test compares with the worst kept entry, e
    res = _run(oracle, [0.5, 0.2, 0.5 + DX], {0: [1, 2]}, k=1, ef=2)
    assert res.ids[0, 0] == 1
    assert res.margin[0] == _margin_l2(0.5, 0.5 + DX) <= TOL
    assert oracle.near_tie(res, TOL)[0]


def test_eviction_against_the_new_worst(oracle):
    # A (0.5 + dx) joins a list of two; u1 (0.2) evicts A, leaving e (0.5) the
    # worst; u2 (0.1) then evicts e.  A is popped last and stopped against u1.
    res = _run(oracle, [0.5, 0.5 + DX, 0.2, 0.1], {0: [1, 2, 3]}, k=1, ef=2)
    assert res.ids[0, 0] == 3
    assert res.margin[0] == _margin_l2(0.5 + DX, 0.5) <= TOL


def test_next_expansion_against_the_following_candidate(oracle):
    # z (0.1), c1 (0.3) and c2 (0.3 + dx) enter a wide list together; after z,
    # c1 is expanded before c2 -- the only decision between the two
    res = _run(oracle, [0.5, 0.1, 0.3, 0.3 + DX], {0: [1, 2, 3]}, k=1, ef=8)
    assert res.ids[0, 0] == 1
    assert res.margin[0] == _margin_l2(0.3, 0.3 + DX) <= TOL


def test_stop_test_against_the_worst_entry(oracle):
    # m (0.3 + dx) is expanded before c (0.3) is found; c is then popped while
    # m is the list's worst entry
    res = _run(oracle, [0.1, 0.3 + DX, 0.3], {0: [1], 1: [2]}, k=1, ef=8)
    assert res.ids[0, 0] == 0
    assert res.margin[0] == _margin_l2(0.3, 0.3 + DX) <= TOL


def test_complete_root_best_against_second(oracle):
    # the root {1, 2, 3} is scanned exhaustively; 1 and 2 nearly tie
    res = _run(oracle, [0.1, 0.3, 0.3 + DX, 0.9], {1: [0]}, k=1, ef=8, root=[1, 2, 3])
    assert res.ids[0, 0] == 0
    assert res.margin[0] == _margin_l2(0.3, 0.3 + DX) <= TOL


@pytest.mark.parametrize("k,flagged", [(3, True), (2, True), (1, False)])
def test_returned_list_adjacency_and_cut(oracle, k, flagged):
    # a chain e (0.1) -> a (0.3) -> b (0.3 + dx): a and b are never compared
    # during the search; they are entries 2 and 3 of the returned list, so the
    # tie is inside the top k (k = 3), at the k / k+1 cut (k = 2) or beyond
    # the cut (k = 1, not a decision)
    res = _run(oracle, [0.1, 0.3, 0.3 + DX], {0: [1], 1: [2]}, k=k, ef=8)
    assert res.ids[0].tolist() == [0, 1, 2][:k]
    if flagged:
        assert res.margin[0] == _margin_l2(0.3, 0.3 + DX) <= TOL
    else:
        assert res.margin[0] == _margin_l2(0.1, 0.3) > 0.5
    assert oracle.near_tie(res, TOL)[0] == flagged


def test_inner_product_margin_is_scaled_by_the_norms(oracle):
    # -<q, x> with q = 2: the margin divides by |q| * max(|a|, |b|)
    xa, xb = 0.9, 0.9 - 2.0 ** -21
    res = _run(oracle, [0.1, xa, xb], {0: [1], 1: [2]}, k=2, ef=8, metric=1, q=2.0)
    assert res.ids[0].tolist() == [1, 2]
    da = -(2.0 * float(np.float32(xa)))
    db = -(2.0 * float(np.float32(xb)))
    want = abs(da - db) / (2.0 * max(abs(float(np.float32(xa))), abs(float(np.float32(xb)))))
    assert res.margin[0] == want <= TOL


def test_tie_between_two_rejected_candidates_is_not_a_decision(oracle):
    # y (0.9) and z (0.9 + dx) are both rejected against the full list's
    # worst entry e; nothing compares them with each other
    res = _run(oracle, [0.5, 0.2, 0.9, 0.9 + DX], {0: [1, 2, 3]}, k=1, ef=2)
    assert res.ids[0, 0] == 1
    assert res.margin[0] > 0.5
    assert not oracle.near_tie(res, TOL)[0]


def test_adjacency_margin_of_expanded_nodes_only(oracle):
    # the trace of the admission test expands e and a, and evaluates t without
    # expanding it: a near tie at t's R / R+1 cut cannot change the search
    xs, nbrs = [0.5, 0.2, 0.5 + 0.1], {0: [1, 2]}
    res = _run(oracle, xs, nbrs, k=1, ef=2, adj_margin=[np.inf, 1e-7, np.inf])
    assert res.adj_margin[0] == 1e-7 and oracle.near_tie(res, TOL)[0]
    res = _run(oracle, xs, nbrs, k=1, ef=2, adj_margin=[np.inf, np.inf, 1e-7])
    assert res.adj_margin[0] == np.inf and not oracle.near_tie(res, TOL)[0]

"""Shared helpers of the GPU parity tests (comparison against the oracle)."""
import math

import numpy as np

TOL = 1e-5  # relative tolerance on returned distances


def exempt_tol(d):
    """Relative decision margin below which FP32 can order two distances
    differently from FP64, for d-dimensional rows.

    The library's FP32 distance rounds q - x once (two units on the square),
    sums each chunk of 8 coordinates with 8 sequential FMAs and adds the chunk
    sums by a pairwise tree over P = next_pow2(ceil(d / 8)) leaves: a relative
    error of at most E = (2 + 8 + log2 P) 2^-24 for squared L2 (all terms are
    positive), and at most (8 + log2 P) 2^-24 |q||x| for inner products.  Two
    distances can only compare differently from FP64 when their relative gap is
    at most 2E, so the exemption threshold is 2E with a 10% allowance: 1.57e-6
    at d = 32, 1.84e-6 at d = 128, 2.23e-6 at d = 768 -- all tighter than the
    specification's 1e-5 (it checks more queries, never fewer)."""
    chunks = -(-int(d) // 8)
    P = 1
    while P < chunks:
        P *= 2
    return 2.2 * (10 + math.log2(P)) * 2.0 ** -24


# kept for the graph-build tests that compare rows at the d = 32 workload
STRICT = exempt_tol(32)


def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def dist_tol(ores_dist, X, Q, ids, metric):
    """Per-entry absolute tolerance: 1e-5 relative (L2) or 1e-5 * |q||x| (IP)."""
    if metric == 0:
        return TOL * np.maximum(np.abs(ores_dist), 1e-30)
    qn = np.linalg.norm(Q.astype(np.float64), axis=1)[:, None]
    xn = np.linalg.norm(X.astype(np.float64)[np.maximum(ids, 0)], axis=2)
    return TOL * qn * xn + 1e-30


def exempt_mask(ores, d, graph_margins=False):
    """Queries exempt from the id check: the oracle trace holds a decision
    within exempt_tol(d); with graph_margins, also an expanded node whose
    graph row was decided that close (only where the GPU searched a graph it
    built itself, not the oracle's)."""
    tol = exempt_tol(d)
    ex = ores.margin <= tol
    if graph_margins:
        ex = ex | (ores.adj_margin <= tol)
    return ex


def assert_search_parity(gids, gdist, ores, X, Q, metric=0, max_exempt=None, k=None,
                         graph_margins=False):
    """Ids bit-exact and distances within 1e-5 relative for every query whose
    oracle trace holds no decision within the FP32 error bound exempt_tol(d);
    exempt queries are counted, printed with the cap, and returned.
    max_exempt is the largest exempt fraction the test allows: about 1.5x the
    oracle's own rate on that test's inputs, so that a near-tie recorder that
    exempts too much fails."""
    k = k or ores.ids.shape[1]
    gids = np.asarray(gids)[:, :k]
    gdist = np.asarray(gdist)[:, :k]
    exempt = exempt_mask(ores, X.shape[1], graph_margins)
    ok = ~exempt
    bad = np.where(ok & ~(gids == ores.ids).all(1))[0]
    assert bad.size == 0, (f"{bad.size} non-exempt queries differ, first {bad[:5]}: "
                           f"gpu {gids[bad[0]]} oracle {ores.ids[bad[0]]}")
    valid = ores.ids >= 0
    tol = dist_tol(ores.dist, X, Q, ores.ids, metric)
    err = np.where(valid, np.abs(gdist.astype(np.float64) - np.where(valid, ores.dist, 0)), 0)
    assert (err[ok] <= tol[ok]).all(), f"distance error {np.max(err[ok] / tol[ok])} x tol"
    assert np.isinf(gdist[~valid & ok[:, None]]).all()
    if max_exempt is not None:
        print(f"exempt {exempt.mean():.4f} of {exempt.size} (cap {max_exempt}, "
              f"tol {exempt_tol(X.shape[1]):.3g})")
        assert exempt.mean() <= max_exempt, f"exempt fraction {exempt.mean():.4f}"
    return exempt


def assert_results_valid(gids, gdist, X, Q, metric=0):
    """Every returned id's FP64 distance matches its returned distance, the
    rows are sorted by (distance, id) and hold no duplicates."""
    from oracle import henn_oracle as ho
    gids = np.asarray(gids)
    gdist = np.asarray(gdist)
    for i in range(gids.shape[0]):
        row = [int(u) for u in gids[i] if u >= 0]
        assert len(set(row)) == len(row)
        ds = [ho.distance(Q[i], X[u], metric) for u in row]
        for j, u in enumerate(row):
            tol = TOL * max(abs(ds[j]), 1e-30) if metric == 0 else TOL * float(
                np.linalg.norm(Q[i]) * np.linalg.norm(X[u])) + 1e-30
            assert abs(float(gdist[i, j]) - ds[j]) <= tol
        keys = list(zip(gdist[i, :len(row)].tolist(), row))
        assert keys == sorted(keys)

"""The worst-case study's recall-bound arithmetic (Sec. 3 definition of
rho_delta; App. G.4 "Average Hits"), checked on the CPU against hand-worked
cases and a brute-force restatement of the definition."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
bench = pytest.importorskip("bench")


def test_hits_curve_and_recall_bound_hand_case():
    # ten searches whose results have these ranks among all points
    ranks = [3, 1, 2, 5, 1, 4, 1, 2, 9, 1]
    assert np.allclose(bench.hits_curve(ranks, 6), [0.4, 0.6, 0.7, 0.8, 0.9, 0.9])
    assert bench.recall_bound(ranks, 0.9) == 5
    assert bench.recall_bound(ranks, 0.4) == 1
    assert bench.recall_bound(ranks, 0.41) == 2
    assert bench.recall_bound(ranks, 1.0) == 9
    # 90 exact hits out of 100: rho_0.9 = 1; one fewer: the next rank
    assert bench.recall_bound([1] * 90 + [7] * 10, 0.9) == 1
    assert bench.recall_bound([1] * 89 + [7] * 11, 0.9) == 7


def test_recall_bound_is_the_smallest_k_reaching_delta():
    rng = np.random.default_rng(0)
    for _ in range(50):
        r = rng.geometric(rng.uniform(0.05, 0.9), size=int(rng.integers(1, 400)))
        for delta in (0.5, 0.9, 0.99):
            kmax = int(r.max())
            want = next(k for k in range(1, kmax + 1) if np.mean(r <= k) >= delta)
            assert bench.recall_bound(r, delta) == want
            assert bench.hits_curve(r, kmax)[want - 1] >= delta


def test_ranks_of_counts_strictly_closer_points():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 5)).astype(np.float32)
    Q = rng.standard_normal((40, 5)).astype(np.float32)
    got = rng.integers(0, 300, size=40)
    r = bench.ranks_of(torch.from_numpy(X), torch.from_numpy(Q), got)
    X64, Q64 = X.astype(np.float64), Q.astype(np.float64)
    for i in range(40):
        d = ((X64 - Q64[i]) ** 2).sum(1)
        assert r[i] == 1 + int((d < d[got[i]]).sum())
    # the nearest point has rank 1
    nn = np.array([int(np.argmin(((X64 - q) ** 2).sum(1))) for q in Q64])
    assert (bench.ranks_of(torch.from_numpy(X), torch.from_numpy(Q), nn) == 1).all()

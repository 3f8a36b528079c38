"""The named workloads draw what their names say."""
import numpy as np

import workloads as wl


def test_named_workloads_use_their_own_generators():
    X, Q = wl.make("gmm1000_10M_d128", n=3000, nq=50)
    assert np.array_equal(X, wl.gauss_mix(3000, 128, 1000, 0.25, 0))
    assert np.array_equal(Q, wl.gauss_mix(50, 128, 1000, 0.25, 1))
    X, Q = wl.make("gmm100_1M_d128", n=3000, nq=50)
    assert np.array_equal(X, wl.gauss_mix(3000, 128, 100, 0.3, 0))
    X, Q = wl.make("uniform_10k_d32")
    assert X.shape == (10000, 32) and Q.shape == (1000, 32)
    assert np.array_equal(X, wl.uniform(10000, 32, 0))
    X, Q = wl.make("curve_1M_d96", n=4000, nq=20)
    assert X.shape == (4000, 96) and Q.shape == (20, 96)
    X, Q = wl.make("spectral_5M_d768", n=100, nq=10)
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, atol=1e-5)


def test_mixture_cluster_count():
    # 1,000 distinct centres for the 1,000-cluster family
    X = wl.gauss_mix(20000, 16, 1000, 1e-6, 0)
    assert len(np.unique(np.round(X[:, :3], 4), axis=0)) >= 995


def test_mixed_requests_and_arrivals():
    k, ef = wl.mixed_requests(3000)
    assert set(k.tolist()) == {1, 10, 100} and set(ef.tolist()) == {32, 64, 128}
    t = wl.poisson_arrivals(20000, 1000.0)
    assert np.all(np.diff(t) > 0) and abs(20000 / t[-1] - 1000.0) < 50.0

"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method: it only draws points,
queries and per-request parameters.  Both the oracle's tests and the HIP
path's tests/benchmark take their inputs from here.

Generators (``np.random.default_rng(seed)``; big arrays are drawn in chunks
of 2**20 rows, labels first and then noise within each chunk):

* ``uniform``    -- i.i.d. U[0,1]^d points (the 10,000 x 32 parity workload).
* ``gauss_mix``  -- Gaussian mixture: centres N(0, I) from seed 2, equal
  weights, isotropic sigma (1M x 128 with 100 clusters, sigma 0.3, stands in
  for the shape of the SIFT benchmark used in Sec. 4: 1M x 128, 10k queries;
  10M x 128 with 1,000 clusters, sigma 0.25, for the batched form).
* ``curve``      -- points along a random smooth curve with exponentially
  shrinking gaps 0.5^(i mod 40), embedded by a random orthonormal map plus
  N(0, 1e-4) noise, queries near the dense end of each period (the skewed,
  adversarial regime of Sec. 4.2).
* ``spectral``   -- anisotropic Gaussian with power-law spectrum
  lambda_i = i^-0.8 in a random orthonormal basis, unit-normalised
  (embedding-like vectors for inner-product search).
* ``expskew``    -- exponential coordinates with a per-point scale: point i
  draws v_i ~ U(0,1) and coordinates Exp(1) / lam^v_i.  lam = 1 is i.i.d.
  Exp(1) data; a larger lam spreads the point scales over a factor lam, so
  the density varies by up to lam^d between the dense core and the sparse
  outskirts (the skewed synthetic data of Sec. 4.2 with an explicit skew
  parameter: i.i.d. Exp(lam) coordinates would only rescale the data).
"""
from __future__ import annotations

import numpy as np

CHUNK = 1 << 20


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random((n, d), dtype=np.float32)


def gauss_mix(n: int, d: int, clusters: int, sigma: float, seed: int,
              centre_seed: int = 2) -> np.ndarray:
    centres = np.random.default_rng(centre_seed).standard_normal((clusters, d))
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float32)
    for b in range(0, n, CHUNK):
        e = min(n, b + CHUNK)
        lab = rng.integers(0, clusters, size=e - b)
        noise = rng.standard_normal((e - b, d))
        out[b:e] = (centres[lab] + sigma * noise).astype(np.float32)
    return out


def _orthonormal(d: int, seed: int) -> np.ndarray:
    a = np.random.default_rng(seed).standard_normal((d, d))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def _curve_params(d: int, seed: int = 2):
    half = d // 2
    rng = np.random.default_rng(seed + 1000)
    omega = 2 * np.pi / rng.uniform(100.0, 1000.0, size=half)
    phase = rng.uniform(0.0, 2 * np.pi, size=half)
    rho = 1.0 / (np.sqrt(half) * omega)
    return omega, phase, rho


def _curve_points(t: np.ndarray, d: int, omega, phase, rho) -> np.ndarray:
    ang = np.outer(t, omega) + phase[None, :]
    g = np.empty((t.shape[0], d))
    g[:, 0::2] = rho * np.cos(ang)
    g[:, 1::2] = rho * np.sin(ang)
    return g


def curve_times(n: int, period: int = 40) -> np.ndarray:
    gaps = 0.5 ** (np.arange(n) % period)
    t = np.zeros(n)
    t[1:] = np.cumsum(gaps[:-1])
    return t


def curve(n: int, d: int, seed: int, noise_var: float = 1e-4, period: int = 40):
    """Points X_i = M gamma(t_i) + N(0, noise_var I); gamma has unit speed."""
    omega, phase, rho = _curve_params(d)
    M = _orthonormal(d, 2)
    t = curve_times(n, period)
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float32)
    sd = np.sqrt(noise_var)
    for b in range(0, n, CHUNK):
        e = min(n, b + CHUNK)
        g = _curve_points(t[b:e], d, omega, phase, rho) @ M.T
        out[b:e] = (g + sd * rng.standard_normal((e - b, d))).astype(np.float32)
    return out


def curve_queries(nq: int, n: int, d: int, seed: int, noise_var: float = 1e-4,
                  period: int = 40):
    """Queries near the dense end (last point) of uniformly drawn periods."""
    omega, phase, rho = _curve_params(d)
    M = _orthonormal(d, 2)
    t = curve_times(n, period)
    rng = np.random.default_rng(seed)
    nper = n // period
    p = rng.integers(0, nper, size=nq)
    tt = t[period * p + period - 1]
    g = _curve_points(tt, d, omega, phase, rho) @ M.T
    return (g + np.sqrt(noise_var) * rng.standard_normal((nq, d))).astype(np.float32)


def spectral(n: int, d: int, seed: int, alpha: float = 0.8, basis_seed: int = 2):
    lam = np.arange(1, d + 1, dtype=np.float64) ** (-alpha)
    M = _orthonormal(d, basis_seed)
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float32)
    for b in range(0, n, CHUNK):
        e = min(n, b + CHUNK)
        z = rng.standard_normal((e - b, d)) * np.sqrt(lam)[None, :]
        x = z @ M.T
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[b:e] = x.astype(np.float32)
    return out


def expskew(n: int, d: int, lam: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty((n, d), dtype=np.float32)
    for b in range(0, n, CHUNK):
        e = min(n, b + CHUNK)
        v = rng.random(e - b)
        coords = rng.standard_exponential((e - b, d))
        out[b:e] = (coords / np.power(float(lam), v)[:, None]).astype(np.float32)
    return out


def mixed_requests(nq: int, k_choices=(1, 10, 100), ef_choices=(32, 64, 128),
                   k_seed: int = 3, ef_seed: int = 4):
    k = np.asarray(k_choices, dtype=np.int32)[np.random.default_rng(k_seed).integers(
        0, len(k_choices), size=nq)]
    ef = np.asarray(ef_choices, dtype=np.int32)[np.random.default_rng(ef_seed).integers(
        0, len(ef_choices), size=nq)]
    return k, ef


def poisson_arrivals(nq: int, rate_qps: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_qps, size=nq)
    return np.cumsum(gaps)


# The five workloads, by name: (points, queries, metric, k, ef)
WORKLOADS = {
    "uniform_10k_d32": dict(n=10_000, d=32, nq=1_000, metric="l2", k=10, ef=32),
    "gmm100_1M_d128": dict(n=1_000_000, d=128, nq=10_000, metric="l2", k=10, ef=64),
    "curve_1M_d96": dict(n=1_000_000, d=96, nq=10_000, metric="l2", k=10, ef=64),
    "gmm1000_10M_d128": dict(n=10_000_000, d=128, nq=100_000, metric="l2", k=10, ef=64),
    "spectral_5M_d768": dict(n=5_000_000, d=768, nq=10_000, metric="ip", k=10, ef=128),
}


def make(name: str, n: int | None = None, nq: int | None = None):
    """Points and queries of a named workload, optionally with fewer rows."""
    w = WORKLOADS[name]
    n = n or w["n"]
    nq = nq or w["nq"]
    d = w["d"]
    family = name.split("_")[0]
    if family == "uniform":
        return uniform(n, d, 0), uniform(nq, d, 1)
    if family == "gmm100":
        return gauss_mix(n, d, 100, 0.3, 0), gauss_mix(nq, d, 100, 0.3, 1)
    if family == "gmm1000":
        return gauss_mix(n, d, 1000, 0.25, 0), gauss_mix(nq, d, 1000, 0.25, 1)
    if family == "curve":
        return curve(n, d, 0), curve_queries(nq, n, d, 1)
    if family == "spectral":
        return spectral(n, d, 0), spectral(nq, d, 1)
    raise KeyError(name)

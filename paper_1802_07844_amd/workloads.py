"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers: it holds none of the summation method's
arithmetic.  Every generator takes a seed and returns float64 numpy arrays, so
the GPU path and the oracle see bit-identical inputs.

The paper's workloads are random point sets in a box with random strengths
(Sec. 6: uniform points in an L^3 box, strengths and orientations U[-1, 1]).
The named workloads below follow the shapes of the benchmark configurations:

* ``uniform_stokeslet``: x1, x2 ~ U[0, 1), x3 = 1 - U[0, 1) in (0, 1], forces
  i.i.d. N(0, 1) per component.
* ``uniform_stresslet``: same positions; strength g ~ N(0, 1)^3 and orientation
  q a unit normal uniform on the sphere (normalised Gaussian); strengths are
  returned as (g, q), N x 6.
* ``uniform_rotlet``: same positions; torque v ~ N(0, 1)^3.
* ``clustered_stokeslet``: x1, x2 ~ U[0, 1), x3 = min(Exp(mean 0.05), 1),
  zeros redrawn; forces N(0, 1).
* ``serving_stream``: Poisson arrivals, N log-uniform in [1e3, 1e6], kernel
  uniform over the three, tolerance uniform over {1e-5, 1e-10}.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1802


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_positions(g: np.random.Generator, n: int) -> np.ndarray:
    y = np.empty((n, 3), dtype=np.float64)
    y[:, 0] = g.random(n)
    y[:, 1] = g.random(n)
    y[:, 2] = 1.0 - g.random(n)  # (0, 1]: strictly above the wall
    return y


def uniform_stokeslet(n: int, seed: int):
    g = rng(seed)
    y = uniform_positions(g, n)
    f = g.standard_normal((n, 3))
    return y, f


def unit_normals(g: np.random.Generator, n: int) -> np.ndarray:
    q = g.standard_normal((n, 3))
    nq = np.linalg.norm(q, axis=1, keepdims=True)
    while np.any(nq == 0.0):  # measure-zero event, redraw for safety
        bad = (nq[:, 0] == 0.0)
        q[bad] = g.standard_normal((int(bad.sum()), 3))
        nq = np.linalg.norm(q, axis=1, keepdims=True)
    return q / nq


def uniform_stresslet(n: int, seed: int):
    g = rng(seed)
    y = uniform_positions(g, n)
    gs = g.standard_normal((n, 3))
    q = unit_normals(g, n)
    return y, np.concatenate([gs, q], axis=1)


def uniform_rotlet(n: int, seed: int):
    g = rng(seed)
    y = uniform_positions(g, n)
    v = g.standard_normal((n, 3))
    return y, v


def clustered_positions(g: np.random.Generator, n: int, mean: float = 0.05) -> np.ndarray:
    y = np.empty((n, 3), dtype=np.float64)
    y[:, 0] = g.random(n)
    y[:, 1] = g.random(n)
    z = g.exponential(mean, n)
    bad = z <= 0.0
    while np.any(bad):
        z[bad] = g.exponential(mean, int(bad.sum()))
        bad = z <= 0.0
    y[:, 2] = np.minimum(z, 1.0)
    return y


def clustered_stokeslet(n: int, seed: int):
    g = rng(seed)
    y = clustered_positions(g, n)
    f = g.standard_normal((n, 3))
    return y, f


def make(kernel: str, n: int, seed: int, layout: str = "uniform"):
    """Positions and strengths for one kernel (stresslet: (g, q); rotlet: torque)."""
    if layout == "clustered":
        if kernel != "stokeslet":
            g = rng(seed)
            y = clustered_positions(g, n)
            if kernel == "stresslet":
                return y, np.concatenate([g.standard_normal((n, 3)), unit_normals(g, n)], axis=1)
            return y, g.standard_normal((n, 3))
        return clustered_stokeslet(n, seed)
    if kernel == "stokeslet":
        return uniform_stokeslet(n, seed)
    if kernel == "stresslet":
        return uniform_stresslet(n, seed)
    if kernel == "rotlet":
        return uniform_rotlet(n, seed)
    raise ValueError(kernel)


def serving_pool(n: int, seed: int):
    """Input pool for a serving stream: uniform positions with stokeslet forces,
    stresslet (g, q) and rotlet torques for each point.  A request of size N
    takes rows [o, o + N) of the pool (a uniform sample itself)."""
    g = rng(seed)
    y = uniform_positions(g, n)
    f = g.standard_normal((n, 3))
    gq = np.concatenate([g.standard_normal((n, 3)), unit_normals(g, n)], axis=1)
    v = g.standard_normal((n, 3))
    return y, f, gq, v


def serving_stream(n_requests: int, seed: int, n_min: float = 1e3, n_max: float = 1e6):
    """Request descriptors: (kernel, N, tol, data seed) in arrival order.

    Inter-arrival times are returned in units of the mean (rate 1); the caller
    rescales them to the chosen arrival rate.
    """
    g = rng(seed)
    kernels = ("stokeslet", "stresslet", "rotlet")
    gaps = g.exponential(1.0, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    logn = g.uniform(np.log10(n_min), np.log10(n_max), n_requests)
    ns = np.round(10.0 ** logn).astype(np.int64)
    ks = g.integers(0, 3, n_requests)
    tols = np.where(g.integers(0, 2, n_requests) == 0, 1e-5, 1e-10)
    seeds = g.integers(1, 2**31 - 1, n_requests)
    return [
        dict(arrival=float(arrivals[i]), kernel=kernels[int(ks[i])], n=int(ns[i]), tol=float(tols[i]),
             seed=int(seeds[i]))
        for i in range(n_requests)
    ]

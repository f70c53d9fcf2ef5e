"""Seeded synthetic integration problems.

This module only draws inputs: integrand parameters, the two interpolation
tables and the run settings.  It holds none of the method's arithmetic, so
both the GPU path and the CPU oracle can be fed from it.

A problem is a plain dict with the keys ``integrand`` ("const",
"gauss_product", "corner_peak" or "gauss_tables"), ``params`` (float64),
``tables`` (float64 of 2*256*256, or None), ``dim``, ``lo``, ``hi``,
``maxcalls``, ``nbins``, ``itmax``, ``ita``, ``alpha``, ``tau_rel``,
``seed`` (the sampling seed, separate from the parameter seed) and
``precision`` ("fp64", or "fp32" for FP32 evaluation with FP64 accumulation),
``one_d`` (True: the m-Cubes1D variant, one grid shared by all axes) and
``chi2_max`` (bound on chi^2/dof for convergence; 0 selects the default).

Parameter layouts:
  const          [v]
  gauss_product  [c_1..c_d, w_1..w_d]   f = exp(-sum ((x_j - c_j)/w_j)^2)
  corner_peak    [a_1..a_d]             f = (1 + sum a_j x_j)^-(d+1)
  gauss_tables   [c_1..c_d, w_1..w_d]   f = gauss_product * T1(x_1,x_2) * T2(x_3,x_4)
"""
from __future__ import annotations

import numpy as np

TABLE_N = 256


def _problem(integrand, params, dim, maxcalls, nbins, itmax, *, tables=None, lo=None, hi=None,
             ita=None, alpha=1.5, tau_rel=0.0, seed=0, precision="fp64", one_d=False, chi2_max=0.0,
             device_steps=False):
    return {
        "integrand": integrand,
        "params": np.ascontiguousarray(params, dtype=np.float64),
        "tables": None if tables is None else np.ascontiguousarray(tables, dtype=np.float64).ravel(),
        "dim": int(dim),
        "lo": np.zeros(dim) if lo is None else np.ascontiguousarray(lo, dtype=np.float64),
        "hi": np.ones(dim) if hi is None else np.ascontiguousarray(hi, dtype=np.float64),
        "maxcalls": int(maxcalls),
        "nbins": int(nbins),
        "itmax": int(itmax),
        "ita": int(itmax if ita is None else ita),
        "alpha": float(alpha),
        "tau_rel": float(tau_rel),
        "seed": int(seed),
        "precision": precision,
        "one_d": bool(one_d),
        "chi2_max": float(chi2_max),
        "device_steps": bool(device_steps),
    }


def smooth_tables(rng: np.random.Generator, n_tables: int = 2, n_waves: int = 8) -> np.ndarray:
    """Positive smooth 256x256 tables: sums of random 2-D cosines, shifted up.

    T(u, v) = 1 + sum|A_q| + sum_q A_q cos(2 pi (a_q u + b_q v) + phi_q) at the
    nodes u = a/255, v = b/255, with A ~ U(0,1), a, b ~ U(0,3), phi ~ U(0, 2 pi);
    every node value is at least 1."""
    nodes = np.arange(TABLE_N) / (TABLE_N - 1.0)
    U, V = np.meshgrid(nodes, nodes, indexing="ij")
    out = np.empty((n_tables, TABLE_N, TABLE_N))
    for k in range(n_tables):
        A = rng.uniform(0.0, 1.0, n_waves)
        fa = rng.uniform(0.0, 3.0, n_waves)
        fb = rng.uniform(0.0, 3.0, n_waves)
        ph = rng.uniform(0.0, 2.0 * np.pi, n_waves)
        T = np.full_like(U, 1.0 + np.abs(A).sum())
        for q in range(n_waves):
            T += A[q] * np.cos(2.0 * np.pi * (fa[q] * U + fb[q] * V) + ph[q])
        out[k] = T
    return out


def const(dim=2, value=1.0, maxcalls=8192, nbins=128, itmax=3, **kw):
    return _problem("const", [value], dim, maxcalls, nbins, itmax, **kw)


def gauss_product(dim, rng_seed, c_range=(0.3, 0.7), w_range=(0.05, 0.2), maxcalls=10_000,
                  nbins=100, itmax=10, **kw):
    rng = np.random.default_rng(rng_seed)
    c = rng.uniform(*c_range, dim)
    w = rng.uniform(*w_range, dim)
    return _problem("gauss_product", np.concatenate([c, w]), dim, maxcalls, nbins, itmax, **kw)


def corner_peak(dim, rng_seed, a_range=(0.5, 2.0), maxcalls=10_000, nbins=100, itmax=10, **kw):
    rng = np.random.default_rng(rng_seed)
    a = rng.uniform(*a_range, dim)
    return _problem("corner_peak", a, dim, maxcalls, nbins, itmax, **kw)


def gauss_tables(dim, rng_seed, c_range=(0.2, 0.8), w_range=(0.02, 0.1), maxcalls=10_000,
                 nbins=100, itmax=10, **kw):
    if dim < 4:
        raise ValueError("gauss_tables needs dim >= 4")
    rng = np.random.default_rng(rng_seed)
    c = rng.uniform(*c_range, dim)
    w = rng.uniform(*w_range, dim)
    tables = smooth_tables(rng)
    return _problem("gauss_tables", np.concatenate([c, w]), dim, maxcalls, nbins, itmax,
                    tables=tables, **kw)


def symmetric_gauss(dim, c=0.5, w=0.1, maxcalls=10_000, nbins=100, itmax=10, **kw):
    """A fully symmetric Gaussian product: the same centre and width on every axis."""
    return _problem("gauss_product", np.concatenate([np.full(dim, c), np.full(dim, w)]), dim,
                    maxcalls, nbins, itmax, **kw)


def symmetric_corner(dim, a=1.0, maxcalls=10_000, nbins=100, itmax=10, **kw):
    """A fully symmetric corner peak: the same coefficient on every axis."""
    return _problem("corner_peak", np.full(dim, a), dim, maxcalls, nbins, itmax, **kw)


# ---- the benchmark configurations ------------------------------------------------------------

def config_small(seed=1, rng_seed=2202):
    """d=2 product of two Gaussians on [0,1]^2, 1e4 samples/iteration, 100 bins, 10 iterations."""
    return gauss_product(2, rng_seed, (0.3, 0.7), (0.05, 0.2), maxcalls=10_000, nbins=100,
                         itmax=10, alpha=1.5, seed=seed)


def config_tables(seed=1, rng_seed=1753, maxcalls=100_000_000, itmax=15, **kw):
    """d=6 Gaussian peaks times two bilinear 256x256 tables, 1e8 samples/iteration, 500 bins."""
    return gauss_tables(6, rng_seed, (0.2, 0.8), (0.02, 0.1), maxcalls=maxcalls, nbins=500,
                        itmax=itmax, alpha=1.5, seed=seed, **kw)


def config_corner8(seed=1, rng_seed=8, maxcalls=1_000_000_000, itmax=20, **kw):
    """d=8 corner peak with a_i ~ U(0.5, 2), 1e9 samples/iteration, 500 bins."""
    return corner_peak(8, rng_seed, (0.5, 2.0), maxcalls=maxcalls, nbins=500, itmax=itmax,
                       alpha=1.5, seed=seed, **kw)


def config_symmetric8(seed=1, maxcalls=1_000_000_000, itmax=20, **kw):
    """d=8 corner peak with one coefficient a = 1 on every axis (symmetric in all
    variables, the m-Cubes1D case), 1e9 samples/iteration, 500 bins."""
    return symmetric_corner(8, a=1.0, maxcalls=maxcalls, nbins=500, itmax=itmax, alpha=1.5, seed=seed,
                            **kw)


def config_gauss8(seed=1, rng_seed=88, maxcalls=1_000_000_000, itmax=20, **kw):
    """d=8 narrow Gaussian product (w = 0.01), 1e9 samples/iteration, 500 bins."""
    rng = np.random.default_rng(rng_seed)
    c = rng.uniform(0.3, 0.7, 8)
    w = np.full(8, 0.01)
    return _problem("gauss_product", np.concatenate([c, w]), 8, maxcalls, 500, itmax, alpha=1.5,
                    seed=seed, **kw)


def config_batch(n=4096, seed=4096, itmax=10, precision="fp64"):
    """n independent integrals: d ~ U{2..10}; Gaussian product (c ~ U(0.3,0.7),
    w ~ U(0.05,0.2)) or corner peak (a ~ U(0.5,2)) with probability 1/2 each;
    samples per iteration log-uniform on [1e4, 1e7]; nb ~ U{100..500}; each
    with its own parameter and sampling seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        d = int(rng.integers(2, 11))
        N = int(10 ** rng.uniform(4.0, 7.0))
        nb = int(rng.integers(100, 501))
        sub = int(rng.integers(0, 2**31))
        kw = dict(maxcalls=N, nbins=nb, itmax=itmax, alpha=1.5, seed=1 + i, precision=precision)
        if rng.random() < 0.5:
            out.append(gauss_product(d, sub, (0.3, 0.7), (0.05, 0.2), **kw))
        else:
            out.append(corner_peak(d, sub, (0.5, 2.0), **kw))
    return out


def served_requests(n=2000, rate=2000.0, seed=2000, precision="fp64", itmax=50):
    """A seeded Poisson stream of integration requests (mean `rate` per
    second): arrival times (s) and problems.  d ~ U{3..10}; target relative
    error log-uniform on [1e-5, 1e-2]; Gaussian product (the small
    configuration's ranges) or, for d >= 4 with probability 1/2, Gaussian
    peaks times two tables (the table configuration's ranges); samples per
    iteration 1e5 for targets >= 1e-3, 1e6 down to 1e-4, 1e7 below; 100
    bins; at most `itmax` iterations."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for i in range(n):
        d = int(rng.integers(3, 11))
        tau = float(10 ** rng.uniform(-5.0, -2.0))
        N = 100_000 if tau >= 1e-3 else (1_000_000 if tau >= 1e-4 else 10_000_000)
        sub = int(rng.integers(0, 2**31))
        kw = dict(maxcalls=N, nbins=100, itmax=itmax, alpha=1.5, seed=1 + i, tau_rel=tau,
                  precision=precision)
        if d >= 4 and rng.random() < 0.5:
            out.append(gauss_tables(d, sub, (0.2, 0.8), (0.02, 0.1), **kw))
        else:
            out.append(gauss_product(d, sub, (0.3, 0.7), (0.05, 0.2), **kw))
    return arrivals, out

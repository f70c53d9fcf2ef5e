"""Exact values of the test integrals, from the mathematics alone.

These pin the oracle: none of them calls it or repeats its arithmetic.
  * Gaussian product: each factor integrates to (w sqrt(pi)/2)(erf((H-c)/w) - erf((L-c)/w)).
  * Corner peak on the unit cube: (1/(d! prod a_j)) sum over subsets S of
    (-1)^|S| / (1 + sum_{j in S} a_j), evaluated in exact rationals.
  * Gaussian times bilinear tables: a bilinear interpolant is sum_ab T_ab phi_a(x) phi_b(y)
    with tent functions phi, so the integral is Phi_1^T T Phi_2 with
    Phi_a = integral of phi_a times the Gaussian factor, in closed form (erf, exp).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def gauss_factor(c, w, lo=0.0, hi=1.0):
    c, w, lo, hi = (mp.mpf(float(v)) for v in (c, w, lo, hi))
    return w * mp.sqrt(mp.pi) / 2 * (mp.erf((hi - c) / w) - mp.erf((lo - c) / w))


def gauss_product(params, d, lo=None, hi=None):
    lo = np.zeros(d) if lo is None else lo
    hi = np.ones(d) if hi is None else hi
    out = mp.mpf(1)
    for j in range(d):
        out *= gauss_factor(params[j], params[d + j], lo[j], hi[j])
    return float(out)


def corner_peak(a):
    """Integral over [0,1]^d of (1 + sum a_j x_j)^-(d+1), exactly, for the given doubles a."""
    d = len(a)
    A = [Fraction(float(v)) for v in a]
    total = Fraction(0)
    for r in range(d + 1):
        for S in itertools.combinations(range(d), r):
            total += Fraction((-1) ** r) / (1 + sum(A[j] for j in S))
    prod = Fraction(1)
    for v in A:
        prod *= v
    return float(total / (math.factorial(d) * prod))


def _tent_gauss_weights(c, w, n=256):
    """Phi_a = integral over [0,1] of tent_a(x) exp(-((x-c)/w)^2), nodes a/(n-1)."""
    c, w = mp.mpf(float(c)), mp.mpf(float(w))
    h = mp.mpf(1) / (n - 1)

    def G(x):  # antiderivative of the Gaussian
        return w * mp.sqrt(mp.pi) / 2 * mp.erf((x - c) / w)

    def H(x):  # antiderivative of (x - c) times the Gaussian
        return -(w * w) / 2 * mp.exp(-((x - c) / w) ** 2)

    out = np.zeros(n)
    for a in range(n):
        xa = a * h
        val = mp.mpf(0)
        if a > 0:  # rising half on [x_{a-1}, x_a]: (x - x_{a-1})/h
            p, q = xa - h, xa
            val += ((H(q) - H(p)) + (c - p) * (G(q) - G(p))) / h
        if a < n - 1:  # falling half on [x_a, x_{a+1}]: (x_{a+1} - x)/h
            p, q = xa, xa + h
            val += ((q - c) * (G(q) - G(p)) - (H(q) - H(p))) / h
        out[a] = float(val)
    return out


def gauss_tables(params, tables, d):
    """Integral over [0,1]^d of the Gaussian product times T1(x1,x2) T2(x3,x4)."""
    c, w = params[:d], params[d:]
    T = np.asarray(tables, dtype=np.float64).reshape(2, 256, 256)
    phi = [_tent_gauss_weights(c[j], w[j]) for j in range(4)]
    first = phi[0] @ T[0] @ phi[1]
    second = phi[2] @ T[1] @ phi[3]
    rest = 1.0
    for j in range(4, d):
        rest *= float(gauss_factor(c[j], w[j]))
    return float(first * second * rest)


def exact(prob):
    d = prob["dim"]
    kind = prob["integrand"]
    lo, hi = prob["lo"], prob["hi"]
    if kind == "const":
        return float(prob["params"][0] * np.prod(hi - lo))
    if kind == "gauss_product":
        return gauss_product(prob["params"], d, lo, hi)
    if kind == "corner_peak":
        assert np.all(lo == 0) and np.all(hi == 1)
        return corner_peak(prob["params"])
    if kind == "gauss_tables":
        assert np.all(lo == 0) and np.all(hi == 1)
        return gauss_tables(prob["params"], prob["tables"], d)
    raise ValueError(kind)

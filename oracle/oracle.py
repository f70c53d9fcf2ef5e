"""Python binding of the m-Cubes VEGAS oracle (``mcubes_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the product path never
imports it.  It imports nothing from the GPU package.

A problem is a plain dict with the keys ``integrand`` (one of "const",
"gauss_product", "corner_peak", "gauss_tables"), ``params``, ``tables``
(or None), ``dim``, ``lo``, ``hi``, ``maxcalls``, ``nbins``, ``itmax``,
``ita``, ``alpha``, ``tau_rel``, ``seed`` and optionally ``precision``
("fp64", the default, or "fp32" for FP32 evaluation with FP64 accumulation),
``one_d`` (True for the m-Cubes1D variant) and ``chi2_max`` (the bound on
chi^2/dof of the convergence check: 0, the default, means 5; negative, none).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "mcubes_oracle.c")
LIBRARY = os.path.join(HERE, "libmcubes_oracle.so")

INTEGRANDS = {"const": 0, "gauss_product": 1, "corner_peak": 2, "gauss_tables": 3}
OK, EINVAL, ENONFINITE = 0, 1, 3


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [
        ("integrand", C.c_int32),
        ("params", C.POINTER(C.c_double)),
        ("tables", C.POINTER(C.c_double)),
        ("dim", C.c_int32),
        ("lo", C.POINTER(C.c_double)),
        ("hi", C.POINTER(C.c_double)),
        ("maxcalls", C.c_int64),
        ("nbins", C.c_int32),
        ("itmax", C.c_int32),
        ("ita", C.c_int32),
        ("alpha", C.c_double),
        ("tau_rel", C.c_double),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("one_d", C.c_int32),
        ("chi2_max", C.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction) next to its source."""
    if force or not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
        tmp = LIBRARY + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-o", tmp, SOURCE, "-lm"],
            check=True,
        )
        os.replace(tmp, LIBRARY)
    return LIBRARY


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build()
        L = C.CDLL(LIBRARY)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_philox4x32_10.restype = None
        L.orc_uniform64.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_uniform64.restype = C.c_double
        L.orc_uniform24.argtypes = [C.c_uint32]
        L.orc_uniform24.restype = C.c_float
        L.orc_shape.argtypes = [C.c_int32, C.c_int64] + [C.POINTER(C.c_int64)] * 3
        L.orc_shape.restype = C.c_int
        L.orc_integrand.argtypes = [C.POINTER(_Problem), dp]
        L.orc_integrand.restype = C.c_double
        L.orc_integrand_many.argtypes = [C.POINTER(_Problem), C.c_int64, dp, dp]
        L.orc_integrand_many.restype = None
        L.orc_map.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp, C.POINTER(C.c_int64)]
        L.orc_map.restype = C.c_double
        L.orc_vsample.argtypes = [C.POINTER(_Problem), C.c_uint32, dp, C.c_int64, C.c_int64,
                                  dp, dp, dp, dp, dp]
        L.orc_vsample.restype = C.c_int
        L.orc_init_grid.argtypes = [C.c_int32, C.c_int32, dp]
        L.orc_init_grid.restype = None
        L.orc_refine.argtypes = [C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_refine.restype = None
        L.orc_refine_1d.argtypes = [C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_refine_1d.restype = None
        L.orc_weighted.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.orc_weighted.restype = None
        L.orc_integrate.argtypes = [C.POINTER(_Problem), dp, C.POINTER(C.c_int64), dp, dp, dp]
        L.orc_integrate.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class _Bound:
    """Keeps the numpy buffers a _Problem points into alive."""

    def __init__(self, prob: dict):
        self.params = _f64(prob["params"])
        self.tables = _f64(prob.get("tables"))
        self.lo = _f64(prob["lo"])
        self.hi = _f64(prob["hi"])
        self.s = _Problem(
            INTEGRANDS[prob["integrand"]], _dp(self.params), _dp(self.tables), int(prob["dim"]),
            _dp(self.lo), _dp(self.hi), int(prob["maxcalls"]), int(prob["nbins"]),
            int(prob["itmax"]), int(prob.get("ita", prob["itmax"])), float(prob["alpha"]),
            float(prob.get("tau_rel", 0.0)), int(prob["seed"]) & (2**64 - 1),
            1 if prob.get("precision", "fp64") == "fp32" else 0,
            1 if prob.get("one_d", False) else 0, float(prob.get("chi2_max", 0.0)))


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def uniform64(whi: int, wlo: int) -> float:
    return lib().orc_uniform64(whi & 0xFFFFFFFF, wlo & 0xFFFFFFFF)


def uniform24(w: int) -> float:
    return lib().orc_uniform24(w & 0xFFFFFFFF)


def shape(d: int, maxcalls: int):
    g, m, p = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_shape(d, maxcalls, C.byref(g), C.byref(m), C.byref(p))
    if rc:
        raise OracleError(rc)
    return g.value, m.value, p.value


def integrand(prob: dict, x) -> float:
    b = _Bound(prob)
    xx = _f64(x)
    return lib().orc_integrand(C.byref(b.s), _dp(xx))


def integrand_many(prob: dict, xs) -> np.ndarray:
    """The integrand at each row of xs (n x d)."""
    b = _Bound(prob)
    xs = _f64(xs)
    n = xs.shape[0]
    out = np.zeros(n)
    lib().orc_integrand_many(C.byref(b.s), n, _dp(xs), _dp(out))
    return out


def map_point(nb: int, grid, lo, hi, y):
    """VEGAS map of y in (0,1)^d: returns (x, bins, J)."""
    grid, lo, hi, y = _f64(grid), _f64(lo), _f64(hi), _f64(y)
    d = len(lo)
    x = np.zeros(d)
    bins = np.zeros(d, dtype=np.int64)
    J = lib().orc_map(d, nb, _dp(grid), _dp(lo), _dp(hi), _dp(y), _dp(x),
                      bins.ctypes.data_as(C.POINTER(C.c_int64)))
    return x, bins, J


def init_grid(d: int, nb: int):
    g = np.zeros(d * (nb + 1))
    lib().orc_init_grid(d, nb, _dp(g))
    return g


def vsample(prob: dict, it: int, grid, t0: int = 0, t1: int | None = None, hist: bool = True,
            trace: bool = False, check: bool = True):
    """One V-Sample pass over sub-cubes [t0, t1).

    Returns a dict with I, var, hist (d*nb or None), strace ((t1-t0)*p x (3d+2)
    or None), ctrace ((t1-t0) x 2 or None) and status."""
    b = _Bound(prob)
    d, nb = int(prob["dim"]), int(prob["nbins"])
    g, m, p = shape(d, int(prob["maxcalls"]))
    t1 = m if t1 is None else t1
    grid = _f64(grid)
    I, V = C.c_double(), C.c_double()
    h = np.zeros(d * nb) if hist else None
    n = t1 - t0
    st = np.zeros((n * p, 3 * d + 2)) if trace else None
    ct = np.zeros((n, 2)) if trace else None
    rc = lib().orc_vsample(C.byref(b.s), it, _dp(grid), t0, t1, C.byref(I), C.byref(V), _dp(h),
                           _dp(st), _dp(ct))
    if check and rc:
        raise OracleError(rc)
    return {"I": I.value, "var": V.value, "hist": h, "strace": st, "ctrace": ct, "status": rc}


def refine(d: int, nb: int, alpha: float, hist, grid):
    out = _f64(grid).copy()
    h = _f64(hist)
    lib().orc_refine(d, nb, alpha, _dp(h), _dp(out))
    return out


def refine_1d(d: int, nb: int, alpha: float, hist, grid):
    """m-Cubes1D adjustment: axis 0 from its contributions, copied to every axis."""
    out = _f64(grid).copy()
    h = _f64(hist)
    lib().orc_refine_1d(d, nb, alpha, _dp(h), _dp(out))
    return out


def weighted(I, var):
    I, var = _f64(I), _f64(var)
    a, s, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_weighted(len(I), _dp(I), _dp(var), C.byref(a), C.byref(s), C.byref(c))
    return a.value, s.value, c.value


def integrate(prob: dict, check: bool = True):
    b = _Bound(prob)
    d, nb, itmax = int(prob["dim"]), int(prob["nbins"]), int(prob["itmax"])
    res = np.zeros(3)
    ires = np.zeros(3, dtype=np.int64)
    Is, Vs = np.zeros(itmax), np.zeros(itmax)
    grid = np.zeros(d * (nb + 1))
    rc = lib().orc_integrate(C.byref(b.s), _dp(res), ires.ctypes.data_as(C.POINTER(C.c_int64)),
                             _dp(Is), _dp(Vs), _dp(grid))
    if check and rc:
        raise OracleError(rc)
    k = int(ires[0])
    return {"estimate": res[0], "error": res[1], "chi2_dof": res[2], "iterations": k,
            "converged": bool(ires[1]), "calls": int(ires[2]), "it_I": Is[:k], "it_var": Vs[:k],
            "grid": grid, "status": rc}

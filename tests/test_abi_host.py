"""Host-side checks of libmcubes that need no GPU: the library loads and
exports every entry point of include/mcubes.h, validation rejects bad
problems before any device work, and the host steps of Alg. 2 (lattice,
Init-Bins, Adjust-Bin-Bounds, Weighted-Estimates) agree bit for bit with the
oracle's independent implementation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2202_01753_amd import mcubes as M
from paper_2202_01753_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mcubes.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|mc_status)\s*(mc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 9
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(M.EXPORTS) == names


def test_status_strings():
    for code in range(5):
        assert M.status_string(code)
    assert M.status_string(99) == "unknown status"


@pytest.mark.parametrize("d,N", [(2, 10_000), (6, 10**8), (8, 10**9), (8, 2 * 12**8), (10, 10**4),
                                 (10, 10**7), (2, 10**7), (1, 4), (16, 2**40), (3, 10**9 + 7)])
def test_shape_matches_oracle(d, N):
    assert M.shape(d, N) == O.shape(d, N)


def test_shape_rejects():
    for d, N in [(0, 100), (17, 100), (2, 3)]:
        with pytest.raises(M.MCubesError) as e:
            M.shape(d, N)
        assert e.value.code == M.EINVAL


def test_init_grid_matches_oracle():
    for d, nb in [(1, 2), (3, 100), (6, 500), (16, 7)]:
        assert np.array_equal(M.init_grid(d, nb), O.init_grid(d, nb))


@pytest.mark.parametrize("seed", range(6))
def test_refine_matches_oracle_bit_for_bit(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 9))
    nb = int(rng.integers(2, 600))
    alpha = float(rng.uniform(0.2, 2.5))
    grid = O.init_grid(d, nb)
    for _ in range(4):  # a few successive refinements from peaked histograms
        hist = rng.gamma(0.3, size=d * nb) ** 3
        hist[rng.random(d * nb) < 0.1] = 0.0
        a = M.refine_grid(d, nb, alpha, hist, grid)
        b = O.refine(d, nb, alpha, hist, grid)
        assert np.array_equal(a, b)
        grid = a
    # degenerate rows
    hist = np.zeros(d * nb)
    assert np.array_equal(M.refine_grid(d, nb, alpha, hist, grid), grid)


def test_weighted_matches_oracle_bit_for_bit():
    rng = np.random.default_rng(3)
    for k in range(1, 30):
        I = rng.normal(1.0, 0.01, k)
        V = rng.uniform(1e-6, 1e-4, k)
        a = M.weighted_estimate(I, V)
        b = O.weighted(I, V)
        assert a[:2] == b[:2]
        assert (np.isnan(a[2]) and np.isnan(b[2])) or a[2] == b[2]
    V[3] = 0.0
    assert M.weighted_estimate(I, V) == O.weighted(I, V)
    # iterations without information (I = 0 and var = 0) are left out alike
    for I, V in [([0.0, 3.0, 5.0], [0.0, 1.0, 1.0]), ([0.0, 2.0], [0.0, 0.5]),
                 ([0.0, 0.0, 0.0], [0.0, 0.0, 0.0]), ([0.0, 2.5, 1.5], [0.0, 0.0, 2.0])]:
        a, b = M.weighted_estimate(I, V), O.weighted(I, V)
        assert a[:2] == b[:2]
        assert (np.isnan(a[2]) and np.isnan(b[2])) or a[2] == b[2]


def _bad_problems():
    good = W.config_small()
    cases = []
    for key, val in [("dim", 0), ("dim", 17), ("nbins", 1), ("maxcalls", 3), ("itmax", 0),
                     ("ita", 11), ("ita", -1), ("alpha", 0.0), ("alpha", float("nan")),
                     ("tau_rel", -1.0)]:
        p = dict(good)
        p[key] = val
        cases.append((f"{key}={val}", p, {}))
    p = dict(good)
    p["hi"] = np.array([1.0, 0.0])
    cases.append(("lo>=hi", p, {}))
    p = dict(good)
    p["lo"] = np.array([0.0, -np.inf])
    cases.append(("lo=-inf", p, {}))
    p = dict(good)
    p["params"] = good["params"][:3]
    cases.append(("n_params", p, {}))
    t = W.gauss_tables(4, 1)
    t["tables"] = t["tables"][:100]
    cases.append(("n_tables", t, {}))
    t = W.gauss_tables(4, 1)
    t["dim"] = 3
    t["params"] = t["params"][:6]
    t["lo"], t["hi"] = t["lo"][:3], t["hi"][:3]
    cases.append(("tables d<4", t, {}))
    big = W.gauss_product(16, 1, nbins=800)
    cases.append(("LDS over budget", big, {}))
    cases.append(("threads=96", good, {"threads": 96}))
    cases.append(("threads=2048", good, {"threads": 2048}))
    cases.append(("blocks<0", good, {"blocks": -1}))
    return cases


@pytest.mark.parametrize("name,prob,kw", _bad_problems(), ids=[c[0] for c in _bad_problems()])
def test_invalid_problems_rejected_before_device_work(name, prob, kw):
    bp = M.BoundProblem(prob, **kw)
    n = C.c_size_t(12345)
    code = M.lib().mc_workspace_bytes(bp.ref, C.byref(n))
    assert code == M.EINVAL
    assert n.value == 12345  # untouched on error
    res = M.Result(estimate=7.0)
    code = M.lib().mc_integrate(bp.ref, None, 0, None, C.byref(res), None, None, None)
    assert code == M.EINVAL and res.estimate == 7.0
    code = M.lib().mc_integrate_prepared(bp.ref, None, 0, None, C.byref(res), None, None, None)
    assert code == M.EINVAL and res.estimate == 7.0


def test_null_arguments_rejected():
    L = M.lib()
    assert L.mc_workspace_bytes(None, None) == M.EINVAL
    assert L.mc_integrate(None, None, 0, None, None, None, None, None) == M.EINVAL
    assert L.mc_refine_grid(2, 10, 1.5, None, None) == M.EINVAL
    assert L.mc_weighted_estimate(0, None, None, None) == M.EINVAL


def test_refine_1d_matches_oracle_bit_for_bit():
    rng = np.random.default_rng(11)
    for d, nb in [(2, 50), (6, 500), (10, 100)]:
        hist = rng.gamma(0.4, size=d * nb) ** 2
        grid = O.init_grid(d, nb)
        for _ in range(3):
            a = M.refine_grid_1d(d, nb, 1.5, hist, grid)
            assert np.array_equal(a, O.refine_1d(d, nb, 1.5, hist, grid))
            grid = a
        rows = grid.reshape(d, nb + 1)
        assert all(np.array_equal(rows[0], rows[j]) for j in range(d))


def test_header_is_plain_c_and_the_library_links_without_python(tmp_path):
    """A C99 program (-pedantic -Werror) includes include/mcubes.h, names every
    declared entry point, links straight against libmcubes.so and calls the
    host-only ones."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = os.path.join(ROOT, "tests", "pins", "abi_from_c.c")
    listed = set(re.findall(r"\(entry_fn\)(mc_\w+)", open(src).read()))
    assert listed == set(_declared())
    M.lib()  # built
    libdir = os.path.dirname(M.LIBRARY)
    exe = str(tmp_path / "abi_from_c")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    src, "-o", exe, f"-L{libdir}", "-l:libmcubes.so", f"-Wl,-rpath,{libdir}", "-lm"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
    assert "shape 19 47045881 2" in out.stdout

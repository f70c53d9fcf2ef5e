"""GPU parity: the HIP sampling path (through the C ABI) against the CPU oracle.

Bars (FP64 path):
  * sample points are bit-exact: uniforms, bin indices, points x and Jacobians J;
  * f is bit-exact for integrands built from basic IEEE operations (constant,
    corner peak); the exponential-based ones differ only by the libm/ocml exp
    rounding (a few ulp);
  * per-iteration estimate and variance agree within 1e-12 relative (the
    estimate relative to sum |I_t|), bin contributions within 1e-12 relative;
  * the grid refined from the GPU's histogram is identical bit for bit in the
    library and in the oracle (lockstep)."""
import math

import numpy as np
import pytest

import closed_forms as CF
import oracle as O
from paper_2202_01753_amd import mcubes as M
from paper_2202_01753_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _ulps(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    ia = np.where(ia < 0, np.int64(-2**63) - ia, ia)
    ib = np.where(ib < 0, np.int64(-2**63) - ib, ib)
    return np.abs(ia - ib)


def _exact_f(prob):
    return prob["integrand"] in ("const", "corner_peak")


def _fp32(prob):
    return prob.get("precision", "fp64") == "fp32"


def _ulps32(a, b):
    """Distance in float32 ulps of values that are exactly representable floats."""
    ia = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(2**31) - ia, ia)
    ib = np.where(ib < 0, -(2**31) - ib, ib)
    return np.abs(ia - ib)


def _tol(prob):
    """Relative tolerance on sums of I_k: order of summation only, unless f comes
    from an FP32 exponential (ocml and glibc expf may differ by an ulp, 2^-23)."""
    return 1e-6 if _fp32(prob) and not _exact_f(prob) else TOL


def _compare_records(prob, gpu, ref, label=""):
    d = prob["dim"]
    G, R = gpu["strace"], ref["strace"]
    assert G.shape == R.shape, label
    assert np.array_equal(G[:, :d], R[:, :d]), f"{label}: uniforms differ"
    assert np.array_equal(G[:, d:2 * d], R[:, d:2 * d]), f"{label}: bins differ"
    assert np.array_equal(G[:, 2 * d:3 * d], R[:, 2 * d:3 * d]), f"{label}: points differ"
    assert np.array_equal(G[:, 3 * d], R[:, 3 * d]), f"{label}: Jacobians differ"
    if _exact_f(prob):
        assert np.array_equal(G[:, 3 * d + 1], R[:, 3 * d + 1]), f"{label}: f differs"
    elif _fp32(prob):
        # expf rounding (ocml vs glibc) and two products; values far below the
        # smallest normal float (exp underflowing into subnormals, where an ulp
        # is 2^-149 absolute) only need to agree in absolute terms
        g, r = G[:, 3 * d + 1], R[:, 3 * d + 1]
        ok = (_ulps32(g, r) <= 8) | (np.maximum(np.abs(g), np.abs(r)) < 2.0**-120)
        assert ok.all(), f"{label}: f beyond 8 float ulp"
    else:
        # exp rounding (ocml vs glibc, each within a couple of ulp in the far tail)
        # followed by up to two products with the table values
        assert _ulps(G[:, 3 * d + 1], R[:, 3 * d + 1]).max() <= 8, f"{label}: f beyond 8 ulp"
    gc, rc = gpu["ctrace"], ref["ctrace"]
    scale = np.abs(rc[:, 0]).sum()
    if _exact_f(prob):
        assert np.array_equal(gc, rc), f"{label}: per-cube values differ"
    else:
        rel = 1e-6 if _fp32(prob) else 1e-14
        # cubes whose values are ~1e-15 of the largest one (integrand far in its
        # tail, where float exp is subnormal) only need to agree in absolute terms
        floor_i = 1e-15 * np.abs(rc[:, 0]).max() + 1e-300
        floor_v = 1e-15 * np.abs(rc[:, 1]).max() + 1e-300
        assert np.all(np.abs(gc[:, 0] - rc[:, 0]) <= rel * np.abs(rc[:, 0]) + floor_i)
        assert np.all(np.abs(gc[:, 1] - rc[:, 1]) <= 100 * rel * np.abs(rc[:, 1]) + rel * rc[:, 0] ** 2 + floor_v)
    return scale


def _compare_totals(gpu, ref, scale, label="", tol=TOL):
    assert abs(gpu["I"] - ref["I"]) <= tol * scale, f"{label}: I {gpu['I']} vs {ref['I']}"
    vtol = tol if tol == TOL else 100 * tol  # a variance of near-equal samples amplifies f's rounding
    assert abs(gpu["var"] - ref["var"]) <= vtol * abs(ref["var"]) + 1e-300, \
        f"{label}: var {gpu['var']} vs {ref['var']}"
    if ref["hist"] is not None:
        h, r = gpu["hist"], ref["hist"]
        # per axis, bins fed only by far-tail samples (1e-15 of the axis's
        # largest bin and below) only need to agree in absolute terms
        n_axes = len(r) // nbins if (nbins := gpu.get("nbins")) else 1
        rows = r.reshape(n_axes, -1)
        floor = np.repeat(1e-15 * rows.max(axis=1), rows.shape[1]) + 1e-300
        assert np.all(np.abs(h - r) <= tol * np.abs(r) + (floor if tol != TOL else 1e-300)), \
            f"{label}: histogram"


def _positive_scale(ref):
    """sum_t |I_t| for an integrand that is never negative (all the closed forms
    and the tables here): the pass total itself."""
    return abs(ref["I"])


def _refined_grids_agree(prob, gpu_hist, ref_hist, grid, gpu_grid, tol):
    """The grid the run goes on with (refined by the library from the GPU
    histogram) against the oracle's own refinement of the oracle's histogram.
    Bit-identical when the two histograms are.  When every bin agrees within
    tol relative, within 100 tol absolute: 1e-12 relative perturbations of
    these histograms move no boundary by more than 3e-13 (measured on the
    CPU).  Lepage's compression weighs a bin by about 1/ln(S/s_i), so a bin
    that is exactly 0 on one side and a tiny subnormal on the other (float
    expf of ocml and glibc differ there) can move boundaries by far more; that
    case arises only for FP32 exponentials and is not compared."""
    d, nb, alpha = prob["dim"], prob["nbins"], prob["alpha"]
    refine = O.refine_1d if prob.get("one_d") else O.refine
    want = refine(d, nb, alpha, ref_hist, grid)
    if np.array_equal(gpu_hist, ref_hist):
        assert np.array_equal(gpu_grid, want), "refined grids differ on equal histograms"
    elif np.all(np.abs(gpu_hist - ref_hist) <= tol * np.abs(ref_hist)):
        assert np.abs(gpu_grid - want).max() <= 100 * tol, "refined grids differ"
    else:
        assert _fp32(prob) and not _exact_f(prob), "histograms differ beyond rounding"


def _lockstep(prob, iters=None, threads=0, blocks=0):
    """Every iteration: the traced pass (same kernel template, tracing
    instantiation) against the oracle sample by sample, then the production
    pass that the benchmark times, untraced, against the same oracle pass;
    the run goes on with the grid refined from the production pass."""
    d, nb = prob["dim"], prob["nbins"]
    s = M.Sampler(prob, blocks=blocks, threads=threads)
    grid = O.init_grid(d, nb)
    iters = prob["itmax"] if iters is None else iters
    tol = _tol(prob)
    for it in range(iters):
        adjust = it < prob["ita"]
        gpu = s.sample(it, grid, adjust, trace_range=(0, s.m))
        gpu["nbins"] = nb
        ref = O.vsample(prob, it, grid, hist=adjust, trace=True)
        scale = _compare_records(prob, gpu, ref, f"iter {it}")
        _compare_totals(gpu, ref, scale, f"iter {it}", tol)
        prod = s.sample(it, grid, adjust)
        prod["nbins"] = nb
        _compare_totals(prod, ref, scale, f"iter {it} (production kernel)", tol)
        if adjust and prob.get("one_d"):
            a = M.refine_grid_1d(d, nb, prob["alpha"], prod["hist"], grid)
            b = O.refine_1d(d, nb, prob["alpha"], prod["hist"], grid)
            assert np.array_equal(a, b), f"iter {it}: refined grids differ"
            _refined_grids_agree(prob, prod["hist"], ref["hist"], grid, a, tol)
            grid = a
        elif adjust:
            a = M.refine_grid(d, nb, prob["alpha"], prod["hist"], grid)
            b = O.refine(d, nb, prob["alpha"], prod["hist"], grid)
            assert np.array_equal(a, b), f"iter {it}: refined grids differ"
            _refined_grids_agree(prob, prod["hist"], ref["hist"], grid, a, tol)
            grid = a
    return grid


# ---------------------------------------------------------------- lockstep, tiny runs

def test_lockstep_small_gaussian_config():
    _lockstep(W.config_small(seed=11))


def test_lockstep_corner_peak_bit_exact():
    _lockstep(W.corner_peak(3, 5, maxcalls=5000, nbins=40, itmax=4, seed=2**40 + 3))


def test_lockstep_tables_d6():
    _lockstep(W.config_tables(seed=7, maxcalls=30_000, itmax=3))


def test_lockstep_constant_exact():
    prob = W.const(2, 2.5, maxcalls=8192, nbins=128, itmax=2, lo=np.array([0.0, -1.0]),
                   hi=np.array([1.0, 3.0]), seed=9)
    s = M.Sampler(prob)
    r = s.sample(0, O.init_grid(2, 128), adjust=False)
    assert r["I"] == 10.0 and r["var"] == 0.0


@pytest.mark.parametrize("case", [
    dict(make=lambda: W.gauss_product(1, 3, maxcalls=4, nbins=2, itmax=3, seed=1), name="d1 m2"),
    dict(make=lambda: W.corner_peak(3, 4, maxcalls=1000, nbins=2, itmax=3, seed=5), name="ragged nb2"),
    dict(make=lambda: W.corner_peak(10, 6, maxcalls=10_000, nbins=64, itmax=3, seed=6), name="p9"),
    dict(make=lambda: W.corner_peak(16, 7, maxcalls=2**17, nbins=16, itmax=2, seed=8), name="d16"),
    dict(make=lambda: W.gauss_product(2, 9, maxcalls=20_000, nbins=4000, itmax=2, seed=4), name="nb4000"),
    dict(make=lambda: W.gauss_product(3, 10, maxcalls=6000, nbins=30, itmax=4, ita=2, seed=3,
                                      lo=np.array([-1.0, 0.5, 2.0]), hi=np.array([1.0, 0.75, 9.0])),
         name="bounds no-adjust"),
], ids=lambda c: c["name"])
def test_lockstep_edge_cases(case):
    _lockstep(case["make"]())


@pytest.mark.parametrize("threads,blocks", [(64, 1), (64, 7), (256, 0), (1024, 0), (512, 3), (768, 5)])
def test_launch_shape_does_not_change_samples(threads, blocks):
    prob = W.corner_peak(4, 12, maxcalls=40_000, nbins=50, itmax=2, seed=77)
    _lockstep(prob, threads=threads, blocks=blocks)


def test_default_launch_shape_follows_occupancy():
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # d = 8, nb = 500: 64 KB of LDS per workgroup, so two fit per CU, and two of
    # 768 threads keep more waves resident than one of 1024; the launch takes
    # four times the resident count where every lane still has 100 sub-cubes
    # to do, twice otherwise (or fewer if the cubes run out first)
    c8 = W.corner_peak(8, 8, maxcalls=20_000_000, nbins=500, itmax=1)
    g, m, p = O.shape(8, 20_000_000)
    assert m < 100 * 4 * (2 * cus) * 768
    r = M.integrate(c8, timing=True)
    assert (r.threads, r.lds_bytes) == (768, 64064)
    assert r.blocks == min(2 * 2 * cus, -(-m // 768))
    big = W.corner_peak(8, 8, maxcalls=1_000_000_000, nbins=500, itmax=1)
    g, m, p = O.shape(8, 1_000_000_000)
    assert m >= 100 * 4 * (2 * cus) * 768
    assert M.launch_shape(M.BoundProblem(big), adjust=True)[:2] == (4 * 2 * cus, 768)
    # the FP32-eval d = 6 tables kernel: two 72 KB workgroups of 768 threads
    # per CU, 13^6 sub-cubes at 1e7, launched twice over
    t32 = W.config_tables(maxcalls=10_000_000, itmax=1, precision="fp32")
    assert M.launch_shape(M.BoundProblem(t32), adjust=True)[:2] == (2 * 2 * cus, 768)
    # d = 6 tables: one 48 KB workgroup of 1024 threads per CU, launched once per CU
    t6 = W.config_tables(maxcalls=2_000_000, itmax=1)
    r6 = M.integrate(t6, timing=True)
    assert (r6.threads, r6.blocks) == (1024, cus)


# ---------------------------------------------------------------- whole runs

def test_integrate_matches_oracle_free_running():
    prob = W.config_small(seed=21)
    g = M.integrate(prob)
    o = O.integrate(prob)
    assert g.iterations == o["iterations"] == 10
    assert np.allclose(g.it_I, o["it_I"], rtol=1e-11, atol=0)
    assert np.allclose(g.it_var, o["it_var"], rtol=1e-10, atol=0)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)
    assert g.error == pytest.approx(o["error"], rel=1e-10)
    assert g.chi2_dof == pytest.approx(o["chi2_dof"], rel=1e-8)
    exact = CF.exact(prob)
    assert abs(g.estimate - exact) < 5 * g.error


def test_integrate_corner_peak_free_running_and_convergence():
    prob = W.corner_peak(5, 14, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=5)
    g = M.integrate(prob)
    o = O.integrate(prob)
    assert g.iterations == o["iterations"] and g.converged == o["converged"]
    assert g.converged and g.error <= 1e-3 * abs(g.estimate)
    assert np.allclose(g.it_I, o["it_I"], rtol=1e-11, atol=0)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)
    assert abs(g.estimate - CF.exact(prob)) < 5 * g.error


def test_deterministic_repeat():
    prob = W.config_tables(seed=3, maxcalls=2_000_000, itmax=1)
    s = M.Sampler(prob)
    grid = O.init_grid(6, 500)
    a = s.sample(0, grid)
    b = s.sample(0, grid)
    assert a["I"] == b["I"] and a["var"] == b["var"]
    assert np.allclose(a["hist"], b["hist"], rtol=TOL, atol=0)


def test_reentrant_on_two_streams():
    """Two integrations on two workspaces and two streams at once, from two
    host threads (ctypes releases the GIL during the calls), give the results
    each gives alone, to the histogram's rounding."""
    import threading

    import torch

    probs = [W.config_tables(seed=21, maxcalls=2_000_000, itmax=4),
             W.corner_peak(6, 3, maxcalls=3_000_000, nbins=200, itmax=5, seed=22)]
    alone = [M.integrate(p) for p in probs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]
    errors = []

    def run(i):
        try:
            out[i] = M.integrate(probs[i], stream=streams[i])
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors and all(not t.is_alive() for t in threads)
    for a, b in zip(out, alone):
        assert a.iterations == b.iterations
        assert a.estimate == pytest.approx(b.estimate, rel=TOL, abs=0)
        assert a.error == pytest.approx(b.error, rel=1e-9, abs=0)


def test_integrate_prepared_matches_integrate():
    """mc_integrate_prepared on a workspace filled once by mc_prepare gives
    mc_integrate's results run after run, for both precisions (to rounding:
    the LDS histogram atomics make bin sums, and so later grids, order-
    dependent in the last ulp)."""
    for precision in ("fp64", "fp32"):
        prob = W.config_tables(seed=8, maxcalls=1_000_000, itmax=4, precision=precision)
        bp = M.BoundProblem(prob)
        ws = M.Workspace(bp)
        M.prepare(prob, ws, bp=bp)
        for seed in (3, 4):
            prob["seed"] = bp.s.seed = seed
            a = M.integrate(prob, ws=ws, bp=bp, prepared=True)
            b = M.integrate(prob)
            assert a.iterations == b.iterations
            assert a.estimate == pytest.approx(b.estimate, rel=TOL, abs=0)
            assert a.error == pytest.approx(b.error, rel=1e-9, abs=0)
            assert np.allclose(a.grid, b.grid, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- full-size configurations

def _sampled_full_size(prob, windows, n=1500):
    s = M.Sampler(prob)
    d, nb = prob["dim"], prob["nbins"]
    rng = np.random.default_rng(1)
    grid = np.concatenate([np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
                           for _ in range(d)])
    full = None
    for frac in windows:
        t0 = min(int(frac * s.m), s.m - n)
        gpu = s.sample(1, grid, True, trace_range=(t0, t0 + n))
        ref = O.vsample(prob, 1, grid, t0=t0, t1=t0 + n, hist=False, trace=True)
        _compare_records(prob, gpu, ref, f"cubes [{t0}, {t0 + n})")
        full = gpu
    # properties of the whole pass: each axis row of the histogram sums to the
    # same total (every sample adds I_k^2 once per axis)
    rows = full["hist"].reshape(d, nb).sum(axis=1)
    assert np.allclose(rows, rows[0], rtol=1e-12)
    assert full["var"] > 0 and full["I"] > 0
    return s, full


def test_full_size_tables_1e8():
    prob = W.config_tables(seed=1)
    s, full = _sampled_full_size(prob, [0.0, 0.37, 1.0])
    # on the uniform grid the pass is an unbiased estimate of the closed form
    r = s.sample(0, O.init_grid(6, 500), adjust=False)
    exact = CF.exact(prob)
    assert abs(r["I"] - exact) < 5 * math.sqrt(r["var"])


def test_full_size_corner8_1e9():
    prob = W.config_corner8(seed=1)
    s, full = _sampled_full_size(prob, [0.0, 0.5, 1.0], n=800)
    r = s.sample(0, O.init_grid(8, 500), adjust=True)
    exact = CF.exact(prob)
    assert abs(r["I"] - exact) < 5 * math.sqrt(r["var"])


def test_counter_high_word():
    """More than 2^32 sub-cubes: the high word of the cube index enters the counter."""
    prob = W.gauss_product(2, 2, maxcalls=2**34, nbins=64, itmax=1, seed=3)
    s = M.Sampler(prob)
    assert s.m > 2**32
    grid = O.init_grid(2, 64)
    t0 = s.m - 1000
    gpu = s.sample(0, grid, False, trace_range=(t0, s.m))
    ref = O.vsample(prob, 0, grid, t0=t0, t1=s.m, hist=False, trace=True)
    _compare_records(prob, gpu, ref, "t >= 2^32")


# ---------------------------------------------------------------- error paths through the C ABI

def test_error_paths():
    import ctypes as C
    import torch
    prob = W.config_small()
    bp = M.BoundProblem(prob)
    need = M.workspace_bytes(bp)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    res = M.Result(estimate=-1.0)
    code = M.lib().mc_integrate(bp.ref, C.c_void_p(ws.data_ptr()), need - 1, None, C.byref(res),
                                None, None, None)
    assert code == M.EWORKSPACE and res.estimate == -1.0
    inf = W.const(2, np.inf, maxcalls=1000, nbins=10, itmax=2)
    with pytest.raises(M.MCubesError) as e:
        M.integrate(inf)
    assert e.value.code == M.ENONFINITE
    # a non-finite pass does not poison the next one on the same workspace
    s = M.Sampler(W.const(2, 1.0, maxcalls=8192, nbins=128, itmax=1))
    assert s.sample(0, O.init_grid(2, 128))["status"] == M.OK
    with pytest.raises(M.MCubesError) as e:
        s.sample(0, O.init_grid(2, 128), adjust=False, trace_range=(0, s.m + 1))
    assert e.value.code == M.EINVAL


# ---------------------------------------------------------------- FP32 evaluation

def _as_fp32(prob):
    q = dict(prob)
    q["precision"] = "fp32"
    return q


@pytest.mark.parametrize("make", [
    lambda: W.config_small(seed=11),
    lambda: W.corner_peak(3, 5, maxcalls=5000, nbins=40, itmax=4, seed=2**40 + 3),
    lambda: W.config_tables(seed=7, maxcalls=30_000, itmax=3),
    lambda: W.corner_peak(16, 7, maxcalls=2**17, nbins=16, itmax=2, seed=8),
    lambda: W.gauss_product(3, 10, maxcalls=6000, nbins=30, itmax=4, ita=2, seed=3,
                            lo=np.array([-1.0, 0.5, 2.0]), hi=np.array([1.0, 0.75, 9.0])),
    lambda: W.const(2, 2.5, maxcalls=8192, nbins=128, itmax=2, seed=9),
], ids=["small", "corner3", "tables6", "corner16", "bounds-noadjust", "const"])
def test_fp32_lockstep_against_float_oracle(make):
    _lockstep(_as_fp32(make()))


def test_fp32_against_fp64_oracle_same_grid():
    """The FP32-eval pass samples the FP64 points to 2^-24; its estimate on a
    fixed grid is within a few 1e-6 of the FP64 oracle's."""
    prob = W.config_tables(seed=2, maxcalls=2_000_000, itmax=1)
    d, nb = prob["dim"], prob["nbins"]
    rng = np.random.default_rng(5)
    grid = np.concatenate([np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
                           for _ in range(d)])
    g32 = M.Sampler(_as_fp32(prob)).sample(0, grid, adjust=False)
    o64 = O.vsample(prob, 0, grid, hist=False)
    assert abs(g32["I"] - o64["I"]) <= 1e-5 * abs(o64["I"])
    assert abs(g32["var"] - o64["var"]) <= 1e-4 * o64["var"]


def test_fp32_full_size_tables_1e8():
    prob = _as_fp32(W.config_tables(seed=1))
    s, full = _sampled_full_size(prob, [0.0, 0.5, 1.0])
    r = s.sample(0, O.init_grid(6, 500), adjust=False)
    assert abs(r["I"] - CF.exact(prob)) < 5 * math.sqrt(r["var"])


def test_fp32_integrate_accuracy():
    prob = W.corner_peak(5, 14, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=5)
    g = M.integrate(_as_fp32(prob))
    assert g.converged and g.error <= 1e-3 * abs(g.estimate)
    assert abs(g.estimate - CF.exact(prob)) < 5 * g.error


# ---------------------------------------------------------------- m-Cubes1D

@pytest.mark.parametrize("make", [
    lambda: W.symmetric_gauss(4, c=0.45, w=0.12, maxcalls=20_000, nbins=50, itmax=3, seed=6, one_d=True),
    lambda: W.symmetric_corner(3, a=1.2, maxcalls=8_000, nbins=40, itmax=3, seed=7, one_d=True),
    lambda: W.symmetric_corner(5, a=0.9, maxcalls=30_000, nbins=40, itmax=2, seed=8, one_d=True,
                               precision="fp32"),
], ids=["gauss4", "corner3", "corner5-fp32"])
def test_one_d_lockstep(make):
    grid = _lockstep(make())
    rows = grid.reshape(make()["dim"], -1)
    assert all(np.array_equal(rows[0], rows[j]) for j in range(len(rows)))


def test_one_d_integrate_matches_oracle():
    prob = W.symmetric_gauss(5, c=0.45, w=0.12, maxcalls=200_000, nbins=60, itmax=6, seed=3, one_d=True)
    g = M.integrate(prob)
    o = O.integrate(prob)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)
    assert np.array_equal(g.grid.reshape(5, -1)[0], g.grid.reshape(5, -1)[4])
    assert abs(g.estimate - CF.exact(prob)) < 5 * g.error


# ---------------------------------------------------------------- production kernels at benchmark shapes
#
# The kernels the benchmark times (not the tracing instantiations), at the
# launch shape the library picks, on problems large enough that every lane
# strides over at least ten sub-cubes (so the grid-stride loop and its digit
# odometer run many times per lane), against the oracle's whole pass:
# estimate, variance and the full d x nb histogram.  The integrands are
# positive, so sum_t |I_t| is the pass total.

def _random_grid(d, nb, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]])
                           for _ in range(d)])


def _gauss_quantile_grid(prob):
    """Per axis, bins of equal mass of the axis's Gaussian factor exp(-((x-c)/w)^2)
    (a grid VEGAS would adapt towards), so that most samples of a narrow peak
    give non-zero values."""
    from scipy.stats import norm
    d, nb = prob["dim"], prob["nbins"]
    c, w = prob["params"][:d], prob["params"][d:]
    rows = []
    for j in range(d):
        lo, hi = norm.cdf(-c[j] / (w[j] / math.sqrt(2))), norm.cdf((1 - c[j]) / (w[j] / math.sqrt(2)))
        q = c[j] + w[j] / math.sqrt(2) * norm.ppf(lo + (hi - lo) * np.arange(1, nb) / nb)
        q = np.maximum.accumulate(np.clip(q, 0.0, 1.0))
        rows.append(np.concatenate([[0.0], q, [1.0]]))
    return np.concatenate(rows)


def _production_passes(prob, grids, noadjust=True):
    d, nb = prob["dim"], prob["nbins"]
    s = M.Sampler(prob)
    blocks, threads, _ = M.launch_shape(s.bp, adjust=True)
    assert s.m >= 10 * blocks * threads, (s.m, blocks, threads)
    tol = _tol(prob)
    for it, grid in enumerate(grids):
        label = f"{prob['integrand']} d={d} {prob.get('precision', 'fp64')} iter {it}"
        print(label, "blocks", blocks, "threads", threads, "cubes", s.m, flush=True)
        gpu = s.sample(it, grid, True)
        gpu["nbins"] = nb
        ref = O.vsample(prob, it, grid, hist=True)
        _compare_totals(gpu, ref, _positive_scale(ref), label, tol)
        a = M.refine_grid(d, nb, prob["alpha"], gpu["hist"], grid)
        _refined_grids_agree(prob, gpu["hist"], ref["hist"], grid, a, tol)
    if noadjust:
        it = len(grids)
        nblocks, nthreads, _ = M.launch_shape(s.bp, adjust=False)
        assert s.m >= 10 * nblocks * nthreads
        gpu = s.sample(it, grids[-1], False)
        ref = O.vsample(prob, it, grids[-1], hist=False)
        _compare_totals(gpu, ref, _positive_scale(ref), f"no-adjust iter {it}", tol)


@pytest.mark.parametrize("precision,threads", [("fp64", 256), ("fp32", 0)])
def test_no_adjust_pass_with_more_workgroups_between_adjusting_passes(precision, threads):
    """d = 2, nb = 4000: the adjusting pass's LDS (grid and histogram, 128 KB)
    fits one workgroup per CU, the no-adjust pass's (the grid, 64 KB) more, so
    the no-adjust pass launches more workgroups and writes more per-workgroup
    totals.  The histogram accumulators that the adjusting passes add into
    must come through it untouched: adjusting, no-adjust, adjusting on one
    workspace, each against the oracle."""
    prob = W.corner_peak(2, 21, maxcalls=4_000_000, nbins=4000, itmax=3, precision=precision)
    s = M.Sampler(prob, threads=threads)
    b_adj = M.launch_shape(s.bp, adjust=True)[0]
    b_noadj = M.launch_shape(s.bp, adjust=False)[0]
    print(precision, "blocks adjusting", b_adj, "no-adjust", b_noadj, flush=True)
    assert b_noadj > b_adj
    grid = _random_grid(2, 4000, 23)
    for it, adjust in enumerate([True, False, True]):
        gpu = s.sample(it, grid, adjust)
        gpu["nbins"] = 4000
        ref = O.vsample(prob, it, grid, hist=adjust)
        _compare_totals(gpu, ref, _positive_scale(ref), f"pass {it} adjust={adjust}", _tol(prob))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_production_tables_d6(precision):
    # FP32 evaluation runs 1024 x 768 lanes (two workgroups per CU, launched
    # twice over): 16^6 sub-cubes give each lane twenty
    maxcalls = 10_000_000 if precision == "fp64" else 2 * 16**6
    prob = W.config_tables(seed=4, maxcalls=maxcalls, itmax=3, precision=precision)
    _production_passes(prob, [O.init_grid(6, 500), _random_grid(6, 500, 3)])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_production_corner_peak_d8(precision):
    prob = W.config_corner8(seed=4, maxcalls=2 * 8**8, itmax=2, precision=precision)
    _production_passes(prob, [_random_grid(8, 500, 5)], noadjust=precision == "fp32")


@pytest.mark.parametrize("precision,g", [("fp64", 7), ("fp32", 8)])
def test_production_narrow_gaussian_d8(precision, g):
    """w = 0.01: on equal bins almost every sample is exp(-(hundreds)); on the
    Gaussian-quantile grid most are of order one.  (The FP32 kernel runs six
    times as many lanes, hence the larger lattice.)"""
    prob = W.config_gauss8(seed=4, maxcalls=2 * g**8, itmax=3, precision=precision)
    _production_passes(prob, [O.init_grid(8, 500), _gauss_quantile_grid(prob)])


# ---------------------------------------------------------------- whole passes at the benchmark sizes
#
# The production kernel at the benchmark's own size and launch shape (1e8
# samples at d = 6 with the tables, 1e9 at d = 8 with the corner peak, both
# precisions), one adjusting pass on a random grid, against the oracle's whole
# pass over every sub-cube (spread over the host's CPUs): estimate, variance
# and the full d x nb histogram, element by element.

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("config", ["tables_d6_1e8", "corner_peak_d8_1e9", "narrow_gaussian_d8_1e9",
                                    "symmetric_corner_d8_1e9_one_d"])
def test_whole_pass_at_benchmark_size(config, precision):
    import oracle_pool as P

    if config == "tables_d6_1e8":
        prob = W.config_tables(seed=1, precision=precision)
    elif config == "corner_peak_d8_1e9":
        prob = W.config_corner8(seed=1, precision=precision)
    elif config == "narrow_gaussian_d8_1e9":
        prob = W.config_gauss8(seed=1, precision=precision)
    else:
        prob = W.config_symmetric8(seed=1, precision=precision, one_d=1)
    d, nb = prob["dim"], prob["nbins"]
    s = M.Sampler(prob)
    bp = M.BoundProblem(prob)
    assert M.launch_shape(s.bp, adjust=True) == M.launch_shape(bp, adjust=True)
    # the w = 0.01 Gaussian on a grid of equal Gaussian mass, where its samples
    # are not almost all zero; the m-Cubes1D pass on one shared random grid
    if config == "narrow_gaussian_d8_1e9":
        grid = _gauss_quantile_grid(prob)
    elif prob.get("one_d"):
        grid = np.tile(_random_grid(1, nb, 17), d)
    else:
        grid = _random_grid(d, nb, 17)
    label = f"{config} {precision}"
    print(label, "shape", M.launch_shape(s.bp, adjust=True), "cubes", s.m, flush=True)
    gpu = s.sample(1, grid, True)
    gpu["nbins"] = nb
    ref = P.vsample(prob, 1, grid, hist=True)
    _compare_totals(gpu, ref, _positive_scale(ref), label, _tol(prob))


def test_narrow_gaussian_d8_free_running_matches_oracle():
    """The whole run at 1e7 samples per iteration, five iterations: each
    iteration's estimate as the oracle's (which adapts the same way from the
    same samples), and neither claims convergence: the estimates climb by tens
    of orders of magnitude as the grid creeps towards a peak of width 0.01."""
    prob = W.config_gauss8(seed=2, maxcalls=10_000_000, itmax=5, tau_rel=1e-3)
    g = M.integrate(prob)
    o = O.integrate(prob)
    assert g.iterations == o["iterations"] == 5
    assert not g.converged and not o["converged"]
    assert np.allclose(g.it_I, o["it_I"], rtol=1e-11, atol=0)
    assert np.allclose(g.it_var, o["it_var"], rtol=1e-10, atol=0)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)
    assert g.error >= 0.5 * abs(g.estimate)


def test_fp32_underflow_is_not_an_exact_zero():
    """FP32 evaluation of the w = 0.01 Gaussian at 1e6 samples: every expf
    underflows, so every iteration is 0 with variance 0.  The result is 0 with
    an infinite error and not converged, as in the oracle (before, such
    iterations counted as exact and the run stopped at 0 +- 0)."""
    prob = W.config_gauss8(seed=2, maxcalls=1_000_000, itmax=4, tau_rel=1e-3, precision="fp32")
    g = M.integrate(prob)
    o = O.integrate(prob)
    assert (g.estimate, g.error, g.iterations, g.converged) == (0.0, math.inf, 4, False)
    assert (o["estimate"], o["error"], o["iterations"], o["converged"]) == (0.0, math.inf, 4, False)


def test_fp32_jacobian_overflow_is_reported():
    """d = 12 on (0, 1e4)^12: the float Jacobian overflows; the FP32 pass must
    report a non-finite value (the FP64 pass of the same problem is finite)."""
    d = 12
    prob = W.symmetric_corner(d, a=1.0, maxcalls=2**13, nbins=8, itmax=2, lo=np.zeros(d),
                              hi=np.full(d, 1e4))
    M.integrate(prob)
    with pytest.raises(M.MCubesError) as e:
        M.integrate(dict(prob, precision="fp32"))
    assert e.value.code == M.ENONFINITE


def test_resume_from_saved_state(tmp_path):
    """Five iterations through the step-level calls, the state (grid and
    per-iteration results) saved and loaded, five more: the 10-iteration
    mc_integrate with the same seed, to the rounding of the histogram sums."""
    prob = W.config_tables(seed=6, maxcalls=1_000_000, itmax=10, ita=8)
    whole = M.integrate(prob)
    s = M.Sampler(prob)
    d, nb = prob["dim"], prob["nbins"]

    def run(it0, it1, grid, Is, Vs):
        for it in range(it0, it1):
            adjust = it < prob["ita"]
            r = s.sample(it, grid, adjust)
            Is.append(r["I"])
            Vs.append(r["var"])
            if adjust:
                grid = M.refine_grid(d, nb, prob["alpha"], r["hist"], grid)
        return grid

    Is, Vs = [], []
    grid = run(0, 5, M.init_grid(d, nb), Is, Vs)
    np.savez(tmp_path / "state.npz", grid=grid, I=np.array(Is), V=np.array(Vs))
    st = np.load(tmp_path / "state.npz")
    Is, Vs = list(st["I"]), list(st["V"])
    grid = run(5, 10, st["grid"], Is, Vs)
    est, err, chi2 = M.weighted_estimate(Is, Vs)
    assert np.allclose(Is, whole.it_I, rtol=1e-12, atol=0)
    assert np.allclose(Vs, whole.it_var, rtol=1e-11, atol=0)
    assert est == pytest.approx(whole.estimate, rel=1e-12)
    assert err == pytest.approx(whole.error, rel=1e-11)
    assert np.abs(grid - whole.grid).max() <= 1e-10

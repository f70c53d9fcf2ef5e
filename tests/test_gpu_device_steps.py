"""Runs whose steps between sampling passes (Weighted-Estimates,
Check-Convergence, Adjust-Bin-Bounds of Alg. 2) stay on the device.

Bars:
  * the device bin adjustment (mc_refine_grid_device) against the host's
    mc_refine_grid / mc_refine_grid_1d on the same histogram: every boundary
    within 1e-12 (the two differ in the order of their sums and in the
    rounding of pow and log: a relative difference of about nb ulps in a
    running sum moves a boundary by that much of the total weight over the
    weight of the bin it falls in, up to 1.3e-13 on these histograms; a wrong
    step, e.g. a boundary placed in the wrong bin, moves one by a bin width,
    about 1/nb), axes without usable weight left exactly as they were, and the
    same output for the same input;
  * whole runs against the host-steps run and the oracle: the same number of
    iterations and the same convergence decision, per-iteration estimates
    within 1e-11 relative, grids within 1e-12."""
import threading

import numpy as np
import pytest

import closed_forms as CF
import oracle as O
from paper_2202_01753_amd import mcubes as M
from paper_2202_01753_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(prob):
    return dict(prob, device_steps=True)


# ---------------------------------------------------------------- the bin adjustment alone

def _histograms(d, nb, seed):
    rng = np.random.default_rng(seed)
    rows = [
        rng.random(nb) ** 4,                                   # smooth, positive
        np.where(rng.random(nb) < 0.7, 0.0, rng.random(nb)),   # mostly empty bins
        np.exp(rng.uniform(-740, 0, nb)),                      # 320 decades, subnormals at the tail
        np.zeros(nb),                                          # no weight: unchanged
        np.where(np.arange(nb) == nb // 3, 1.0, 0.0),          # one bin
        np.full(nb, 0.25),                                     # equal weights
        rng.random(nb) * 1e306,                                # the total overflows (nb > 2): unchanged
    ]
    return np.concatenate([rows[(j + seed) % len(rows)] for j in range(d)])


def _random_grid(d, nb, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.concatenate([[0.0], np.sort(rng.random(nb - 1)), [1.0]]) for _ in range(d)])


@pytest.mark.parametrize("d,nb", [(7, 2), (7, 3), (7, 9), (7, 100), (7, 500), (2, 4000)])
@pytest.mark.parametrize("seed", [0, 1])
def test_device_refine_matches_host(d, nb, seed):
    hist = _histograms(d, nb, seed)
    for grid in (M.init_grid(d, nb), _random_grid(d, nb, seed + 5)):
        for alpha in (1.5, 0.5):
            host = M.refine_grid(d, nb, alpha, hist, grid)
            dev = M.refine_grid_device(d, nb, alpha, hist, grid)
            assert np.abs(dev - host).max() <= 1e-12, (d, nb, alpha)
            rows = dev.reshape(d, nb + 1)
            assert np.all(rows[:, 0] == 0.0) and np.all(rows[:, -1] == 1.0)
            assert np.all(np.diff(rows, axis=1) >= 0.0)
            # axes that keep their boundaries (no usable weight) keep them exactly
            same = np.all(host.reshape(d, nb + 1) == grid.reshape(d, nb + 1), axis=1)
            assert np.array_equal(rows[same], grid.reshape(d, nb + 1)[same])


def test_device_refine_is_deterministic():
    """The same histogram and grid give the same boundaries, bit for bit, call
    after call (fixed summation order, no atomics)."""
    d, nb = 6, 500
    grid = _random_grid(d, nb, 9)
    hist = _histograms(d, nb, 0)
    first = M.refine_grid_device(d, nb, 1.5, hist, grid)
    for _ in range(3):
        np.testing.assert_array_equal(M.refine_grid_device(d, nb, 1.5, hist, grid), first)


@pytest.mark.parametrize("nb", [2, 50, 500])
def test_device_refine_1d_matches_host(nb):
    d = 6
    hist = _histograms(d, nb, 3)
    grid = np.tile(_random_grid(1, nb, 4), d)
    host = M.refine_grid_1d(d, nb, 1.5, hist, grid)
    dev = M.refine_grid_device(d, nb, 1.5, hist, grid, one_d=True)
    assert np.abs(dev - host).max() <= 1e-12
    rows = dev.reshape(d, nb + 1)
    assert np.all(rows == rows[0])


def test_device_refine_rejects_bad_arguments():
    import ctypes as C

    import torch

    buf = torch.zeros(4 * (M.MC_DEVICE_STEPS_MAX_BINS + 2), dtype=torch.float64, device="cuda")
    p = C.c_void_p(buf.data_ptr())
    f = M.lib().mc_refine_grid_device
    for args in [(0, 8, 1.5, 0, p, p), (M.MC_MAX_DIM + 1, 8, 1.5, 0, p, p), (2, 1, 1.5, 0, p, p),
                 (1, M.MC_DEVICE_STEPS_MAX_BINS + 1, 1.5, 0, p, p), (2, 8, 0.0, 0, p, p),
                 (2, 8, float("nan"), 0, p, p), (2, 8, float("inf"), 0, p, p), (2, 8, 1.5, 2, p, p),
                 (2, 8, 1.5, 0, None, p), (2, 8, 1.5, 0, p, None)]:
        assert f(*args, None) == M.EINVAL, args
    torch.cuda.synchronize()
    assert not buf.any()  # nothing ran


# ---------------------------------------------------------------- whole runs

def _same_run(a, b, rel=1e-11, grid_atol=1e-12):
    assert a.iterations == b.iterations and a.converged == b.converged
    assert np.allclose(a.it_I, b.it_I, rtol=rel, atol=0)
    assert np.allclose(a.it_var, b.it_var, rtol=100 * rel, atol=0)
    assert a.estimate == pytest.approx(b.estimate, rel=rel)
    assert a.error == pytest.approx(b.error, rel=100 * rel)
    assert np.abs(a.grid - b.grid).max() <= grid_atol


CASES = [
    dict(make=lambda: W.config_small(seed=21), name="gauss d2 free running"),
    dict(make=lambda: W.corner_peak(5, 14, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=5),
         name="corner d5 converges"),
    dict(make=lambda: W.gauss_product(3, 10, maxcalls=60_000, nbins=30, itmax=6, ita=3, seed=3,
                                      lo=np.array([-1.0, 0.5, 2.0]), hi=np.array([1.0, 0.75, 9.0])),
         name="bounds, no-adjust tail"),
    dict(make=lambda: W.config_tables(seed=8, maxcalls=1_000_000, itmax=4), name="tables d6"),
    dict(make=lambda: W.config_tables(seed=8, maxcalls=1_000_000, itmax=4, precision="fp32"),
         name="tables d6 fp32"),
    dict(make=lambda: W.symmetric_corner(6, a=1.0, maxcalls=400_000, nbins=200, itmax=5, one_d=1, seed=4),
         name="m-Cubes1D"),
    dict(make=lambda: W.gauss_product(3, 12, maxcalls=100_000, nbins=50, itmax=4, ita=0, seed=6),
         name="no adjusting pass"),
    dict(make=lambda: W.corner_peak(4, 13, maxcalls=100_000, nbins=64, itmax=1, seed=7), name="one pass"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_device_steps_match_host_steps(case):
    prob = case["make"]()
    host = M.integrate(prob)
    dev = M.integrate(_dev(prob), timing=True)
    print(case["name"], "iterations", dev.iterations, "estimate", dev.estimate, flush=True)
    _same_run(dev, host)
    assert dev.sample_ms > 0.0 and dev.finalize_ms > 0.0


def test_device_steps_match_the_oracle():
    prob = W.config_small(seed=21)
    g = M.integrate(_dev(prob))
    o = O.integrate(prob)
    assert g.iterations == o["iterations"] == 10
    assert np.allclose(g.it_I, o["it_I"], rtol=1e-11, atol=0)
    assert np.allclose(g.it_var, o["it_var"], rtol=1e-10, atol=0)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)
    assert g.chi2_dof == pytest.approx(o["chi2_dof"], rel=1e-8)
    assert abs(g.estimate - CF.exact(prob)) < 5 * g.error


def test_device_steps_convergence_matches_the_oracle():
    prob = W.corner_peak(5, 14, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=5)
    g = M.integrate(_dev(prob))
    o = O.integrate(prob)
    assert g.iterations == o["iterations"] < 12 and g.converged and o["converged"]
    assert np.allclose(g.it_I, o["it_I"], rtol=1e-11, atol=0)
    assert g.estimate == pytest.approx(o["estimate"], rel=1e-11)


def test_device_steps_report_a_non_finite_integrand():
    """d = 12 on (0, 1e4)^12: the float Jacobian overflows in FP32 evaluation."""
    d = 12
    prob = W.symmetric_corner(d, a=1.0, maxcalls=2**13, nbins=8, itmax=3, lo=np.zeros(d),
                              hi=np.full(d, 1e4), device_steps=True)
    M.integrate(prob)
    with pytest.raises(M.MCubesError) as e:
        M.integrate(dict(prob, precision="fp32"))
    assert e.value.code == M.ENONFINITE
    # the workspace and the library stay usable
    r = M.integrate(prob)
    assert r.iterations == 3


def test_device_steps_prepared_runs_repeat():
    """mc_integrate_prepared with device steps, run after run on one workspace
    (each run starts from a fresh grid and run state), including a run that
    converges early followed by one that does not."""
    prob = _dev(W.corner_peak(5, 14, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=5))
    bp = M.BoundProblem(prob)
    ws = M.Workspace(bp)
    M.prepare(prob, ws, bp=bp)
    first = M.integrate(prob, ws=ws, bp=bp, prepared=True)
    assert first.converged
    bp.s.tau_rel = 0.0
    full = M.integrate(prob, ws=ws, bp=bp, prepared=True)
    assert full.iterations == 12 and not full.converged
    again = M.integrate(dict(prob, tau_rel=0.0))
    _same_run(full, again)
    bp.s.tau_rel = 1e-3
    _same_run(M.integrate(prob, ws=ws, bp=bp, prepared=True), first)


def test_device_steps_above_the_bin_limit_run_on_the_host():
    nb = M.MC_DEVICE_STEPS_MAX_BINS + 1
    prob = W.corner_peak(1, 3, maxcalls=40_000, nbins=nb, itmax=3, seed=2)
    _same_run(M.integrate(_dev(prob)), M.integrate(prob))


def test_device_steps_on_two_streams():
    import torch

    probs = [_dev(W.config_tables(seed=21, maxcalls=2_000_000, itmax=4)),
             _dev(W.corner_peak(6, 3, maxcalls=3_000_000, nbins=200, itmax=5, seed=22))]
    alone = [M.integrate(p) for p in probs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out, errors = [None, None], []

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
        _same_run(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("config", ["tables_d6_1e8", "corner_peak_d8_1e9"])
def test_device_steps_at_benchmark_size(config, precision):
    """The benchmarked runs themselves (all passes, the launch shapes the
    benchmark uses) with the steps on the device against the same runs with
    the steps on the host, whose passes the lockstep and whole-pass tests hold
    to the oracle: same iterations, per-iteration estimates within 1e-11,
    grids within 1e-12."""
    if config == "tables_d6_1e8":
        prob = W.config_tables(seed=3, precision=precision)
    else:
        prob = W.config_corner8(seed=3, precision=precision)
    host = M.integrate(prob)
    dev = M.integrate(_dev(prob), timing=True)
    print(config, precision, "iterations", dev.iterations, "estimate", dev.estimate, "+-", dev.error,
          "sample ms/pass", dev.sample_ms / dev.iterations, flush=True)
    _same_run(dev, host)
    assert abs(dev.estimate - CF.exact(prob)) < 5 * dev.error

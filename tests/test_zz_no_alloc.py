"""The entry point that allocates nothing, mc_integrate_noalloc, against
mc_integrate on the same problems: two calls in a row on the one scratch
array, the second with a smaller problem, each with mc_integrate's results
to the rounding of the LDS histogram sums (the same bar as runs that reuse a
prepared workspace)."""
import ctypes as C

import numpy as np
import pytest

from paper_2202_01753_amd import mcubes as M
from paper_2202_01753_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _same_run(a, b):
    assert a.iterations == b.iterations and a.converged == b.converged
    assert np.allclose(a.it_I, b.it_I, rtol=TOL, atol=0)
    assert np.allclose(a.it_var, b.it_var, rtol=1e-9, atol=0)
    assert a.estimate == pytest.approx(b.estimate, rel=TOL, abs=0)
    assert a.error == pytest.approx(b.error, rel=1e-9, abs=0)
    assert np.allclose(a.grid, b.grid, rtol=0, atol=1e-12)


def test_noalloc_matches_integrate_on_successive_calls():
    probs = [W.config_tables(seed=8, maxcalls=2_000_000, itmax=4),
             W.config_tables(seed=9, maxcalls=600_000, itmax=3, precision="fp32"),
             W.config_small(seed=10)]
    for prob in probs:
        print("noalloc", prob["integrand"], prob["dim"], prob["maxcalls"], prob["precision"], flush=True)
        a = M.integrate_noalloc(prob)
        b = M.integrate(prob)
        _same_run(a, b)


def test_noalloc_rejects_problems_beyond_the_scratch():
    # 2^20 workgroups asked for: their totals alone are 32 MB
    prob = W.config_corner8(seed=1)
    bp = M.BoundProblem(prob, 1 << 20)
    assert M.workspace_bytes(bp) > 16 << 20
    # the benchmark's own d = 8 shape fits
    assert M.workspace_bytes(M.BoundProblem(prob)) < 16 << 20
    res = M.Result(estimate=-3.0)
    code = M.lib().mc_integrate_noalloc(bp.ref, None, C.byref(res), None, None)
    assert code == M.EWORKSPACE and res.estimate == -3.0
    bad = dict(W.config_small(), nbins=1)
    code = M.lib().mc_integrate_noalloc(M.BoundProblem(bad).ref, None, C.byref(res), None, None)
    assert code == M.EINVAL and res.estimate == -3.0
    # the scratch is still usable after a rejected call
    small = W.config_small(seed=12)
    _same_run(M.integrate_noalloc(small), M.integrate(small))

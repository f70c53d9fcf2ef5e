"""GPU tests of the batched launch and the serving loop (through the C ABI).

The bar: each integral's result is the same alone and in the mix, within the
stated tolerance.  Its samples are identical in both (the random numbers are
keyed by its own seed, iteration, cube and sample); what can differ is the
order in which sums are formed (different work splits), which moves grids by
ulps and estimates by far less than 1e-10 relative."""
import math

import numpy as np
import pytest

import closed_forms as CF
import oracle as O
from paper_2202_01753_amd import mcubes as M
from paper_2202_01753_amd import workloads as W

pytestmark = pytest.mark.gpu

MIX_TOL = 1e-10


def _mix(seed=0, n=14):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        d = int(rng.integers(2, 11))
        kind = ["gauss_product", "corner_peak", "gauss_tables", "const"][i % 4]
        if kind == "gauss_tables" and d < 4:
            d = 4 + i % 3
        N = int(10 ** rng.uniform(3.5, 5.5))
        nb = int(rng.integers(20, 200))
        itmax = int(rng.integers(2, 7))
        kw = dict(maxcalls=N, nbins=nb, itmax=itmax, seed=100 + i,
                  precision="fp32" if i % 5 == 4 else "fp64")
        if kind == "gauss_product":
            p = W.gauss_product(d, 10 + i, **kw)
        elif kind == "corner_peak":
            p = W.corner_peak(d, 10 + i, **kw)
        elif kind == "gauss_tables":
            p = W.gauss_tables(d, 10 + i, w_range=(0.1, 0.3), **kw)
        else:
            p = W.const(d, 1.5, **kw)
        if i % 3 == 0:
            p["ita"] = max(1, itmax - 1)
        if i % 7 == 3:
            p["tau_rel"] = 2e-3
        out.append(p)
    return out


def _close(a, b, tol=MIX_TOL):
    assert a["iterations"] == b["iterations"], (a, b)
    assert a["converged"] == b["converged"]
    assert a["estimate"] == pytest.approx(b["estimate"], rel=tol, abs=1e-300)
    assert a["error"] == pytest.approx(b["error"], rel=100 * tol, abs=1e-300)


def test_batch_alone_vs_mix():
    probs = _mix()
    mixed, stats = M.batch_integrate(probs)
    assert stats.steps == max(r["iterations"] for r in mixed)
    for i, p in enumerate(probs):
        alone, _ = M.batch_integrate([p])
        _close(mixed[i], alone[0])


def test_batch_matches_single_integral_path_and_oracle():
    probs = [W.config_small(seed=4), W.corner_peak(5, 14, maxcalls=100_000, nbins=80, itmax=6, seed=5),
             W.config_tables(seed=6, maxcalls=300_000, itmax=4),
             dict(W.corner_peak(3, 2, maxcalls=20_000, nbins=60, itmax=5, seed=8), precision="fp32")]
    mixed, _ = M.batch_integrate(probs)
    for i, p in enumerate(probs):
        single = M.integrate(p)
        r = {"estimate": single.estimate, "error": single.error, "iterations": single.iterations,
             "converged": single.converged}
        _close(mixed[i], r)
        o = O.integrate(p)
        assert mixed[i]["estimate"] == pytest.approx(o["estimate"], rel=1e-9 if p.get("precision") == "fp32" else MIX_TOL)
        assert abs(mixed[i]["estimate"] - CF.exact(p)) < 5 * mixed[i]["error"]


def test_batch_first_pass_against_oracle():
    """One non-adjusting iteration per integral: the batch estimate is the
    oracle's V-Sample estimate on the uniform grid, to summation order."""
    probs = []
    for i, p in enumerate(_mix(seed=3, n=8)):
        q = dict(p, itmax=1, ita=0, tau_rel=0.0)
        probs.append(q)
    mixed, _ = M.batch_integrate(probs)
    for p, r in zip(probs, mixed):
        ref = O.vsample(p, 0, O.init_grid(p["dim"], p["nbins"]), hist=False, trace=True)
        scale = float(np.abs(ref["ctrace"][:, 0]).sum())
        tol = 1e-6 if p.get("precision") == "fp32" and p["integrand"] not in ("const", "corner_peak") else 1e-12
        assert abs(r["estimate"] - ref["I"]) <= tol * scale + 1e-300, (p["integrand"], p["dim"])


def test_batch_nonfinite_is_isolated():
    good = W.config_small(seed=1)
    bad = W.const(3, np.inf, maxcalls=1000, nbins=10, itmax=2, seed=2)
    res, _ = M.batch_integrate([good, bad, W.corner_peak(4, 1, maxcalls=5000, nbins=30, itmax=3, seed=3)])
    assert isinstance(res[1], M.MCubesError) and res[1].code == M.ENONFINITE
    alone, _ = M.batch_integrate([good])
    _close(res[0], alone[0])
    assert res[2]["iterations"] == 3


def test_batch_rejects_high_dimension():
    with pytest.raises(M.MCubesError) as e:
        M.batch_integrate([W.gauss_product(11, 1, maxcalls=10_000, nbins=10, itmax=1)])
    assert e.value.code == M.EINVAL


def test_server_admits_by_memory_and_matches_alone():
    probs = _mix(seed=7, n=10)
    assert sum(p["integrand"] == "gauss_tables" for p in probs) >= 2
    # an arena with room for one integral with FP64 tables (1 MiB) and a few
    # small ones: the second table integral must wait for the first to finish
    srv = M.Server(ws_bytes=512 * 2**20, arena_bytes=int(1.5 * 2**20), max_active=64)
    ids = [srv.submit(p) for p in probs[:6]]
    seen_queued = False
    steps = 0
    while True:
        a, q, f = srv.step()
        steps += 1
        seen_queued |= q > 0
        if steps == 2:
            ids += [srv.submit(p) for p in probs[6:]]  # arrivals while others run
        if a == 0 and q == 0 and steps > 2:
            break
        assert steps < 500
    assert seen_queued
    for rid, p in zip(ids, probs):
        st, res, status = srv.poll(rid)
        assert st == M.REQ_DONE and status == M.OK
        alone, _ = M.batch_integrate([p])
        _close(res, alone[0])
        srv.release(rid)
    s = srv.stats()
    assert 0 < s.steps <= steps and s.calls > 0
    srv.close()


def test_batch_one_d_matches_single_path():
    probs = [W.symmetric_gauss(5, c=0.45, w=0.12, maxcalls=200_000, nbins=60, itmax=6, seed=3, one_d=True),
             W.symmetric_corner(4, a=1.3, maxcalls=100_000, nbins=60, itmax=5, seed=4, one_d=True),
             W.config_small(seed=2)]
    mixed, _ = M.batch_integrate(probs)
    for i, p in enumerate(probs):
        single = M.integrate(p)
        _close(mixed[i], {"estimate": single.estimate, "error": single.error,
                          "iterations": single.iterations, "converged": single.converged})


def test_batch_large_lds_groups_and_fp32_tables():
    """Integrals whose LDS footprint limits the workgroups per CU (d = 10 with
    500 bins needs 80 KB and runs in the wide-workgroup launch group) and the
    FP32 table kernel, each the same alone and in a mix with small integrals,
    and the same as the single-integral path."""
    probs = [
        W.gauss_product(10, 31, maxcalls=2_000_000, nbins=500, itmax=3, seed=41),
        dict(W.corner_peak(9, 32, maxcalls=1_500_000, nbins=480, itmax=3, seed=42), precision="fp32"),
        W.gauss_tables(6, 33, w_range=(0.1, 0.3), maxcalls=400_000, nbins=150, itmax=4, seed=43,
                       precision="fp32"),
        W.gauss_tables(8, 34, w_range=(0.1, 0.3), maxcalls=600_000, nbins=300, itmax=3, seed=44),
        W.config_small(seed=45),
        W.corner_peak(3, 35, maxcalls=20_000, nbins=60, itmax=4, seed=46),
    ]
    mixed, _ = M.batch_integrate(probs)
    for i, p in enumerate(probs):
        # FP32 evaluation can turn an ulp of difference in a boundary (from
        # the order of the histogram sums, or device vs host pow/log) into a
        # float rounding of a point, hence the looser bound there
        tol = 1e-7 if p.get("precision") == "fp32" else MIX_TOL
        alone, _ = M.batch_integrate([p])
        _close(mixed[i], alone[0], tol)
        single = M.integrate(p)
        _close(mixed[i], {"estimate": single.estimate, "error": single.error,
                          "iterations": single.iterations, "converged": single.converged}, tol)


def _serve_all(probs, budget=0, max_skip=4, late=()):
    """Runs probs through a server (late ones submitted after the second
    step); returns the results by index, the samples the server had taken
    when each finished, and the stats."""
    srv = M.Server(ws_bytes=512 * 2**20, arena_bytes=64 * 2**20, max_active=256)
    if budget:
        srv.set_step_budget(budget, max_skip)
    ids = {srv.submit(p): i for i, p in enumerate(probs) if i not in late}
    out, done_at, steps = {}, {}, 0
    while len(out) < len(probs):
        srv.step()
        steps += 1
        if steps == 2:
            ids.update({srv.submit(probs[i]): i for i in late})
        calls = srv.stats().calls
        for rid in srv.finished():
            st, res, status = srv.poll(rid)
            assert st == M.REQ_DONE and status == M.OK
            out[ids[rid]] = res
            done_at[ids[rid]] = calls
            srv.release(rid)
        assert steps < 2000
    s = srv.stats()
    srv.close()
    return out, done_at, s


def test_server_step_budget_same_results_short_requests_first():
    # two long requests (many samples per iteration, all iterations) among
    # short ones; under a budget smaller than one long iteration each result is
    # the same as without it, and the short requests finish after fewer samples
    # of the whole stream have been taken
    probs = _mix(seed=11, n=12)
    longs = (0, 5)
    for i in longs:
        probs[i] = dict(probs[i], maxcalls=2_000_000, itmax=6, tau_rel=0.0)
    budget, max_skip = 300_000, 2
    for i in longs:
        _, m, p = M.shape(probs[i]["dim"], probs[i]["maxcalls"])
        assert m * p > budget
    free, at0, s0 = _serve_all(probs, late=(3, 9))
    capped, at1, s1 = _serve_all(probs, budget=budget, max_skip=max_skip, late=(3, 9))
    for i in range(len(probs)):
        _close(capped[i], free[i])
    assert s1.calls == s0.calls  # the same iterations, in other steps
    assert s1.steps > s0.steps
    shorts = [i for i in range(len(probs)) if i not in longs]
    assert sum(at1[i] for i in shorts) < 0.5 * sum(at0[i] for i in shorts)


def test_server_step_budget_rejects_negative():
    srv = M.Server(ws_bytes=64 * 2**20, arena_bytes=16 * 2**20, max_active=8)
    with pytest.raises(M.MCubesError):
        srv.set_step_budget(-1, 4)
    with pytest.raises(M.MCubesError):
        srv.set_step_budget(10, -1)
    srv.set_step_budget(0, 0)
    srv.close()


def test_served_requests_match_the_oracle():
    """Requests served with continuous batching (one arriving after two steps,
    while the others run) against the oracle's whole run of each, not against
    the batch engine alone: a d = 6 table integral, a d = 10 Gaussian with 500
    bins per axis (80 KB of LDS: the wide-workgroup launch group), a corner
    peak that converges to its target, and a d = 3 Gaussian product.  The
    served grids are refined on the device (device pow and log), so estimates
    agree to 1e-10 relative rather than bit for bit."""
    probs = [
        W.config_tables(seed=61, maxcalls=400_000, itmax=4),
        W.gauss_product(10, 62, w_range=(0.1, 0.3), maxcalls=1_000_000, nbins=500, itmax=3, seed=63),
        W.corner_peak(5, 64, maxcalls=200_000, nbins=100, itmax=12, tau_rel=1e-3, seed=65),
        W.gauss_product(3, 66, maxcalls=50_000, nbins=100, itmax=6, seed=67),
    ]
    served, _, _ = _serve_all(probs, late=(3,))
    for i, p in enumerate(probs):
        print("served request", i, p["integrand"], p["dim"], p["nbins"], flush=True)
        o = O.integrate(p)
        r = served[i]
        assert r["iterations"] == o["iterations"] and r["converged"] == o["converged"]
        assert r["estimate"] == pytest.approx(o["estimate"], rel=MIX_TOL, abs=0)
        assert r["error"] == pytest.approx(o["error"], rel=100 * MIX_TOL, abs=0)
    assert served[2]["converged"] and served[2]["iterations"] < 12

"""Throughput of the m-Cubes VEGAS sampling path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload tables|corner8|gauss8|small|symmetric8|batch|serve]
                    [--precision fp64|fp32] [--no-cpu-baseline] [--no-corner8]

One step is one complete m-Cubes run (mc_integrate_prepared: every
iteration of sampling kernel, fixed-order reduction, weighting, convergence
check and bin adjustment) on the workload's synthetic inputs, with the steps
between passes on the device (device_steps; --host-steps runs them on the
host, and the default run reports that figure beside the headline one); the workspace is allocated and the integrand's constants and tables
are uploaded (mc_prepare) before the timed region, so the inputs are resident
in device memory when it starts.  `value` is integrand samples per second
over the K timed steps (iterations * m * p per step) of the FP64 path; the
FP32-evaluation path of the same workload, and the time of one run to a 1e-3
relative error in both, are reported beside it.  The default (d = 6 tables)
run also measures the d = 8 corner peak at 1e9 samples per iteration, the
largest single-GPU configuration, in both precisions.

The roofline entry is for the sampling kernel: its average launch duration
comes from HIP events recorded by the library on the launch stream, and its
algorithmic work is the per-sample VALU work of the method's steps in issue
slots (each instruction class at its measured cost: a full slot for the
64-bit class, half for simple 32-bit operations, more for the exponential and
the reciprocals), times the samples per launch, against the chip's issue rate
of 64-bit-class instructions.  Where the kernel's rocprofv3 summary was
taken from the same code, its measured VALU instructions per sample, issue
ratio and HBM traffic are attached.  The CPU baseline times the FP64 oracle
on this host, on one core and on one process per usable CPU (at most 16, one
GPU's share of the host), before the GPU is used, including one run to a
1e-3 relative error.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs, each issuing one wave64 instruction of the
# 64-bit class (FP64 add/mul/fma, 32x32->64 products) every 4 clocks, at
# 2.4 GHz: 3.93e13 lane issue slots per second (the FP64 vector rate, 78.6
# TFLOP/s counted as FMAs).
CUS, LANES_PER_CU_CLK, CLOCK_HZ = 256, 64, 2.4e9
VALU_PEAK_OPS = CUS * LANES_PER_CU_CLK * CLOCK_HZ  # 3.93e13 slots/s

# Issue cost of each VALU instruction class in those slots, as measured on
# gfx950 by paper_2202_01753_amd/ubench/valu_rates.hip (cycles per wave64
# instruction per SIMD / 4): the 64-bit class, 32-bit products, funnel shifts,
# shift-and-add and conversions take a full slot; simple 32-bit operations
# (FP32 add, mul, min, floor and two-operand fmac; integer add; bitwise ops)
# half of one; the three-operand v_fma_f32 3.5 cycles; v_exp_f32 about 10,
# v_rcp_f32 8 and v_rcp_f64 16.  Compares and selects, not measured on their
# own, count as simple 32-bit operations.
SLOT_COST = {"full": 1.0, "half": 0.5, "fma32": 0.875, "exp32": 2.5, "rcp32": 2.0, "rcp64": 4.0}
SLOT_OP = ("one lane's share of a 4-cycle VALU issue slot (64-bit class 1, simple 32-bit "
           "instructions 1/2, v_fma_f32 0.875, v_exp_f32 2.5, v_rcp_f32 2, v_rcp_f64 4)")


def _add(mix: dict, n: float = 1.0, **ops: float) -> None:
    for k, v in ops.items():
        mix[k] = mix.get(k, 0.0) + n * v


def op_mix(prob: dict, g_m_p, adjust: bool, fp32: bool = False) -> dict:
    """Algorithmic VALU lane-operations per sample by issue class, for the
    FP64 path (or the FP32-evaluation path with fp32 set): the method's steps
    as gfx950 instructions, with work that is uniform across the wavefront or
    invariant across a sub-cube's samples excluded.

                                FP64 path                      FP32 evaluation
      Philox4x32-10 block       17 products + 19 XOR (two-     the same, ceil(d/4) blocks
                                and three-input), ceil(d/2)
      per axis                  16: uniform 3 (two funnel      14: uniform 2, coordinate 2,
                                shifts, subtract), coordinate  bin index and clamp 5,
                                2, bin index and clamp 5,      address 1, point 2,
                                address 1, width 1, point 2,   Jacobian 2
                                Jacobian 2
      Gaussian product          3 per axis + exp 20            3 per axis + expf 10
      corner peak               d fma + binary powering +      the same in FP32 (division
                                division 11 (one v_rcp_f64)    11, one v_rcp_f32)
      two bilinear tables       2 x 20 + 2 products            2 x 18 + 2
      f J / (m p), finiteness   4                              6 (two widening conversions)
      shifted sums              3 (p-1)/p (FP64 in both paths)
      bin contributions         1 + d addresses (adjusting iterations; 1 + 1 in m-Cubes1D)
      per sub-cube, / p         variance 5, two compensated additions 14 (FP64),
                                digit odometer 4 d, digit conversion d
    """
    d = int(prob["dim"])
    _, _, p = g_m_p
    kind = prob["integrand"]
    mix: dict = {}
    _add(mix, math.ceil(d / (4 if fp32 else 2)), full=17, half=19)
    if fp32:
        _add(mix, d, full=3, half=10, fma32=1)
    else:
        _add(mix, d, full=16)
    if kind in ("gauss_product", "gauss_tables"):
        if fp32:
            _add(mix, d, half=3)
            _add(mix, exp32=1, full=3, fma32=2, half=4)
        else:
            _add(mix, d, full=3)
            _add(mix, full=18, half=2)
    if kind == "corner_peak":
        e = d + 1
        powering = (e.bit_length() - 1) + (bin(e).count("1") - 1)
        if fp32:
            _add(mix, half=d + powering)
            _add(mix, full=4, rcp32=1, fma32=3, half=3)
        else:
            _add(mix, full=d + powering + 10, rcp64=1)
    if kind == "gauss_tables":
        if fp32:
            _add(mix, 2, full=6, half=9, fma32=3)
            _add(mix, half=2)
        else:
            _add(mix, full=2 * 20 + 2)
    if fp32:
        _add(mix, full=5, half=1)
    else:
        _add(mix, full=3, half=1)
    _add(mix, full=3 * (p - 1) / p)
    if adjust:
        axes = 1 if prob.get("one_d") else d  # histogram rows (m-Cubes1D: the first axis only)
        _add(mix, full=1 + axes)
    _add(mix, 1.0 / p, full=5 + 14 + d, half=4 * d)
    return mix


def ops_per_sample(prob: dict, g_m_p, adjust: bool, fp32: bool = False) -> float:
    """VALU lane-operations per sample (all classes counted alike)."""
    return float(sum(op_mix(prob, g_m_p, adjust, fp32).values()))


def slots_per_sample(prob: dict, g_m_p, adjust: bool, fp32: bool = False) -> float:
    """Issue slots per sample: op_mix weighted by SLOT_COST, the work the
    roofline prices against VALU_PEAK_OPS."""
    return float(sum(SLOT_COST[k] * v for k, v in op_mix(prob, g_m_p, adjust, fp32).items()))


# The tables kernel's HBM traffic per launch comes from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs (scaled by a copy-kernel calibration) recorded in its
# profile summary, together with a digest of the code (comments excluded) the
# kernel is built from; it is reported only while that code is unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "vsample_tables_d6_1e8.md")
# The kernel and its launch shape (workgroup size and count, chosen on the host).
KERNEL_SOURCES = ("paper_2202_01753_amd/csrc/vsample.hpp", "paper_2202_01753_amd/csrc/vsample_tables.hip",
                  "paper_2202_01753_amd/csrc/internal.hpp", "paper_2202_01753_amd/csrc/mcubes_api.cpp",
                  "paper_2202_01753_amd/csrc/host.cpp", "paper_2202_01753_amd/build.py")


def _code_only(text: str, python: bool) -> str:
    """The text without comments and with runs of whitespace collapsed, so
    that editing a comment does not count as changing the kernel."""
    if python:
        text = re.sub(r"(?m)^\s*#.*$", "", text)
        text = re.sub(r'"""[\s\S]*?"""', "", text)
    else:
        text = re.sub(r"/\*[\s\S]*?\*/", "", text)
        text = re.sub(r"//[^\n]*", "", text)
    return " ".join(text.split())


def kernel_sources_digest(root: str = ROOT, read=None) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(root, rel)) as f:
                text = f.read()
        else:
            text = read(rel)
        h.update(_code_only(text, rel.endswith(".py")).encode())
    return h.hexdigest()


def profiled(kind: str):
    """Figures of the tables kernel ('fp64' or 'fp32') recorded in its profile
    summary: HBM bytes per launch (FETCH_SIZE, WRITE_SIZE), VALU lane-
    instructions per sample and the VALU issue ratio (SQ_INSTS_VALU,
    SQ_BUSY_CYCLES), or None where absent or taken from other kernel sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    digest = kernel_sources_digest()
    out = {}
    m = re.search(r"traffic-per-launch fp64=(\d+) fp32=(\d+) sources=([0-9a-f]{64})", text)
    if m and m.group(3) == digest:
        out["traffic"] = int(m.group(1) if kind == "fp64" else m.group(2))
    m = re.search(r"valu-per-sample fp64=([0-9.]+)/([0-9.]+) fp32=([0-9.]+)/([0-9.]+) "
                  r"sources=([0-9a-f]{64})", text)
    if m and m.group(5) == digest:
        i = 1 if kind == "fp64" else 3
        out["valu_insts_per_sample"] = float(m.group(i))
        out["valu_issue_ratio"] = float(m.group(i + 1))
    return out or None


def profiled_traffic(kind: str):
    """HBM bytes per launch of the tables kernel from its profile summary, or None."""
    return (profiled(kind) or {}).get("traffic")


WORKLOADS = {
    "tables": ("gauss_tables_d6_1e8", lambda W, seed: W.config_tables(seed=seed)),
    "batch": ("batch_4096_mixed", None),
    "serve": ("served_poisson_2000_per_s", None),
    "small": ("gauss_product_d2_1e4", lambda W, seed: W.config_small(seed=seed)),
    "corner8": ("corner_peak_d8_1e9", lambda W, seed: W.config_corner8(seed=seed)),
    "gauss8": ("gauss_product_d8_w0.01_1e9", lambda W, seed: W.config_gauss8(seed=seed)),
    "symmetric8": ("symmetric_corner_peak_d8_1e9", lambda W, seed: W.config_symmetric8(seed=seed)),
}


def _oracle_block(job):
    """One worker of the CPU baseline: the oracle's V-Sample over sub-cubes
    [t0, t1) of iteration `it` on `grid`; returns (I, var, histogram or None, s)."""
    prob, it, grid, t0, t1, hist = job
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    t = time.perf_counter()
    r = O.vsample(prob, it, grid, t0, t1, hist=hist)
    return r["I"], r["var"], r["hist"], time.perf_counter() - t


def _host_cpus():
    """(CPUs this process may run on, CPUs the host reports, CPU model)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return usable, os.cpu_count() or usable, model


def cpu_baseline(prob, target_s: float = 6.0, max_workers: int = 16, tau_rel: float = 1e-3):
    """Times the FP64 oracle on this host: one core on a bounded block of
    sub-cubes (iteration 0, uniform grid, histogram on), then one V-Sample pass
    over all sub-cubes split into one block per worker process, and a whole
    run to tau_rel relative error in the same way (each iteration's blocks
    merged in block order, then the oracle's own weighting and bin adjustment
    and the convergence test of the library).  Workers: the CPUs this process
    may use, at most max_workers (the share of a host that one GPU's job gets).
    Runs before the GPU is touched, so the workers fork from a process without
    device state."""
    import multiprocessing as mp

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    d, nb = prob["dim"], prob["nbins"]
    g, m, p = O.shape(d, prob["maxcalls"])
    grid0 = O.init_grid(d, nb)
    n = min(m, 20_000)
    dt = _oracle_block((prob, 0, grid0, 0, n, True))[3]
    n1 = int(min(m, max(n, n * target_s / max(dt, 1e-6))))
    dt1 = _oracle_block((prob, 0, grid0, 0, n1, True))[3]
    usable, reported, model = _host_cpus()
    workers = max(1, min(usable, max_workers))
    cuts = [m * k // workers for k in range(workers + 1)]

    def one_pass(pool, it, grid, hist):
        jobs = [(prob, it, grid, cuts[k], cuts[k + 1], hist) for k in range(workers)]
        parts = pool.map(_oracle_block, jobs)
        I = math.fsum(r[0] for r in parts)
        V = math.fsum(r[1] for r in parts)
        H = None
        if hist:
            H = np.zeros(d * nb)
            for r in parts:
                H = H + r[2]
        return I, V, H

    with mp.get_context("fork").Pool(workers) as pool:
        t = time.perf_counter()
        one_pass(pool, 0, grid0, True)
        wall = time.perf_counter() - t
        # time to tau_rel: the oracle's steps of Alg. 2, each pass spread over the workers
        run = dict(prob, tau_rel=tau_rel)
        t = time.perf_counter()
        grid, Is, Vs, conv = grid0, [], [], False
        for it in range(run["itmax"]):
            adjust = it < run["ita"]
            I, V, H = one_pass(pool, it, grid, adjust)
            Is.append(I)
            Vs.append(V)
            est, err, chi2 = O.weighted(Is, Vs)
            if adjust:
                grid = O.refine(d, nb, run["alpha"], H, grid)
            if len(Is) >= 2 and err <= tau_rel * abs(est) and chi2 <= 5.0:
                conv = True
                break
        t_target = time.perf_counter() - t
    return {"value": m * p / wall, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"one FP64 V-Sample pass of iteration 0 over all {m} sub-cubes ({m * p} samples, "
                      f"uniform grid, histogram on) split into {workers} blocks on {workers} processes: "
                      f"{wall:.2f} s wall; one core alone: {n1 * p} samples in {dt1:.1f} s",
            "single_core": n1 * p / dt1,
            "host": {"cpus_usable": usable, "cpus_reported": reported, "cpu_model": model},
            "time_to_1e-3": {"ms": t_target * 1e3, "iterations": len(Is), "converged": conv,
                             "estimate": est, "rel_error": err / abs(est) if est else None}}


def cpu_baseline_sample(prob, target_s: float = 4.0, max_workers: int = 16):
    """The FP64 oracle on a bounded sample of a configuration too large for a
    whole pass: one core on a block of sub-cubes (iteration 0, uniform grid,
    histogram on) for the per-core rate, then the first B sub-cubes, B sized
    from that rate for about target_s, split into one block per worker
    process.  Runs before the GPU is touched (fork)."""
    import multiprocessing as mp

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    d, nb = prob["dim"], prob["nbins"]
    g, m, p = O.shape(d, prob["maxcalls"])
    grid0 = O.init_grid(d, nb)
    n = min(m, 20_000)
    dt = _oracle_block((prob, 0, grid0, 0, n, True))[3]
    usable, reported, model = _host_cpus()
    workers = max(1, min(usable, max_workers))
    B = int(min(m, max(workers, n / max(dt, 1e-6) * workers * target_s)))
    cuts = [B * k // workers for k in range(workers + 1)]
    jobs = [(prob, 0, grid0, cuts[k], cuts[k + 1], True) for k in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        t = time.perf_counter()
        pool.map(_oracle_block, jobs)
        wall = time.perf_counter() - t
    return {"value": B * p / wall, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"one FP64 V-Sample pass of iteration 0 over the first {B} of the {m} sub-cubes "
                      f"({B * p} samples, uniform grid, histogram on) split into {workers} blocks on "
                      f"{workers} processes: {wall:.2f} s wall; one core alone: {n * p} samples in {dt * 1e3:.1f} ms",
            "single_core": n * p / dt,
            "host": {"cpus_usable": usable, "cpus_reported": reported, "cpu_model": model}}


def _base_line(args, name, value, ms_per_step, dtype, config):
    return {"metric": "integrand samples/sec/GPU", "value": value, "unit": "samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": dict({"workload": name}, **config)}


def bench_batch(args, M, W, torch):
    """4096 independent integrals run to completion together; one step = one
    whole batch (every integral's itmax iterations, one persistent launch per
    iteration)."""
    probs = W.config_batch(n=args.batch_size, precision=args.precision)
    ws = torch.empty(M.batch_workspace_bytes(probs), dtype=torch.uint8, device="cuda")
    bound = M.BatchProblems(probs)  # the problem descriptions, marshalled once
    for _ in range(args.warmup):
        M.batch_integrate(bound, ws=ws)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(M.batch_integrate(bound, ws=ws)[1])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    calls = sum(s.calls for s in stats)
    sample_s = sum(s.sample_ms for s in stats) / 1e3
    ops = 0.0
    for p in probs:
        gmp = M.shape(p["dim"], p["maxcalls"])
        per = slots_per_sample(p, gmp, adjust=True, fp32=p["precision"] == "fp32")
        ops += per * gmp[1] * gmp[2] * p["itmax"]
    ops *= args.steps
    line = _base_line(args, "batch_4096_mixed", calls / el, el / args.steps * 1e3,
                      "f64" if args.precision == "fp64" else "f32-eval/f64-accumulate",
                      {"integrals": len(probs), "dim": "U{2..10}", "maxcalls": "log-U[1e4,1e7]",
                       "nbins": "U{100..500}", "itmax": probs[0]["itmax"],
                       "integrands": "Gaussian product / corner peak",
                       "step": "one whole batch to completion (mc_batch_integrate)"})
    line["roofline"] = {"bound": "alu", "achieved": ops / sample_s / 1e12,
                        "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s", "op": SLOT_OP,
                        "frac": ops / sample_s / VALU_PEAK_OPS, "traffic": None,
                        "kernel": "vsample_batch_kernel",
                        "avg_launch_ms": sample_s / sum(s.steps for s in stats) * 1e3}
    line["kernel_samples_per_s"] = calls / sample_s
    line["steps_per_batch"] = stats[0].steps
    line["host_ms_per_batch"] = sum(s.host_ms for s in stats) / len(stats)
    print(json.dumps(line))


def _serve_stream(args, M, torch, arrivals, probs, budget):
    """Serves the Poisson stream once; returns (stats, wall s, latencies ms, failures)."""
    srv = M.Server(ws_bytes=args.serve_gib * 2**30, arena_bytes=args.serve_gib * 2**30 // 2,
                   max_active=8192)
    if budget:
        srv.set_step_budget(budget, args.max_skip)
    # warm-up: a few requests through the server before the clock starts
    for p in probs[:8]:
        srv.submit(dict(p, seed=p["seed"] + 10**6))
    while True:
        a, q, _ = srv.step()
        for rid in srv.finished():
            srv.release(rid)
        if a == 0 and q == 0:
            break
    torch.cuda.synchronize()
    base = srv.stats()
    done_at, ids = {}, {}
    nxt, n = 0, len(probs)
    t0 = time.perf_counter()
    while len(done_at) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            ids[srv.submit(probs[nxt])] = nxt
            nxt += 1
        if len(ids) > len(done_at):
            srv.step()
            t = time.perf_counter() - t0
            for rid in srv.finished():
                done_at[ids[rid]] = t
        elif nxt < n:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    el = time.perf_counter() - t0
    st = srv.stats()
    for f in ("calls", "steps", "sample_ms", "host_ms", "step_ms"):
        setattr(st, f, getattr(st, f) - getattr(base, f))
    lat = np.array([done_at[i] - arrivals[i] for i in range(n)]) * 1e3
    fails = 0
    for rid in list(ids):
        state, _, _ = srv.poll(rid)
        fails += state != M.REQ_DONE
    srv.close()
    return st, el, lat, fails


def bench_serve(args, M, W, torch):
    """A Poisson stream of requests served with continuous batching; reports
    samples/s over the run and p50/p99 time from arrival to answer, under the
    step budget (least remaining work first) and, for comparison, with every
    active request in every step."""
    arrivals, probs = W.served_requests(n=args.requests, rate=args.rate, precision=args.precision)
    runs = {}
    for budget in (args.step_budget, 0) if args.step_budget else (0,):
        runs[budget] = _serve_stream(args, M, torch, arrivals, probs, budget)
    st, el, lat, fails = runs[args.step_budget]
    n = len(probs)

    def summary(st, el, lat, fails):
        return {"samples_per_s": st.calls / el,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                               "mean": float(lat.mean()), "max": float(lat.max())},
                "failed": fails, "server_steps": st.steps, "max_active": st.max_active,
                "sampling_ms": st.sample_ms, "server_host_ms": st.host_ms,
                "server_step_ms": st.step_ms, "wall_ms": el * 1e3}

    line = _base_line(args, "served_poisson", st.calls / el, el * 1e3,
                      "f64" if args.precision == "fp64" else "f32-eval/f64-accumulate",
                      {"requests": n, "rate_per_s": args.rate, "dim": "U{3..10}",
                       "tau_rel": "log-U[1e-5,1e-2]", "maxcalls": "1e5/1e6/1e7 by target",
                       "nbins": 100, "step_budget_samples": args.step_budget,
                       "max_skip": args.max_skip, "step": "the whole served stream"})
    line["steps"] = 1
    s = summary(st, el, lat, fails)
    line["latency_ms"] = s.pop("latency_ms")
    s.pop("samples_per_s")
    line["served"] = s
    if args.step_budget:
        line["every_request_every_step"] = summary(*runs[0])
    print(json.dumps(line))


def measure_single(args, M, torch, prob, precision, steps, warmup, exact, profiled_here,
                   device_steps=True):
    """K full runs of one problem in one precision on a prepared workspace
    (inputs resident, no per-kernel timing: the throughput), then K more with
    the library's HIP-event timing (the sampling kernel's launch time and
    roofline), and the wall time of one run to a 1e-3 relative error (the
    median of five, after one untimed run)."""
    p = dict(prob, precision=precision, device_steps=device_steps)
    bp = M.BoundProblem(p, args.blocks, args.threads)
    ws = M.Workspace(bp)
    M.prepare(p, ws, bp=bp)

    def run(seed, **kw):
        p["seed"] = bp.s.seed = seed
        return M.integrate(p, ws=ws, bp=bp, prepared=True, **kw)

    for w in range(warmup):
        run(1000 + w)
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for k in range(steps):
        res.append(run(1 + k))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = [run(1 + k, timing=True) for k in range(steps)]
    gmp = M.shape(p["dim"], p["maxcalls"])
    calls_per_iter = gmp[1] * gmp[2]
    launches = sum(r.iterations for r in timed)
    avg_launch_s = sum(r.sample_ms for r in timed) / launches / 1e3
    fp32 = precision == "fp32"
    ops = ops_per_sample(p, gmp, adjust=p["ita"] > 0, fp32=fp32)
    slots = slots_per_sample(p, gmp, adjust=p["ita"] > 0, fp32=fp32)
    achieved = slots * calls_per_iter / avg_launch_s
    r0 = timed[0]
    prof = (profiled(precision) if profiled_here else None) or {}
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
            "unit": "TOP/s", "op": SLOT_OP, "frac": achieved / VALU_PEAK_OPS, "traffic": prof.get("traffic"),
            "kernel": "vsample_kernel" + (" (FP32-eval)" if fp32 else ""),
            "avg_launch_ms": avg_launch_s * 1e3, "ops_per_sample": ops, "slots_per_sample": slots,
            "launch": {"blocks": r0.blocks, "threads": r0.threads, "lds_bytes": r0.lds_bytes}}
    if "valu_insts_per_sample" in prof:
        # the compiled kernel's own instruction count (rocprofv3 SQ_INSTS_VALU)
        # and its wave instructions x 4 cycles over the busy cycles (what the
        # VALU would be occupied if every instruction took a full slot)
        roof["measured"] = {
            "valu_insts_per_sample": prof["valu_insts_per_sample"],
            "valu_issue_ratio": prof["valu_issue_ratio"],
            "valu_lane_insts_per_s": prof["valu_insts_per_sample"] * calls_per_iter / avg_launch_s / 1e12}

    # time to 1e-3 relative error, on a workspace of its own
    pt = dict(p, tau_rel=1e-3, seed=77)
    bpt = M.BoundProblem(pt, args.blocks, args.threads)
    wst = M.Workspace(bpt)
    M.prepare(pt, wst, bp=bpt)
    M.integrate(pt, ws=wst, bp=bpt, prepared=True)
    torch.cuda.synchronize()
    walls = []
    for _ in range(5):
        t = time.perf_counter()
        rt = M.integrate(pt, ws=wst, bp=bpt, prepared=True)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t)
    tt = sorted(walls)[len(walls) // 2]
    return {"value": sum(r.calls for r in res) / elapsed, "unit": "samples/s",
            "ms_per_step": elapsed / steps * 1e3, "calls_per_iter": calls_per_iter,
            "kernel_samples_per_s": calls_per_iter / avg_launch_s,
            "finalize_ms_per_iter": sum(r.finalize_ms for r in timed) / launches,
            "roofline": roof,
            "time_to_1e-3": {"ms": tt * 1e3, "min_ms": min(walls) * 1e3, "runs": len(walls),
                             "iterations": rt.iterations, "converged": rt.converged,
                             "estimate": rt.estimate,
                             "rel_error": rt.error / abs(rt.estimate) if rt.estimate else None,
                             "chi2_dof": rt.chi2_dof,
                             "true_rel_error": abs(rt.estimate - exact) / abs(exact)},
            "first": r0, "first_estimate": (r0.estimate, r0.error)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tables", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-corner8", action="store_true",
                    help="tables workload: skip the d = 8 corner-peak entry")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="evaluation precision for the batch and serve workloads")
    ap.add_argument("--batch-size", type=int, default=4096)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--serve-gib", type=int, default=16)
    ap.add_argument("--step-budget", type=int, default=200_000_000,
                    help="serve: samples per server step, least remaining work first (0: no budget)")
    ap.add_argument("--max-skip", type=int, default=8,
                    help="serve: steps a request may be left out in a row under the budget")
    ap.add_argument("--host-steps", action="store_true",
                    help="run the steps between sampling passes on the host for every figure")
    ap.add_argument("--one-d", action="store_true",
                    help="the m-Cubes1D variant (one shared grid; for symmetric integrands)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nbytes = 256 * 1024 * 1024
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_each_way": nbytes, "dispatches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    cpu = None
    if args.workload in WORKLOADS and WORKLOADS[args.workload][1] is not None and not args.no_cpu_baseline:
        from paper_2202_01753_amd import workloads as W0
        cpu = cpu_baseline(WORKLOADS[args.workload][1](W0, 1))
    cpu8 = None
    if args.workload == "tables" and not args.no_corner8 and not args.no_cpu_baseline:
        from paper_2202_01753_amd import workloads as W0
        cpu8 = cpu_baseline_sample(W0.config_corner8(seed=1))

    import torch

    from paper_2202_01753_amd import mcubes as M
    from paper_2202_01753_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args, M, W, torch)
    if args.workload == "serve":
        return bench_serve(args, M, W, torch)
    name, make = WORKLOADS[args.workload]
    prob = make(W, 1)
    if args.one_d:
        prob["one_d"] = True
        name += "_1d"
    # where the profile summary (traffic, measured VALU figures) was taken
    on_tables = args.workload == "tables" and not args.one_d
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import closed_forms as CF

    dev = not args.host_steps
    m64 = measure_single(args, M, torch, prob, "fp64", args.steps, args.warmup, CF.exact(prob),
                         on_tables, dev)
    m32 = measure_single(args, M, torch, prob, "fp32", args.steps, args.warmup, CF.exact(prob),
                         on_tables, dev)
    host_steps = {}
    if dev:
        # the same runs with the steps between passes on the host
        for prec, key in (("fp64", "fp64"), ("fp32", "fp32_eval")):
            h = measure_single(args, M, torch, prob, prec, args.steps, args.warmup, CF.exact(prob),
                               False, False)
            host_steps[key] = {"value": h["value"], "ms_per_step": h["ms_per_step"],
                               "time_to_1e-3_ms": h["time_to_1e-3"]["ms"]}
    r0 = m64.pop("first")
    m32.pop("first")
    first32 = m32.pop("first_estimate")
    m64.pop("first_estimate")
    m32["vs_fp64_same_seed"] = {
        "rel_diff": (first32[0] - r0.estimate) / abs(r0.estimate),
        "in_sigma": (first32[0] - r0.estimate) / math.hypot(first32[1], r0.error)}
    line = {
        "metric": "integrand samples/sec/GPU",
        "value": m64.pop("value"),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m64.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "dim": prob["dim"], "maxcalls": prob["maxcalls"],
                   "calls_per_iter": m64["calls_per_iter"], "nbins": prob["nbins"],
                   "itmax": prob["itmax"], "alpha": prob["alpha"],
                   "step": "one full m-Cubes run (mc_integrate_prepared, inputs resident)",
                   "steps_between_passes": "device" if dev else "host"},
    }
    line.update(m64)
    if args.workload == "small":
        # about 1e4 samples per pass: launch and host latency, not the kernel's
        # arithmetic, set the pace, so the fraction says little here
        line["per_iteration_ms"] = line["ms_per_step"] / prob["itmax"]
        line["roofline"]["note"] = ("1e4 samples per pass: launch and host latency dominate; "
                                    "the fraction is not meaningful for this configuration")
    line["estimate"] = {"value": r0.estimate, "error": r0.error, "chi2_dof": r0.chi2_dof,
                        "exact": CF.exact(prob)}
    line["fp32_eval"] = m32
    if host_steps:
        line["host_steps"] = host_steps
    if args.workload == "tables" and not args.no_corner8:
        # the largest single-GPU configuration beside it: d = 8 corner peak at
        # 1e9 samples per iteration, 20 iterations, in both precisions
        c8 = W.config_corner8(seed=1)
        k = max(1, min(args.steps, 3))
        sub = {}
        for prec in ("fp64", "fp32"):
            r = measure_single(args, M, torch, c8, prec, k, 1, CF.exact(c8), False, dev)
            r.pop("first")
            r.pop("first_estimate")
            sub["fp64" if prec == "fp64" else "fp32_eval"] = r
        sub["config"] = {"dim": 8, "maxcalls": c8["maxcalls"], "calls_per_iter": sub["fp64"]["calls_per_iter"],
                         "nbins": c8["nbins"], "itmax": c8["itmax"], "steps": k}
        if cpu8 is not None:
            sub["cpu_baseline"] = cpu8
        line["corner_peak_d8_1e9"] = sub
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()

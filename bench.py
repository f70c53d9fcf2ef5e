"""Throughput of the m-Cubes VEGAS sampling path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload tables|corner8|gauss8|small|batch|serve] [--precision fp64|fp32]

One step is one complete m-Cubes run (mc_integrate_prepared: every
iteration of sampling kernel + fixed-order reduction + read-back + host
weighting, bin adjustment and convergence check) on the workload's synthetic
inputs; the workspace is allocated and the integrand's constants and tables
are uploaded (mc_prepare) before the timed region, so the inputs are resident
in device memory when it starts.  `value` is integrand samples per second
over the K timed steps (iterations * m * p per step).

The roofline entry is for the sampling kernel: its average launch duration
comes from HIP events recorded by the library on the launch stream, and its
algorithmic work is the per-sample VALU lane-operation count of the method's
steps (one issue slot per full-rate instruction), times the samples per launch,
against the chip's VALU issue rate.  The CPU baseline times the FP64 oracle on
bounded blocks of sub-cubes of the same workload, on one core and on one
process per host core (at most 16), before the GPU is used.
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

# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock at 2.4 GHz = VALU lane-op issue rate
# (a wave64 full-rate VALU instruction occupies a SIMD for 4 clocks).
CUS, LANES_PER_CU_CLK, CLOCK_HZ = 256, 64, 2.4e9
VALU_PEAK_OPS = CUS * LANES_PER_CU_CLK * CLOCK_HZ  # 3.93e13 lane-ops/s


PHILOX_BLOCK_OPS = 17 + 18


def ops_per_sample(prob: dict, g_m_p, adjust: bool, fp32: bool = False) -> float:
    """Algorithmic VALU lane-operations per sample of the FP64 path (or of the
    FP32-evaluation path with fp32 set).

    Counted from the method's steps at one issue slot per full-rate VALU
    instruction (measured on gfx950: 32x32->64 integer products, FP64 add/mul/
    fma and conversions all issue at the full rate; v_rcp_f64, v_rcp_f32 count
    4 and v_exp_f32 2; a three-input XOR is one v_bitop3_b32), with work that
    is uniform across the wavefront or invariant across a sub-cube's samples
    excluded:
                                FP64 path                      FP32 evaluation
      Philox4x32-10 block       17 products + 18 three-way XOR, ceil(d/2) blocks; ceil(d/4)
      per axis                  20: uniform 5, coordinate 2,   15: uniform 3, coordinate 2,
                                bin index and clamp 7, address bin index and clamp 5, address
                                and width 2, point 2,          1, point 2, Jacobian 2
                                Jacobian 2
      Gaussian product          3 per axis + exp 20            3 per axis + expf 10
      corner peak               d fma + binary powering +      d fma + powering +
                                division 13                    division 12
      two bilinear tables       2 x 21 + 2 products (on top of the Gaussian), both paths
      f J / (m p), finiteness   4                              6 (two widening conversions)
      shifted sums              3 (p-1)/p
      bin contributions         1 + d addresses (adjusting iterations; 1 + 1 in m-Cubes1D)
      per sub-cube, / p         variance 5, two compensated additions 14,
                                digit odometer 4 d, digit conversion d
    """
    d = int(prob["dim"])
    _, _, p = g_m_p
    kind = prob["integrand"]
    philox = math.ceil(d / (4 if fp32 else 2)) * PHILOX_BLOCK_OPS
    per_axis = (15 if fp32 else 20) * d
    expo, div = (10, 12) if fp32 else (20, 13)
    if kind == "const":
        f = 0
    elif kind == "gauss_product":
        f = 3 * d + expo
    elif kind == "corner_peak":
        e = d + 1
        f = d + (e.bit_length() - 1) + (bin(e).count("1") - 1) + div
    else:
        f = 3 * d + expo + 2 * 21 + 2
    axes = 1 if prob.get("one_d") else d  # histogram rows (m-Cubes1D: the first axis only)
    tail = (6 if fp32 else 4) + 3 * (p - 1) / p + ((1 + axes) if adjust else 0) + (19 + 5 * d) / p
    return float(philox + per_axis + f + tail)


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


def profiled_traffic(kind: str):
    """HBM bytes per launch of the tables kernel ('fp64' or 'fp32') from the
    profile summary, or None if absent or taken from other kernel sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"traffic-per-launch fp64=(\d+) fp32=(\d+) sources=([0-9a-f]{64})", text)
    if not m or m.group(3) != kernel_sources_digest():
        return None
    return int(m.group(1) if kind == "fp64" else m.group(2))


WORKLOADS = {
    "tables": ("gauss_tables_d6_1e8", lambda W, seed: W.config_tables(seed=seed)),
    "batch": ("batch_4096_mixed", None),
    "serve": ("served_poisson_2000_per_s", None),
    "small": ("gauss_product_d2_1e4", lambda W, seed: W.config_small(seed=seed)),
    "corner8": ("corner_peak_d8_1e9", lambda W, seed: W.config_corner8(seed=seed)),
    "gauss8": ("gauss_product_d8_w0.01_1e9", lambda W, seed: W.config_gauss8(seed=seed)),
    "symmetric8": ("symmetric_corner_peak_d8_1e9", lambda W, seed: W.config_symmetric8(seed=seed)),
}


def _oracle_pass(job):
    """One worker of the CPU baseline: the oracle's V-Sample over sub-cubes [t0, t1)."""
    prob, t0, t1 = job
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    grid = O.init_grid(prob["dim"], prob["nbins"])
    t = time.perf_counter()
    O.vsample(prob, 0, grid, t0, t1, hist=True)
    return time.perf_counter() - t


def cpu_baseline(prob, target_s: float = 6.0, max_workers: int = 16):
    """Times the oracle's V-Sample (iteration 0, uniform grid, histogram on) on
    the first sub-cubes of the workload: on one core, then on one process per
    host core (at most max_workers, each on its own block of sub-cubes).  Runs
    before the GPU is touched, so the worker processes fork from a process
    without device state."""
    import multiprocessing as mp

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    g, m, p = O.shape(prob["dim"], prob["maxcalls"])
    n = min(m, 20_000)
    dt = _oracle_pass((prob, 0, n))
    n1 = int(min(m, max(n, n * target_s / max(dt, 1e-6))))
    dt1 = _oracle_pass((prob, 0, n1))
    workers = max(1, min(os.cpu_count() or 1, max_workers))
    per = max(1, min(n1, m // workers))
    jobs = [(prob, k * per, (k + 1) * per) for k in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        t = time.perf_counter()
        pool.map(_oracle_pass, jobs)
        wall = time.perf_counter() - t
    return {"value": workers * per * p / wall, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"V-Sample passes of iteration 0 (uniform grid, histogram on): {workers} processes, "
                      f"each over {per} of the {m} sub-cubes ({workers * per * p} samples, {wall:.1f} s "
                      f"wall); one core alone: {n1 * p} samples in {dt1:.1f} s",
            "single_core": n1 * p / dt1}


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
        per = ops_per_sample(p, gmp, adjust=True, fp32=p["precision"] == "fp32")
        ops += per * gmp[1] * gmp[2] * p["itmax"]
    ops *= args.steps
    line = _base_line(args, "batch_4096_mixed", calls / el, el / args.steps * 1e3,
                      "f64" if args.precision == "fp64" else "f32-eval/f64-accumulate",
                      {"integrals": len(probs), "dim": "U{2..10}", "maxcalls": "log-U[1e4,1e7]",
                       "nbins": "U{100..500}", "itmax": probs[0]["itmax"],
                       "integrands": "Gaussian product / corner peak",
                       "step": "one whole batch to completion (mc_batch_integrate)"})
    line["roofline"] = {"bound": "alu", "achieved": ops / sample_s / 1e12,
                        "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tables", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    on_tables = args.workload == "tables" and not args.one_d  # where the traffic profile was taken
    prob = make(W, 1)
    if args.one_d:
        prob["one_d"] = True
        name += "_1d"
    bp = M.BoundProblem(prob, args.blocks, args.threads)
    ws = M.Workspace(bp)
    M.prepare(prob, ws, bp=bp)
    gmp = M.shape(prob["dim"], prob["maxcalls"])
    calls_per_iter = gmp[1] * gmp[2]
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import closed_forms as CF
    exact = CF.exact(prob)

    def step(seed):
        prob["seed"] = seed
        bp.s.seed = seed
        return M.integrate(prob, ws=ws, bp=bp, timing=True, prepared=True)

    for w in range(args.warmup):
        step(1000 + w)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        results.append(step(1 + k))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    calls = sum(r.calls for r in results)
    launches = sum(r.iterations for r in results)
    sample_ms = sum(r.sample_ms for r in results)
    fin_ms = sum(r.finalize_ms for r in results)
    avg_launch_s = sample_ms / launches / 1e3
    ops = ops_per_sample(prob, gmp, adjust=prob["ita"] > 0) * calls_per_iter
    achieved = ops / avg_launch_s
    r0 = results[0]

    def time_to_target(precision):
        """Wall time of one run to a 1e-3 relative error, after one untimed run."""
        pt = dict(prob, tau_rel=1e-3, precision=precision, seed=77)
        bpt = M.BoundProblem(pt, args.blocks, args.threads)
        wst = M.Workspace(bpt)
        M.prepare(pt, wst, bp=bpt)
        M.integrate(pt, ws=wst, bp=bpt, prepared=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = M.integrate(pt, ws=wst, bp=bpt, prepared=True)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    rt, tt = time_to_target("fp64")

    # the FP32-evaluation path on the same workload: throughput, time to 1e-3,
    # and its distance from the FP64 run with the same seed
    p32 = dict(prob, precision="fp32")
    bp32 = M.BoundProblem(p32, args.blocks, args.threads)
    ws32 = M.Workspace(bp32)
    M.prepare(p32, ws32, bp=bp32)
    for w in range(args.warmup):
        p32["seed"] = bp32.s.seed = 1000 + w
        M.integrate(p32, ws=ws32, bp=bp32, prepared=True)
    torch.cuda.synchronize()
    res32 = []
    t2 = time.perf_counter()
    for k in range(args.steps):
        p32["seed"] = bp32.s.seed = 1 + k
        res32.append(M.integrate(p32, ws=ws32, bp=bp32, timing=True, prepared=True))
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t2
    rt32, tt32 = time_to_target("fp32")
    k32 = sum(r.sample_ms for r in res32) / sum(r.iterations for r in res32) / 1e3
    ops32 = ops_per_sample(prob, gmp, adjust=prob["ita"] > 0, fp32=True) * calls_per_iter
    fp32_eval = {
        "value": sum(r.calls for r in res32) / el32, "unit": "samples/s",
        "ms_per_step": el32 / args.steps * 1e3, "kernel_samples_per_s": calls_per_iter / k32,
        "avg_launch_ms": k32 * 1e3,
        "roofline": {"bound": "alu", "achieved": ops32 / k32 / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": ops32 / k32 / VALU_PEAK_OPS,
                     "traffic": profiled_traffic("fp32") if on_tables else None,
                     "kernel": "vsample_kernel (FP32-eval)",
                     "ops_per_sample": ops32 / calls_per_iter},
        "time_to_1e-3": {"ms": tt32 * 1e3, "iterations": rt32.iterations,
                         "converged": rt32.converged, "estimate": rt32.estimate,
                         "rel_error": rt32.error / abs(rt32.estimate),
                         "true_rel_error": abs(rt32.estimate - exact) / abs(exact)},
        "vs_fp64_same_seed": {
            "rel_diff": (res32[0].estimate - results[0].estimate) / abs(results[0].estimate),
            "in_sigma": (res32[0].estimate - results[0].estimate)
                        / math.hypot(res32[0].error, results[0].error)},
    }

    line = {
        "metric": "integrand samples/sec/GPU",
        "value": calls / elapsed,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "dim": prob["dim"], "maxcalls": prob["maxcalls"],
                   "calls_per_iter": calls_per_iter, "nbins": prob["nbins"],
                   "itmax": prob["itmax"], "alpha": prob["alpha"],
                   "step": "one full m-Cubes run (mc_integrate_prepared, inputs resident)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": profiled_traffic("fp64") if on_tables else None,
                     "kernel": "vsample_kernel", "avg_launch_ms": avg_launch_s * 1e3,
                     "ops_per_sample": ops / calls_per_iter,
                     "launch": {"blocks": r0.blocks, "threads": r0.threads,
                                "lds_bytes": r0.lds_bytes}},
        "kernel_samples_per_s": calls_per_iter / avg_launch_s,
        "finalize_ms_per_iter": fin_ms / launches,
        "time_to_1e-3": {"ms": tt * 1e3, "iterations": rt.iterations, "converged": rt.converged,
                         "estimate": rt.estimate, "rel_error": rt.error / abs(rt.estimate),
                         "true_rel_error": abs(rt.estimate - exact) / abs(exact)},
        "estimate": {"value": r0.estimate, "error": r0.error, "chi2_dof": r0.chi2_dof,
                     "exact": exact},
        "fp32_eval": fp32_eval,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()

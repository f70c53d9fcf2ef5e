"""Python binding of libmcubes (the C ABI in include/mcubes.h).

Argument marshalling only: every step of the sampling pass runs in the HIP
kernels of libmcubes.so, and the per-iteration host steps run in its C++
driver.  PyTorch provides the device workspace and the stream.  There is no
fallback: if the library is missing, loading it raises.

Problems are the dicts produced by ``paper_2202_01753_amd.workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libmcubes.so")

OK, EINVAL, EWORKSPACE, ENONFINITE, EDEVICE = 0, 1, 2, 3, 4
INTEGRANDS = {"const": 0, "gauss_product": 1, "corner_peak": 2, "gauss_tables": 3}
PRECISIONS = {"fp64": 0, "fp32": 1}
MC_MAX_DIM = 16
MC_DEVICE_STEPS_MAX_BINS = 4000  # bins per axis up to which device_steps keeps the steps on the device
EXPORTS = ("mc_status_string", "mc_shape", "mc_workspace_bytes", "mc_launch_shape", "mc_prepare",
           "mc_sample_iteration", "mc_refine_grid", "mc_refine_grid_1d", "mc_refine_grid_device",
           "mc_init_grid",
           "mc_weighted_estimate", "mc_integrate", "mc_integrate_prepared", "mc_integrate_noalloc",
           "mc_batch_workspace_bytes", "mc_batch_integrate", "mc_server_create",
           "mc_server_set_step_budget", "mc_server_submit", "mc_server_step", "mc_server_poll", "mc_server_finished",
           "mc_server_release", "mc_server_stats", "mc_server_destroy")
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class MCubesError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: status {code} ({status_string(code)})")


class Problem(C.Structure):
    _fields_ = [
        ("integrand", C.c_int32),
        ("dim", C.c_int32),
        ("params", C.POINTER(C.c_double)),
        ("n_params", C.c_int64),
        ("tables", C.POINTER(C.c_double)),
        ("n_tables", C.c_int64),
        ("lo", C.POINTER(C.c_double)),
        ("hi", C.POINTER(C.c_double)),
        ("maxcalls", C.c_int64),
        ("nbins", C.c_int32),
        ("itmax", C.c_int32),
        ("ita", C.c_int32),
        ("precision", C.c_int32),
        ("alpha", C.c_double),
        ("tau_rel", C.c_double),
        ("seed", C.c_uint64),
        ("blocks", C.c_int32),
        ("threads", C.c_int32),
        ("one_d", C.c_int32),
        ("chi2_max", C.c_double),
        ("device_steps", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("error", C.c_double), ("chi2_dof", C.c_double),
                ("iterations", C.c_int32), ("converged", C.c_int32), ("calls", C.c_int64)]


class BatchStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("max_active", C.c_int32), ("sample_ms", C.c_double),
                ("step_ms", C.c_double), ("calls", C.c_int64), ("host_ms", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("sample_ms", C.c_double), ("finalize_ms", C.c_double), ("launches", C.c_int32),
                ("blocks", C.c_int32), ("threads", C.c_int32), ("lds_bytes", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Loads libmcubes.so from the package directory; raises if it is not built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; importing it first makes libmcubes bind
        # to that same runtime (one HIP runtime per process).
        import torch  # noqa: F401
        if not os.path.exists(LIBRARY):
            raise ImportError(f"{LIBRARY} is not built: run `python -m paper_2202_01753_amd.build`")
        L = C.CDLL(LIBRARY)
        dp, vp, sz = C.POINTER(C.c_double), C.c_void_p, C.c_size_t
        P = C.POINTER(Problem)
        sig = {
            "mc_status_string": ([C.c_int32], C.c_char_p),
            "mc_shape": ([C.c_int32, C.c_int64] + [C.POINTER(C.c_int64)] * 3, C.c_int32),
            "mc_workspace_bytes": ([P, C.POINTER(C.c_size_t)], C.c_int32),
            "mc_launch_shape": ([P, C.c_int32] + [C.POINTER(C.c_int32)] * 3, C.c_int32),
            "mc_prepare": ([P, vp, sz, vp], C.c_int32),
            "mc_sample_iteration": ([P, C.c_uint32, C.c_int32, dp, vp, sz, vp, dp, dp, vp, sz,
                                     C.c_int64, C.c_int64], C.c_int32),
            "mc_refine_grid": ([C.c_int32, C.c_int32, C.c_double, dp, dp], C.c_int32),
            "mc_refine_grid_1d": ([C.c_int32, C.c_int32, C.c_double, dp, dp], C.c_int32),
            "mc_refine_grid_device": ([C.c_int32, C.c_int32, C.c_double, C.c_int32, vp, vp, vp],
                                      C.c_int32),
            "mc_init_grid": ([C.c_int32, C.c_int32, dp], C.c_int32),
            "mc_weighted_estimate": ([C.c_int32, dp, dp, dp], C.c_int32),
            "mc_integrate": ([P, vp, sz, vp, C.POINTER(Result), dp, dp, C.POINTER(Timing)],
                             C.c_int32),
            "mc_integrate_prepared": ([P, vp, sz, vp, C.POINTER(Result), dp, dp,
                                       C.POINTER(Timing)], C.c_int32),
            "mc_integrate_noalloc": ([P, vp, C.POINTER(Result), dp, dp], C.c_int32),
            "mc_batch_workspace_bytes": ([P, C.c_int32, C.POINTER(C.c_size_t)], C.c_int32),
            "mc_batch_integrate": ([P, C.c_int32, vp, sz, vp, C.POINTER(Result),
                                    C.POINTER(C.c_int32), C.POINTER(BatchStats)], C.c_int32),
            "mc_server_create": ([vp, sz, sz, C.c_int32, vp, C.POINTER(vp)], C.c_int32),
            "mc_server_set_step_budget": ([vp, C.c_int64, C.c_int32], C.c_int32),
            "mc_server_submit": ([vp, P, C.POINTER(C.c_int64)], C.c_int32),
            "mc_server_step": ([vp] + [C.POINTER(C.c_int32)] * 3, C.c_int32),
            "mc_server_poll": ([vp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(Result),
                                C.POINTER(C.c_int32)], C.c_int32),
            "mc_server_finished": ([vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)],
                                   C.c_int32),
            "mc_server_release": ([vp, C.c_int64], C.c_int32),
            "mc_server_stats": ([vp, C.POINTER(BatchStats)], C.c_int32),
            "mc_server_destroy": ([vp], C.c_int32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().mc_status_string(code).decode()


def _check(code: int, what: str):
    if code != OK:
        raise MCubesError(code, what)


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class BoundProblem:
    """An mc_problem struct plus the host arrays it points into."""

    def __init__(self, prob: dict, blocks: int = 0, threads: int = 0):
        self.src = prob
        self.params = _f64(prob["params"])
        self.tables = _f64(prob.get("tables"))
        self.lo = _f64(prob["lo"])
        self.hi = _f64(prob["hi"])
        self.s = Problem(
            integrand=INTEGRANDS[prob["integrand"]], dim=int(prob["dim"]), params=_dp(self.params),
            n_params=len(self.params), tables=_dp(self.tables),
            n_tables=0 if self.tables is None else len(self.tables), lo=_dp(self.lo),
            hi=_dp(self.hi), maxcalls=int(prob["maxcalls"]), nbins=int(prob["nbins"]),
            itmax=int(prob["itmax"]), ita=int(prob.get("ita", prob["itmax"])),
            precision=PRECISIONS[prob.get("precision", "fp64")],
            alpha=float(prob["alpha"]), tau_rel=float(prob.get("tau_rel", 0.0)),
            seed=int(prob["seed"]) & (2**64 - 1), blocks=int(blocks), threads=int(threads),
            one_d=1 if prob.get("one_d", False) else 0, chi2_max=float(prob.get("chi2_max", 0.0)),
            device_steps=1 if prob.get("device_steps", False) else 0)

    @property
    def ref(self):
        return C.byref(self.s)


def shape(dim: int, maxcalls: int):
    g, m, p = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().mc_shape(dim, maxcalls, C.byref(g), C.byref(m), C.byref(p)), "mc_shape")
    return g.value, m.value, p.value


def workspace_bytes(bp: BoundProblem) -> int:
    n = C.c_size_t()
    _check(lib().mc_workspace_bytes(bp.ref, C.byref(n)), "mc_workspace_bytes")
    return n.value


def launch_shape(bp: BoundProblem, adjust: bool = True):
    """(workgroups, threads per workgroup, LDS bytes) of the sampling launch."""
    b, t, l = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().mc_launch_shape(bp.ref, 1 if adjust else 0, C.byref(b), C.byref(t), C.byref(l)),
           "mc_launch_shape")
    return b.value, t.value, l.value


def refine_grid(dim: int, nbins: int, alpha: float, hist, grid):
    out = _f64(grid).copy()
    h = _f64(hist)
    _check(lib().mc_refine_grid(dim, nbins, alpha, _dp(h), _dp(out)), "mc_refine_grid")
    return out


def refine_grid_1d(dim: int, nbins: int, alpha: float, hist, grid):
    out = _f64(grid).copy()
    h = _f64(hist)
    _check(lib().mc_refine_grid_1d(dim, nbins, alpha, _dp(h), _dp(out)), "mc_refine_grid_1d")
    return out


def refine_grid_device(dim: int, nbins: int, alpha: float, hist, grid, one_d: bool = False,
                       stream=None):
    """mc_refine_grid_device on copies of hist and grid in device memory;
    returns the adjusted grid (host)."""
    torch = _torch()
    h = torch.from_numpy(_f64(hist).copy()).to("cuda")
    g = torch.from_numpy(_f64(grid).copy()).to("cuda")
    torch.cuda.synchronize()
    _check(lib().mc_refine_grid_device(dim, nbins, alpha, 1 if one_d else 0, C.c_void_p(h.data_ptr()),
                                       C.c_void_p(g.data_ptr()), _stream(stream)),
           "mc_refine_grid_device")
    torch.cuda.synchronize()
    return g.cpu().numpy()


def init_grid(dim: int, nbins: int):
    g = np.zeros(dim * (nbins + 1))
    _check(lib().mc_init_grid(dim, nbins, _dp(g)), "mc_init_grid")
    return g


def weighted_estimate(I, var):
    I, var = _f64(I), _f64(var)
    out = np.zeros(3)
    _check(lib().mc_weighted_estimate(len(I), _dp(I), _dp(var), _dp(out)), "mc_weighted_estimate")
    return float(out[0]), float(out[1]), float(out[2])


# ---------------------------------------------------------------- device-side calls (torch)

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the m-Cubes sampling kernels need an MI355X")
    return torch


class Workspace:
    """Device workspace (a torch uint8 tensor) sized for one problem."""

    def __init__(self, bp: BoundProblem, device="cuda"):
        torch = _torch()
        self.nbytes = workspace_bytes(bp)
        self.tensor = torch.empty(self.nbytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.tensor.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class IntegrationResult:
    estimate: float
    error: float
    chi2_dof: float
    iterations: int
    converged: bool
    calls: int
    it_I: np.ndarray
    it_var: np.ndarray
    grid: np.ndarray
    sample_ms: float = 0.0
    finalize_ms: float = 0.0
    blocks: int = 0
    threads: int = 0
    lds_bytes: int = 0


def prepare(prob: dict, ws: Workspace, stream=None, bp: BoundProblem | None = None) -> None:
    """mc_prepare: uploads the problem's constants and tables into ws."""
    bp = bp or BoundProblem(prob)
    _check(lib().mc_prepare(bp.ref, ws.ptr, ws.nbytes, _stream(stream)), "mc_prepare")


def integrate(prob: dict, ws: Workspace | None = None, stream=None, blocks: int = 0,
              threads: int = 0, timing: bool = False, bp: BoundProblem | None = None,
              prepared: bool = False):
    """mc_integrate, or mc_integrate_prepared when prepared is set (ws then
    already holds this problem's constants and tables, see prepare())."""
    bp = bp or BoundProblem(prob, blocks, threads)
    if prepared and ws is None:
        raise ValueError("prepared=True needs the prepared workspace")
    ws = ws or Workspace(bp)
    d, nb, itmax = int(prob["dim"]), int(prob["nbins"]), int(prob["itmax"])
    res = Result()
    iters = np.zeros(2 * itmax)
    grid = np.zeros(d * (nb + 1))
    tm = Timing() if timing else None
    fn = lib().mc_integrate_prepared if prepared else lib().mc_integrate
    _check(fn(bp.ref, ws.ptr, ws.nbytes, _stream(stream), C.byref(res), _dp(iters),
              _dp(grid), C.byref(tm) if tm is not None else None), "mc_integrate")
    k = res.iterations
    out = IntegrationResult(res.estimate, res.error, res.chi2_dof, k, bool(res.converged),
                            res.calls, iters[0:2 * k:2].copy(), iters[1:2 * k:2].copy(), grid)
    if tm is not None:
        out.sample_ms, out.finalize_ms = tm.sample_ms, tm.finalize_ms
        out.blocks, out.threads, out.lds_bytes = tm.blocks, tm.threads, tm.lds_bytes
    return out


def integrate_noalloc(prob: dict, stream=None, bp: BoundProblem | None = None):
    """mc_integrate_noalloc: the whole run in the library's device scratch array
    (no workspace, nothing allocated by the call)."""
    bp = bp or BoundProblem(prob)
    d, nb, itmax = int(prob["dim"]), int(prob["nbins"]), int(prob["itmax"])
    res = Result()
    iters = np.zeros(2 * itmax)
    grid = np.zeros(d * (nb + 1))
    _check(lib().mc_integrate_noalloc(bp.ref, _stream(stream), C.byref(res), _dp(iters), _dp(grid)),
           "mc_integrate_noalloc")
    k = res.iterations
    return IntegrationResult(res.estimate, res.error, res.chi2_dof, k, bool(res.converged),
                             res.calls, iters[0:2 * k:2].copy(), iters[1:2 * k:2].copy(), grid)


class Sampler:
    """Step-level access: one prepared workspace, one sampling pass per call."""

    def __init__(self, prob: dict, blocks: int = 0, threads: int = 0, stream=None):
        self.prob = prob
        self.bp = BoundProblem(prob, blocks, threads)
        self.ws = Workspace(self.bp)
        self.stream = stream
        self.d, self.nb = int(prob["dim"]), int(prob["nbins"])
        self.g, self.m, self.p = shape(self.d, int(prob["maxcalls"]))
        _check(lib().mc_prepare(self.bp.ref, self.ws.ptr, self.ws.nbytes, _stream(stream)),
               "mc_prepare")

    def sample(self, it: int, grid, adjust: bool = True, trace_range=None):
        """Returns dict(I, var, hist, strace, ctrace) like the oracle's vsample."""
        torch = _torch()
        grid = _f64(grid)
        out = np.zeros(2)
        hist = np.zeros(self.d * self.nb) if adjust else None
        tr, t0, t1, nbytes = None, 0, 0, 0
        if trace_range is not None:
            t0, t1 = trace_range
            rec = 3 * self.d + 2
            n = (t1 - t0) * self.p * rec + 2 * (t1 - t0)
            tr = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device=self.ws.tensor.device)
            nbytes = n * 8
        code = lib().mc_sample_iteration(
            self.bp.ref, it, 1 if adjust else 0, _dp(grid), self.ws.ptr, self.ws.nbytes,
            _stream(self.stream), _dp(out), _dp(hist),
            C.c_void_p(tr.data_ptr()) if tr is not None else None, nbytes, t0, t1)
        res = {"I": float(out[0]), "var": float(out[1]), "hist": hist, "strace": None,
               "ctrace": None, "status": code}
        if code not in (OK, ENONFINITE):
            _check(code, "mc_sample_iteration")
        if tr is not None and code == OK:
            a = tr.cpu().numpy()
            ns = (t1 - t0) * self.p
            res["strace"] = a[:ns * rec].reshape(ns, rec)
            res["ctrace"] = a[ns * rec:ns * rec + 2 * (t1 - t0)].reshape(t1 - t0, 2)
        return res


# ---------------------------------------------------------------- batches and serving

def _problem_array(bps):
    arr = (Problem * len(bps))()
    for i, bp in enumerate(bps):
        arr[i] = bp.s
    return arr


def batch_workspace_bytes(probs) -> int:
    bps = [BoundProblem(p) for p in probs]
    n = C.c_size_t()
    _check(lib().mc_batch_workspace_bytes(_problem_array(bps), len(bps), C.byref(n)),
           "mc_batch_workspace_bytes")
    return n.value


class BatchProblems:
    """The mc_problem array of a batch and the host arrays it points into,
    built once and reusable across batch_integrate calls."""

    def __init__(self, probs):
        self.bps = [BoundProblem(p) for p in probs]
        self.arr = _problem_array(self.bps)
        self.n = len(self.bps)


def batch_integrate(probs, stream=None, ws=None):
    """Runs the problems (a list of problem dicts or a BatchProblems) together;
    returns (list of result dicts or MCubesError per integral, BatchStats)."""
    torch = _torch()
    bp = probs if isinstance(probs, BatchProblems) else BatchProblems(probs)
    arr, n = bp.arr, bp.n
    need = C.c_size_t()
    _check(lib().mc_batch_workspace_bytes(arr, n, C.byref(need)), "mc_batch_workspace_bytes")
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    res = (Result * n)()
    sts = (C.c_int32 * n)()
    stats = BatchStats()
    _check(lib().mc_batch_integrate(arr, n, C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                    res, sts, C.byref(stats)), "mc_batch_integrate")
    out = []
    for i in range(n):
        if sts[i] != OK:
            out.append(MCubesError(sts[i], f"integral {i}"))
        else:
            r = res[i]
            out.append({"estimate": r.estimate, "error": r.error, "chi2_dof": r.chi2_dof,
                        "iterations": r.iterations, "converged": bool(r.converged),
                        "calls": r.calls})
    return out, stats


class Server:
    """Continuous-batching server (mc_server_*) on a torch-allocated workspace."""

    def __init__(self, ws_bytes: int, arena_bytes: int, max_active: int = 8192, stream=None):
        torch = _torch()
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream
        h = C.c_void_p()
        _check(lib().mc_server_create(C.c_void_p(self.ws.data_ptr()), ws_bytes, arena_bytes,
                                      max_active, _stream(stream), C.byref(h)), "mc_server_create")
        self.h = h
        self._keep = {}

    def set_step_budget(self, samples: int, max_skip: int = 8):
        """At most `samples` integrand samples per step, least remaining work
        first; a request waits at most `max_skip` steps (0 samples: no limit)."""
        _check(lib().mc_server_set_step_budget(self.h, int(samples), int(max_skip)),
               "mc_server_set_step_budget")

    def submit(self, prob) -> int:
        bp = BoundProblem(prob)
        rid = C.c_int64()
        _check(lib().mc_server_submit(self.h, bp.ref, C.byref(rid)), "mc_server_submit")
        return rid.value

    def step(self):
        a, q, f = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().mc_server_step(self.h, C.byref(a), C.byref(q), C.byref(f)), "mc_server_step")
        return a.value, q.value, f.value

    def poll(self, rid: int):
        st, status = C.c_int32(), C.c_int32()
        r = Result()
        _check(lib().mc_server_poll(self.h, rid, C.byref(st), C.byref(r), C.byref(status)),
               "mc_server_poll")
        res = None
        if st.value == REQ_DONE:
            res = {"estimate": r.estimate, "error": r.error, "chi2_dof": r.chi2_dof,
                   "iterations": r.iterations, "converged": bool(r.converged), "calls": r.calls}
        return st.value, res, status.value

    def finished(self, cap: int = 65536):
        """Ids of the requests that finished in the last step."""
        ids = (C.c_int64 * cap)()
        n = C.c_int32()
        _check(lib().mc_server_finished(self.h, ids, cap, C.byref(n)), "mc_server_finished")
        return list(ids[:n.value])

    def release(self, rid: int):
        _check(lib().mc_server_release(self.h, rid), "mc_server_release")

    def stats(self) -> BatchStats:
        s = BatchStats()
        _check(lib().mc_server_stats(self.h, C.byref(s)), "mc_server_stats")
        return s

    def close(self):
        if self.h:
            _check(lib().mc_server_destroy(self.h), "mc_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

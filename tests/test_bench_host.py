"""Host-side logic of bench.py, on the CPU: the op model's per-sample counts,
the source digest that gates the recorded HBM traffic, and the refusal of
more than one GPU."""
import importlib.util
import os
import subprocess
import sys

from paper_2202_01753_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
B = importlib.util.module_from_spec(_spec)
sys.modules["bench_host"] = B  # worker processes look the module up by name
_spec.loader.exec_module(B)


def test_op_model_tables_workload():
    # d = 6 Gaussian x two tables, g = 19, p = 2: 3 Philox blocks (FP64) or 2
    # (FP32-eval), 16 / 14 operations per axis, the integrand, and the tail
    prob = W.config_tables()
    shape = (19, 19 ** 6, 2)
    assert B.op_mix(prob, shape, adjust=True) == {"full": 249.0, "half": 72.0}
    assert B.ops_per_sample(prob, shape, adjust=True) == 321.0
    assert B.slots_per_sample(prob, shape, adjust=True) == 249.0 + 72.0 / 2
    mix32 = B.op_mix(prob, shape, adjust=True, fp32=True)
    assert mix32 == {"full": 93.0, "half": 153.0, "fma32": 14.0, "exp32": 1.0}
    assert B.slots_per_sample(prob, shape, adjust=True, fp32=True) == 93 + 153 / 2 + 14 * 0.875 + 2.5
    # No-Adjust drops the 1 + d histogram addresses
    assert B.ops_per_sample(prob, shape, adjust=False) == 321.0 - 7


def test_op_model_corner_peak_d8():
    # 4 / 2 Philox blocks; d fma, x^9 by three squarings and one product, one
    # correctly rounded division (one reciprocal in it)
    prob = W.config_corner8()
    shape = (12, 12 ** 8, 2)
    mix = B.op_mix(prob, shape, adjust=True)
    assert mix["rcp64"] == 1.0
    assert B.ops_per_sample(prob, shape, adjust=True) == 339.0
    mix32 = B.op_mix(prob, shape, adjust=True, fp32=True)
    assert mix32["rcp32"] == 1.0 and "rcp64" not in mix32
    # every slot cost is positive and at most a quarter-rate instruction's
    assert all(0 < c <= 4 for c in B.SLOT_COST.values())
    # the peak is the 64-bit-class issue rate of 256 CUs at 2.4 GHz
    assert B.VALU_PEAK_OPS == 256 * 64 * 2.4e9


def test_op_model_one_d_keeps_one_histogram_row():
    prob = W.config_symmetric8()
    shape = (12, 12 ** 8, 2)
    sep = B.ops_per_sample(prob, shape, adjust=True)
    one = B.ops_per_sample(dict(prob, one_d=1), shape, adjust=True)
    assert sep - one == 8 - 1


def test_digest_ignores_comments_and_sees_code():
    base = {}
    for rel in B.KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            base[rel] = f.read()
    d0 = B.kernel_sources_digest(read=base.__getitem__)
    assert d0 == B.kernel_sources_digest()
    cpp = next(r for r in B.KERNEL_SOURCES if r.endswith(".hpp"))
    py = next(r for r in B.KERNEL_SOURCES if r.endswith(".py"))
    edited = dict(base)
    edited[cpp] += "\n// a note\n/* another\n   note */\n"
    edited[py] += "\n# a note\n"
    assert B.kernel_sources_digest(read=edited.__getitem__) == d0
    edited[cpp] += "\nstatic int extra;\n"
    assert B.kernel_sources_digest(read=edited.__getitem__) != d0


def test_profiled_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profile.md"
    monkeypatch.setattr(B, "TRAFFIC_PROFILE", str(prof))
    assert B.profiled_traffic("fp64") is None  # no profile
    prof.write_text(f"traffic-per-launch fp64=123 fp32=45 sources={B.kernel_sources_digest()}\n")
    assert (B.profiled_traffic("fp64"), B.profiled_traffic("fp32")) == (123, 45)
    prof.write_text("traffic-per-launch fp64=123 fp32=45 sources=" + "0" * 64 + "\n")
    assert B.profiled_traffic("fp64") is None  # taken from other kernel code


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_sample_times_a_bounded_block():
    """The CPU leg for a configuration too large for a whole pass: the first B
    sub-cubes over worker processes, B sized from the per-core rate."""
    prob = W.corner_peak(4, 3, maxcalls=2_000_000, nbins=50, itmax=2)
    r = B.cpu_baseline_sample(prob, target_s=0.05, max_workers=2)
    assert r["kind"] == "oracle" and r["value"] > 0 and 1 <= r["cores"] <= 2
    assert "sub-cubes" in r["sample"] and r["single_core"] > 0


def test_cpu_baseline_runs_the_oracle_on_the_host():
    """The CPU leg on the small configuration: a pass over all sub-cubes split
    across worker processes, a run to 1e-3, and the host's CPUs recorded."""
    prob = W.config_small(seed=1)
    r = B.cpu_baseline(prob, target_s=0.1, max_workers=4)
    assert r["kind"] == "oracle" and r["value"] > 0 and 1 <= r["cores"] <= 4
    assert r["host"]["cpus_usable"] >= 1 and r["host"]["cpu_model"]
    t = r["time_to_1e-3"]
    assert t["converged"] and t["iterations"] >= 2 and t["rel_error"] <= 1e-3

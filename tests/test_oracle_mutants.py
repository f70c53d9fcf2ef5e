"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of the oracle's C source (in a temporary directory, never
in oracle/), builds it, and runs the pins that should catch it against the
mutant in a fresh Python process; at least one must fail.  This checks the
pins, not the oracle."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCE = os.path.join(ROOT, "oracle", "mcubes_oracle.c")

# (name, text in the oracle, replacement, pins expected to catch it (-k expression))
MUTANTS = [
    ("jacobian without the span", "J = J * (width * q[j]);", "J = J * (width * (double)nb);",
     "dyadic_grid_is_identity"),
    ("clamped last bin with fraction 0", "            i = nb - 1;\n            frac = 1.0;",
     "            i = nb - 1;\n            frac = 0.0;", "continuous_at_the_ends"),
    ("variance over p", "double vt = num * inv_pm1;", "double vt = num / pd;", "variance_calibrated"),
    ("cube sum without p I0", "double It = fma(pd, I0, S1);", "double It = S1 + I0;", "constant_integrand_exact"),
    ("corner-peak power d", "S = fma(params[j], x[j], S);\n    unsigned e = (unsigned)(d + 1);",
     "S = fma(params[j], x[j], S);\n    unsigned e = (unsigned)(d);",
     "corner_peak_integrand_quadrature"),
    ("Gaussian exp(-acc/2)", "    return exp(-acc);\n}", "    return exp(-0.5 * acc);\n}",
     "gaussian_product_integrand_quadrature"),
    ("table axes swapped", "    double along0 = lerp(t00, t10, tx);\n    double along1 = lerp(t01, t11, tx);",
     "    double along0 = lerp(t00, t01, tx);\n    double along1 = lerp(t10, t11, tx);", "table_integrand_nodes"),
    ("uniform X 2^-52", "    uint64_t odd = 2u * X + 1u;            /* < 2^53: exact in a double */\n"
     "    return (double)odd * 0x1p-53;", "    return (double)X * 0x1p-52;", "uniform_endpoints"),
    ("uniform from a mis-shifted low word", "uint64_t X = ((uint64_t)whi << 20) | (uint64_t)(wlo >> 12);",
     "uint64_t X = ((uint64_t)whi << 20) | (uint64_t)(wlo >> 11);", "uniform_endpoints"),
    ("no refinement", "        orc_weighted(k, Is, Vs, &Ibar, &sigma, &chi2);\n        if (adjust) {",
     "        orc_weighted(k, Is, Vs, &Ibar, &sigma, &chi2);\n        if (0) {", "integrate_closed_forms"),
    ("weights 1/sigma", "        double w = 1.0 / var[i];\n        W = W + w;",
     "        double w = 1.0 / sqrt(var[i]);\n        W = W + w;", "weighted_hand_cases"),
    ("chi2 over n", "chi / (double)(n - 1)", "chi / (double)(n)", "weighted_hand_cases"),
    ("compression without the exponent",
     "wt[i] = pow((1.0 - sm[i] / S) / log(S / sm[i]), alpha);", "wt[i] = (1.0 - sm[i] / S) / log(S / sm[i]);",
     "logarithmic_mean or damping_exponent"),
    ("compression with 1 + s/S",
     "wt[i] = pow((1.0 - sm[i] / S) / log(S / sm[i]), alpha);",
     "wt[i] = pow((1.0 + sm[i] / S) / log(S / sm[i]), alpha);", "logarithmic_mean"),
    ("compression with alpha / 2",
     "wt[i] = pow((1.0 - sm[i] / S) / log(S / sm[i]), alpha);",
     "wt[i] = pow((1.0 - sm[i] / S) / log(S / sm[i]), 0.5 * alpha);", "logarithmic_mean"),
    ("edge bin not smoothed", "sm[0] = (C[0] + C[1]) / 2.0;", "sm[0] = C[0];", "uniform_and_degenerate"),
    ("smoothing over 2", "sm[i] = ((C[i - 1] + C[i]) + C[i + 1]) / 3.0;", "sm[i] = ((C[i - 1] + C[i]) + C[i + 1]) / 2.0;",
     "uniform_and_degenerate or logarithmic_mean"),
    ("float uniform from 24 bits", "    uint32_t odd = 2u * (w >> 9) + 1u;", "    uint32_t odd = 2u * (w >> 8) + 1u;",
     "fp32 or uniform"),
    ("float table axes swapped", "return lerpf_(lerpf_(t00, t10, tx), lerpf_(t01, t11, tx), ty);",
     "return lerpf_(lerpf_(t00, t01, tx), lerpf_(t10, t11, tx), ty);", "fp32_eval_tracks"),
    ("float Gaussian exp(-acc/2)", "    float G = expf(-acc);", "    float G = expf(-0.5f * acc);", "fp32_eval_tracks"),
    ("float corner-peak power d", "S = fmaf(K->pa[j], x[j], S);\n        unsigned e = (unsigned)(d + 1);",
     "S = fmaf(K->pa[j], x[j], S);\n        unsigned e = (unsigned)(d);", "fp32_eval_tracks"),
    ("one adjusting iteration too many", "        int adjust = it < P->ita;\n        rc = orc_vsample",
     "        int adjust = it <= P->ita;\n        rc = orc_vsample", "resume_reproduces"),
]

_RUNNER = """
import sys
sys.path[:0] = [{oracle!r}, {root!r}, {tests!r}]
import oracle
oracle.LIBRARY = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", {pins!r}, "-k", {sel!r}]))
"""


@pytest.mark.parametrize("name,old,new,sel", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, sel):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    text = open(SOURCE).read()
    assert text.count(old) == 1, f"{name}: the oracle no longer has the text to mutate"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run([cc, "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", lib, str(src), "-lm"], check=True)
    runner = _RUNNER.format(oracle=os.path.join(ROOT, "oracle"), root=ROOT, tests=HERE, lib=lib,
                            pins=os.path.join(HERE, "test_oracle_pins.py"), sel=sel)
    out = subprocess.run([sys.executable, "-c", runner], capture_output=True, text=True, timeout=300)
    assert "passed" in out.stdout or "failed" in out.stdout, out.stdout + out.stderr
    assert out.returncode == 1, f"{name}: no pin failed\n{out.stdout[-2000:]}"

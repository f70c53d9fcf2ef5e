"""The oracle's pass spread over worker processes (tests/oracle_pool.py, used
by the GPU tests at the benchmark sizes) against one sequential call of the
oracle: the same estimate and variance up to the order of summation, the
same histogram."""
import numpy as np

import oracle as O
import oracle_pool as P
from paper_2202_01753_amd import workloads as W


def test_pooled_pass_matches_one_call():
    for precision in ("fp64", "fp32"):
        prob = W.config_tables(seed=4, maxcalls=400_000, itmax=3, precision=precision)
        rng = np.random.default_rng(3)
        grid = np.concatenate([np.concatenate([[0.0], np.sort(rng.random(499)), [1.0]]) for _ in range(6)])
        a = P.vsample(prob, 1, grid, hist=True, max_workers=4)
        b = O.vsample(prob, 1, grid, hist=True)
        assert abs(a["I"] - b["I"]) <= 1e-14 * abs(b["I"])
        assert abs(a["var"] - b["var"]) <= 1e-13 * b["var"]
        assert np.allclose(a["hist"], b["hist"], rtol=1e-13, atol=0)
        c = P.vsample(prob, 1, grid, hist=False, max_workers=3)
        assert c["hist"] is None and abs(c["I"] - b["I"]) <= 1e-14 * abs(b["I"])

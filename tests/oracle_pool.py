"""The oracle's V-Sample pass (Alg. 3) at full size, spread over worker
processes: the sub-cubes are cut into contiguous blocks, each block is one
call of the oracle, and the block totals and histograms are merged in block
order.  Only the order of summation differs from one sequential call (the
oracle sums each block with compensation; the merge of block totals is
correctly rounded), far inside the parity bars.

Test infrastructure: the workers are started fresh (spawn), so they load
numpy and the oracle only and never touch the GPU of the process that starts
them."""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

_PROB = None


def _init(prob):
    global _PROB
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    _PROB = prob


def _block(job):
    import oracle as O

    it, grid, t0, t1, hist = job
    r = O.vsample(_PROB, it, grid, t0, t1, hist=hist)
    return r["I"], r["var"], r["hist"]


def workers(max_workers: int = 16) -> int:
    """The CPUs this process may run on, at most max_workers (one GPU's share
    of the host)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return max(1, min(usable, max_workers))


def vsample(prob: dict, it: int, grid, hist: bool = True, max_workers: int = 16) -> dict:
    """{"I", "var", "hist"} of the oracle's whole pass over all m sub-cubes."""
    import multiprocessing as mp

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    d, nb = prob["dim"], prob["nbins"]
    _, m, _ = O.shape(d, prob["maxcalls"])
    w = workers(max_workers)
    nblk = min(m, 4 * w)
    cuts = [m * k // nblk for k in range(nblk + 1)]
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    jobs = [(it, grid, cuts[k], cuts[k + 1], hist) for k in range(nblk)]
    # a pool that raises (BrokenProcessPool) rather than waits if a worker dies
    from concurrent.futures import ProcessPoolExecutor

    with ProcessPoolExecutor(w, mp_context=mp.get_context("spawn"), initializer=_init,
                             initargs=(prob,)) as pool:
        parts = list(pool.map(_block, jobs))
    out = {"I": math.fsum(p[0] for p in parts), "var": math.fsum(p[1] for p in parts), "hist": None}
    if hist:
        H = np.zeros(d * nb)
        for p in parts:
            H = H + p[2]
        out["hist"] = H
    return out

"""CPU checks of the batch engine's host planning (no GPU): the work split
covers every integral exactly once in bounded pieces, the queue order is
largest first, and the workspace arena behaves as a first-fit allocator with
coalescing, compared with a plain Python model of one."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("plan") / "batch_plan_check")
    # built with the address and undefined-behaviour sanitizers where the
    # compiler has them, so that every check also runs the planning code
    # under them (host code only)
    src = os.path.join(HERE, "pins", "batch_plan_check.cpp")
    inc = ["-I", os.path.join(ROOT, "paper_2202_01753_amd", "csrc")]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    if subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", *san, *inc, src, "-o", exe]).returncode != 0:
        subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", *inc, src, "-o", exe], check=True)
    return exe


def _run(exe, text):
    return subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout


def _split(exe, m, cost, parts):
    text = f"split {len(m)} {parts}\n" + "".join(f"{a} {c!r}\n" for a, c in zip(m, cost))
    pieces, first = [], {}
    for line in _run(exe, text).splitlines():
        t = line.split()
        if t[0] == "piece":
            pieces.append((int(t[1]), int(t[2]), int(t[3])))
        else:
            first[int(t[1])] = int(t[2])
    return pieces, first


@pytest.mark.parametrize("seed", range(8))
def test_split_covers_each_integral_in_bounded_pieces(driver, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    m = [int(v) for v in 10 ** rng.uniform(0, 7, n)]
    cost = [float(v) for v in rng.uniform(50, 900, n)]
    parts = int(rng.integers(1, 3000))
    pieces, first = _split(driver, m, cost, parts)
    assert len(pieces) <= n + parts + 1
    share = sum(a * c for a, c in zip(m, cost)) / parts
    k = 0
    for i in range(n):
        assert first[i] == k
        t = 0
        while k < len(pieces) and pieces[k][0] == i:
            _, t0, t1 = pieces[k]
            assert t0 == t and t1 > t0
            # a piece spans at most one share of work (plus rounding to whole sub-cubes)
            assert (t1 - t0) * cost[i] <= share + 2 * cost[i] + 1e-6 * share
            t = t1
            k += 1
        assert t == m[i]
    assert k == len(pieces)


def test_split_edge_cases(driver):
    # one part: every integral whole
    pieces, _ = _split(driver, [5, 1, 9], [1.0, 2.0, 3.0], 1)
    assert pieces == [(0, 0, 5), (1, 0, 1), (2, 0, 9)]
    # one integral, one sub-cube, many parts
    pieces, _ = _split(driver, [1], [7.0], 1000)
    assert pieces == [(0, 0, 1)]
    # equal shares of one integral
    pieces, _ = _split(driver, [1000], [1.0], 4)
    assert pieces == [(0, 0, 250), (0, 250, 500), (0, 500, 750), (0, 750, 1000)]


def test_largest_first_order(driver):
    rng = np.random.default_rng(5)
    n = 400
    rows = []
    for k in range(n):
        t0 = int(rng.integers(0, 1000))
        rows.append((k, t0, t0 + int(rng.integers(1, 5000)), float(rng.choice([1.0, 2.0, 3.5]))))
    text = f"order {n}\n" + "".join(f"{a} {b} {c} {d!r}\n" for a, b, c, d in rows)
    order = [int(v) for v in _run(driver, text).split()]
    assert sorted(order) == list(range(n))
    work = [(r[2] - r[1]) * r[3] for r in rows]
    top = max(work)
    # counting sort on work quantised to 1/256 of the largest: buckets from the
    # largest down, index order inside a bucket
    bucket = [min(255, int(w / top * 256)) for w in work]
    want = sorted(range(n), key=lambda k: (-bucket[k], k))
    assert order == want
    # so the order is within one bucket of decreasing work
    for a, b in zip(order, order[1:]):
        assert work[b] <= work[a] + top / 256
class _FirstFit:
    """Reference: sorted free list, first fit, neighbours merged on release."""

    def __init__(self, cap, align=256):
        self.align = align
        cap = cap // align * align
        self.free = [[0, cap]] if cap else []

    def _round(self, b):
        return (b + self.align - 1) // self.align * self.align

    def alloc(self, b):
        b = self._round(b)
        for idx, (off, ln) in enumerate(self.free):
            if ln >= b:
                if ln == b:
                    self.free.pop(idx)
                else:
                    self.free[idx] = [off + b, ln - b]
                return off
        return None

    def release(self, off, b):
        self.free.append([off, self._round(b)])
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1][1] += ln
            else:
                merged.append([o, ln])
        self.free = merged


@pytest.mark.parametrize("seed", range(6))
def test_arena_matches_first_fit_model(driver, seed):
    rng = np.random.default_rng(100 + seed)
    cap = int(rng.integers(1, 64)) * 4096 + int(rng.integers(0, 256))
    model = _FirstFit(cap)
    live, ops, want = [], [], []
    for _ in range(400):
        if live and rng.random() < 0.45:
            off, b = live.pop(int(rng.integers(0, len(live))))
            ops.append(f"r {off} {b}")
            model.release(off, b)
            want.append("released")
        else:
            b = int(rng.integers(1, 9000))
            off = model.alloc(b)
            ops.append(f"a {b}")
            if off is None:
                want.append("fail")
            else:
                live.append((off, b))
                want.append(f"ok {off}")
    out = _run(driver, f"arena {cap} {len(ops)}\n" + "\n".join(ops) + "\n").splitlines()
    assert out[:-1] == want
    free_bytes = sum(ln for _, ln in model.free)
    assert out[-1] == f"free {free_bytes} {len(model.free)}"
    # releasing everything restores one range of the whole capacity
    ops += [f"r {off} {b}" for off, b in live]
    out = _run(driver, f"arena {cap} {len(ops)}\n" + "\n".join(ops) + "\n").splitlines()
    assert out[-1] == f"free {cap // 256 * 256} 1"


# ---------------------------------------------------------------- step budget of the serving loop

def _select(exe, cand, budget, max_skip):
    text = f"select {len(cand)} {budget} {max_skip}\n" + "".join(
        f"{w!r} {s} {k} {i}\n" for w, s, k, i in cand)
    return [int(v) for v in _run(exe, text).split()]


def _select_model(cand, budget, max_skip):
    """Plain model: the overdue all run; the rest by (work, arrival) while the
    non-overdue samples fit; an empty step takes the first by that order."""
    order = sorted(range(len(cand)), key=lambda i: (cand[i][0], cand[i][3]))
    run, used = [0] * len(cand), 0
    for i in order:
        w, s, k, _ = cand[i]
        if k >= max_skip:
            run[i] = 1
        elif used + s <= budget:
            run[i], used = 1, used + s
    if order and not any(run):
        run[order[0]] = 1
    return run


@pytest.mark.parametrize("seed", range(10))
def test_select_for_step_matches_model(driver, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 80))
    cand = [(float(rng.choice([1.0, 2.0, 5.0])) * float(10 ** rng.integers(0, 4)),
             int(rng.choice([10**5, 10**6, 10**7])), int(rng.integers(0, 6)), int(i))
            for i in range(n)]
    budget = int(rng.choice([0, 10**5, 3 * 10**6, 2 * 10**7, 10**9]))
    max_skip = int(rng.integers(0, 6))
    got = _select(driver, cand, budget, max_skip)
    assert got == _select_model(cand, budget, max_skip)
    assert sum(got) >= 1
    # everything overdue runs; the others that run fit the budget (or are the only one)
    for (w, s, k, _), r in zip(cand, got):
        if k >= max_skip:
            assert r == 1
    rest = sum(s for (w, s, k, _), r in zip(cand, got) if r and k < max_skip)
    assert rest <= budget or sum(got) == 1


def test_select_for_step_prefers_short_and_bounds_waiting(driver):
    # one long request (10 units of work per step) and a stream of short ones:
    # with the budget the short ones run at once, and the long one still runs
    # at least once every max_skip + 1 steps
    budget, max_skip = 3 * 10**6, 3
    long_req = [1000.0, 10**7, 0, 0]
    waits, longest_gap, gap = [], 0, 0
    for step in range(40):
        shorts = [(1.0, 10**6, 0, 1 + 2 * step), (2.0, 10**6, 0, 2 + 2 * step)]
        cand = [tuple(long_req)] + shorts
        run = _select(driver, cand, budget, max_skip)
        assert run[1] == 1 and run[2] == 1
        if run[0]:
            long_req[2] = 0
            gap = 0
        else:
            long_req[2] += 1
            gap += 1
        longest_gap = max(longest_gap, gap)
    assert longest_gap == max_skip


def test_expected_iterations(driver):
    cases = [
        (0, 10, 1e-3, 0.0, 0.0),      # no estimate yet: the two the test needs
        (1, 10, 1e-3, 1.0, 0.1),      # one iteration: one more
        (2, 10, 0.0, 1.0, 0.1),       # no target: all that is left
        (4, 50, 1e-3, 2.0, 4e-3),     # e = 2e-3: 4 (2)^2 = 16 in all, 12 more
        (4, 10, 1e-3, 2.0, 4e-3),     # capped by itmax
        (4, 50, 1e-3, 2.0, 1e-3),     # already below the target: at least one
        (3, 50, 1e-3, -2.0, 6e-3),    # sign of the estimate does not matter: 3 * 9 = 27, 24 more
        (2, 50, 1e-3, 0.0, 1e-3),     # zero estimate: as if no estimate
        (2, 50, 1e-3, 1.0, float("nan")),
        (50, 50, 1e-3, 1.0, 0.1),     # nothing left
    ]
    text = f"iters {len(cases)}\n" + "".join(f"{a} {b} {c!r} {d!r} {e!r}\n" for a, b, c, d, e in cases)
    got = [float(v) for v in _run(driver, text).split()]
    assert got == [2.0, 1.0, 8.0, 12.0, 6.0, 1.0, 24.0, 1.0, 1.0, 1.0]

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
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_2202_01753_amd", "csrc"),
                    os.path.join(HERE, "pins", "batch_plan_check.cpp"), "-o", exe], check=True)
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

"""Host-side logic of bench.py (no GPU): the one-GPU guard, the dense cell
counts the GCUPS figures divide by, and the HBM-traffic lookup's refusal of
summaries measured on other kernel sources."""
import importlib.util
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def brute_cells(kind, ratio, lq, lr):
    """Cells (i, j), 1 <= i <= lq, 1 <= j <= lr, inside the Sakoe-Chiba window
    of the pair (w = floor(ratio * max(lq, lr))); 0 when the window admits no
    path (w < |lq - lr|)."""
    if kind not in ("cdtw", "erp") or ratio >= 1:
        return lq * lr
    w = int(np.floor(ratio * max(lq, lr)))
    if w < abs(lq - lr):
        return 0
    return sum(1 for i, j in itertools.product(range(1, lq + 1), range(1, lr + 1)) if abs(i - j) <= w)


@pytest.mark.parametrize("kind,ratio", [("dtw", 2.0), ("cdtw", 0.0), ("cdtw", 0.05), ("cdtw", 0.1), ("cdtw", 0.5),
                                        ("erp", 0.2), ("cdtw", 1.0)])
def test_dense_cells_match_brute_force(bench, kind, ratio):
    rng = np.random.default_rng(3)
    lq = rng.integers(1, 40, 7)
    lr = rng.integers(1, 40, 9)
    lq[0], lr[0] = 25, 25          # equal lengths
    lr[1] = lq[1] + 30             # far apart: no path in narrow windows
    q_off = np.concatenate([[0], np.cumsum(lq)]).astype(np.int64)
    r_off = np.concatenate([[0], np.cumsum(lr)]).astype(np.int64)
    p = {"kind": kind} if kind == "dtw" else {"kind": kind, "window_ratio": ratio}
    want = sum(brute_cells(kind, ratio, int(a), int(b)) for a in lq for b in lr)
    assert bench.dense_cells(kind, p, q_off, r_off) == want


def test_hbm_traffic_refuses_other_sources(bench, monkeypatch):
    monkeypatch.setattr(bench, "_source_hash", lambda: "0000000000000000")
    value, note = bench.hbm_traffic("rows128 8x16 sweep, MSM main stage, fp32")
    assert value is None and "no counter summary" in note

"""ctypes wrapper of the CPU oracle library.

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg.  The device library never uses it.

Parameters are passed as a dict with keys kind ('dtw', 'cdtw', 'wdtw', 'erp',
'msm', 'twe'), window_ratio, g, gap, c, nu, lam; missing keys take the
defaults below.  Series are float64 numpy arrays.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

KINDS = {"dtw": 0, "cdtw": 1, "wdtw": 2, "erp": 3, "msm": 4, "twe": 5}

_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(
                os.path.join(HERE, "eap_oracle.c")):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_window.restype = _i64
        L.orc_window.argtypes = [ctypes.c_int, _d, _i64, _i64]
        L.orc_wdtw_weights.restype = None
        L.orc_wdtw_weights.argtypes = [_d, _i64, _pd]
        L.orc_dp.restype = _d
        L.orc_dp.argtypes = [ctypes.c_int, _pd, _i64, _pd, _i64, _pd, _pd]
        L.orc_brute.restype = _d
        L.orc_brute.argtypes = [ctypes.c_int, _pd, _i64, _pd, _i64, _pd, _pi64]
        L.orc_eap.restype = _d
        L.orc_eap.argtypes = [ctypes.c_int, _pd, _i64, _pd, _i64, _pd, _d, _pi64, _pi64, _pi64]
        L.orc_eabase.restype = _d
        L.orc_eabase.argtypes = [ctypes.c_int, _pd, _i64, _pd, _i64, _pd, _d, _pi64]
        L.orc_envelope.restype = None
        L.orc_envelope.argtypes = [_pd, _i64, _i64, _i64, _pd, _pd]
        L.orc_lb_keogh.restype = _d
        L.orc_lb_keogh.argtypes = [_pd, _i64, _pd, _i64, _i64]
        L.orc_lb_kim.restype = _d
        L.orc_lb_kim.argtypes = [_pd, _i64, _pd, _i64]
        L.orc_ub.restype = _d
        L.orc_ub.argtypes = [ctypes.c_int, _pd, _i64, _pd, _i64, _pd]
        L.orc_nn1.restype = None
        L.orc_nn1.argtypes = [ctypes.c_int, _pd, _pd, _pi64, _i64, _pd, _pi64, _i64, ctypes.c_int, _pi64, _pd,
                              ctypes.c_int, _pi64]
        L.orc_pairwise.restype = None
        L.orc_pairwise.argtypes = [ctypes.c_int, _pd, _pd, _pi64, _i64, ctypes.c_int, _pd, ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _prm(p: dict) -> np.ndarray:
    return np.array([float(p.get("window_ratio", float("inf"))), float(p.get("g", 0.0)), float(p.get("gap", 0.0)),
                     float(p.get("c", 0.0)), float(p.get("nu", 0.0)), float(p.get("lam", p.get("lambda", 0.0))),
                     float(p.get("dims", 1))], dtype=np.float64)


def _pts(x: np.ndarray, p: dict) -> int:
    """Points in a series of values (one value per channel per point)."""
    d = dims(p)
    if len(x) % d:
        raise ValueError(f"{len(x)} values do not make whole points of {d} channels")
    return len(x) // d


def dims(p: dict) -> int:
    """Channels per series point (multivariate DTW / CDTW); values are stored
    point after point, so a series of L points holds L * dims values."""
    return max(1, int(p.get("dims", 1)))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_pd)


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(_pi64)


def kind_id(p: dict) -> int:
    return KINDS[p["kind"]]


def window(p: dict, lx: int, ly: int) -> int:
    return int(lib().orc_window(kind_id(p), float(p.get("window_ratio", float("inf"))), lx, ly))


def wdtw_weights(g: float, L: int) -> np.ndarray:
    out = np.empty(L, dtype=np.float64)
    lib().orc_wdtw_weights(float(g), L, _ptr(out))
    return out


def dp(p: dict, x, y, return_matrix: bool = False):
    x, y = _f64(x), _f64(y)
    prm = _prm(p)
    if return_matrix:
        M = np.empty((_pts(x, p) + 1, _pts(y, p) + 1), dtype=np.float64)
        d = lib().orc_dp(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm), _ptr(M))
        return d, M
    return lib().orc_dp(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm), None)


def brute(p: dict, x, y):
    x, y = _f64(x), _f64(y)
    prm = _prm(p)
    n = ctypes.c_int64(0)
    d = lib().orc_brute(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm), ctypes.byref(n))
    return d, n.value


def eap(p: dict, x, y, cutoff: float = float("inf")):
    """EAPruned distance: (value, cells evaluated, (abandon_i, abandon_j))."""
    x, y = _f64(x), _f64(y)
    prm = _prm(p)
    c, ai, aj = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    d = lib().orc_eap(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm), float(cutoff), ctypes.byref(c),
                      ctypes.byref(ai), ctypes.byref(aj))
    return d, c.value, (ai.value, aj.value)


def eabase(p: dict, x, y, cutoff: float = float("inf")):
    """EABase (Alg. 4): (value, cells evaluated); +inf when a row is dead."""
    x, y = _f64(x), _f64(y)
    prm = _prm(p)
    c = ctypes.c_int64(0)
    d = lib().orc_eabase(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm), float(cutoff), ctypes.byref(c))
    return d, c.value


def envelope(x, w: int, n: int = 0):
    """(up, lo) of x under window w at positions 1..n (default len(x))."""
    x = _f64(x)
    n = n or len(x)
    up, lo = np.empty(n), np.empty(n)
    lib().orc_envelope(_ptr(x), len(x), int(w), n, _ptr(up), _ptr(lo))
    return up, lo


def lb_keogh(q, c, w: int) -> float:
    """LB_Keogh(Q, C): envelope of q under window w against the values of c."""
    q, c = _f64(q), _f64(c)
    return lib().orc_lb_keogh(_ptr(q), len(q), _ptr(c), len(c), int(w))


def lb_kim(q, c) -> float:
    """LB_Kim, first and last points."""
    q, c = _f64(q), _f64(c)
    return lib().orc_lb_kim(_ptr(q), len(q), _ptr(c), len(c))


def ub(p: dict, x, y) -> float:
    x, y = _f64(x), _f64(y)
    prm = _prm(p)
    return lib().orc_ub(kind_id(p), _ptr(x), _pts(x, p), _ptr(y), _pts(y, p), _ptr(prm))


NN_MODES = {"dp": 0, "eap": 1, "eabase": 2, "eap_lb": 3}


def nn1(p: dict, q, q_off, r, r_off, mode: str = "eap", nthreads: int = 0):
    """Alg. 1 over ragged sets; mode 'dp' (full DP), 'eap' (EAPruned), 'eabase'
    (Alg. 4) or 'eap_lb' (EAPruned behind LB_Kim, LB_Keogh and the reversed
    LB_Keogh, Alg. 2; DTW and CDTW).
    Returns (idx int64[nq], dist float64[nq], cells evaluated)."""
    q, r = _f64(q), _f64(r)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    nq, nr = len(q_off) - 1, len(r_off) - 1
    idx = np.empty(nq, dtype=np.int64)
    dist = np.empty(nq, dtype=np.float64)
    cells = ctypes.c_int64(0)
    prm = _prm(p)
    lib().orc_nn1(kind_id(p), _ptr(prm), _ptr(q), _iptr(q_off), nq, _ptr(r), _iptr(r_off), nr,
                  NN_MODES[mode], _iptr(idx), _ptr(dist), int(nthreads), ctypes.byref(cells))
    return idx, dist, cells.value


def pairwise(p: dict, s, s_off, mode: str = "prune", nthreads: int = 0) -> np.ndarray:
    s = _f64(s)
    s_off = np.ascontiguousarray(s_off, dtype=np.int64)
    n = len(s_off) - 1
    out = np.empty(n * (n - 1) // 2, dtype=np.float64)
    prm = _prm(p)
    lib().orc_pairwise(kind_id(p), _ptr(prm), _ptr(s), _iptr(s_off), n, 0 if mode == "prune" else 1, _ptr(out),
                       int(nthreads))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def derivative(v, off) -> np.ndarray:
    """First-derivative series for the derivative variants (DDTW, DCDTW,
    DWDTW: the distance of the derivative series, Section 2.3 names them
    without a formula).  Reading: the estimate of Keogh and Pazzani (2001),
    for 1 < i < m: d_i = ((q_i - q_{i-1}) + (q_{i+1} - q_{i-1}) / 2) / 2,
    evaluated in that order in binary64; the ends copy their neighbours,
    d_1 = d_2 and d_m = d_{m-1}; m = 2 gives d_1 = d_2 = q_2 - q_1 and m = 1
    gives 0.  A plain loop over the values of each series."""
    v = _f64(v)
    off = np.asarray(off, dtype=np.int64)
    out = np.empty_like(v)
    for s in range(len(off) - 1):
        a, m = int(off[s]), int(off[s + 1] - off[s])
        q = v[a:a + m]
        if m == 1:
            out[a] = 0.0
            continue
        if m == 2:
            out[a] = out[a + 1] = q[1] - q[0]
            continue
        for i in range(1, m - 1):
            out[a + i] = ((q[i] - q[i - 1]) + (q[i + 1] - q[i - 1]) / 2.0) / 2.0
        out[a] = out[a + 1]
        out[a + m - 1] = out[a + m - 2]
    return out


def subseq_windows(s, m: int) -> np.ndarray:
    """Candidates of a sub-sequence search (Section 5.3: the closest match of
    a query within a long series): every window of length m, z-normalised on
    its own as the UCR suite does (reading: population standard deviation; a
    constant window gives zeros).  For window w, in binary64 and in this order:
    mean = (sum over k, left to right, of s[w+k]) / m, var = (sum of
    (s[w+k] - mean)^2, left to right) / m, sd = sqrt(var), value k =
    (s[w+k] - mean) / sd.  Returns the windows back to back, (n-m+1) * m
    values.  The loops run over k, each step applied to all windows at once
    (element-wise binary64 operations, so every window sees exactly the
    sequence of operations written above)."""
    s = _f64(s)
    nw = len(s) - m + 1
    acc = np.zeros(nw)
    for k in range(m):
        acc = acc + s[k:k + nw]
    mean = acc / m
    v = np.zeros(nw)
    for k in range(m):
        d = s[k:k + nw] - mean
        v = v + d * d
    sd = np.sqrt(v / m)
    out = np.zeros((nw, m))
    ok = sd > 0.0
    for k in range(m):
        out[ok, k] = (s[k:k + nw][ok] - mean[ok]) / sd[ok]
    return out.reshape(-1)

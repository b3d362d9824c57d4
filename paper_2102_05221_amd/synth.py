"""Seeded synthetic series with the shapes of the paper's NN-classification workloads.

The paper measures NN classification over the UCR archive (Section 5.1) and
sub-sequence search over long recordings (Section 5.3).  Neither is available
here, so these generators stand in for them: z-normalised random walks and
five-class template series that are randomly time-warped, at the lengths and
set sizes of the workloads this package is measured on.

This module only draws inputs.  It holds none of the distance arithmetic, so
both the device path and the CPU oracle can be fed from it without sharing any
of the method's code.

Ragged sets are returned as ``(values, offsets)``: ``values`` is one float64
array with every series concatenated, ``offsets`` an int64 array of length
``n + 1`` with series ``k`` at ``values[offsets[k]:offsets[k + 1]]``.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2102052210


def znorm(x: np.ndarray) -> np.ndarray:
    """Z-normalise with the population standard deviation; a constant series
    becomes all zeros."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean()
    sd = x.std()
    if not np.isfinite(sd) or sd == 0.0:
        return np.zeros_like(x)
    return (x - mu) / sd


def pack(series) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate a list of 1-D arrays into ``(values, offsets)``."""
    lens = np.array([len(s) for s in series], dtype=np.int64)
    off = np.zeros(len(series) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    vals = np.concatenate([np.asarray(s, dtype=np.float64) for s in series]) if series else np.zeros(0)
    return np.ascontiguousarray(vals, dtype=np.float64), off


def unpack(values: np.ndarray, offsets: np.ndarray):
    return [values[offsets[k]:offsets[k + 1]] for k in range(len(offsets) - 1)]


def _lengths(rng, n, length):
    if isinstance(length, (tuple, list)):
        lo, hi = int(length[0]), int(length[1])
        return rng.integers(lo, hi + 1, size=n)
    return np.full(n, int(length), dtype=np.int64)


def random_walks(rng, n: int, length) -> list[np.ndarray]:
    """Gaussian random walks x_t = sum_{u<=t} eps_u, eps ~ N(0,1), z-normalised.
    ``length`` is an int or an inclusive ``(lo, hi)`` range drawn uniformly."""
    lens = _lengths(rng, n, length)
    return [znorm(np.cumsum(rng.standard_normal(int(L)))) for L in lens]


def class_templates(rng, n_classes: int = 5):
    """Per class: 3 distinct integer frequencies from 1..8 and 3 phases in
    [0, 2*pi); T_c(u) = sum_k sin(2*pi*f_k*u + phi_k) on u in [0, 1]."""
    out = []
    for _ in range(n_classes):
        f = rng.choice(np.arange(1, 9), size=3, replace=False).astype(np.float64)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
        out.append((f, ph))
    return out


def warped_series(rng, template, length: int, noise_sd: float = 0.1) -> np.ndarray:
    """One series of the given class: the template read through a random
    monotone piecewise-linear warp with knots at k/5 moved by U[-0.1, 0.1],
    plus N(0, noise_sd) noise, then z-normalised."""
    f, ph = template
    knots_x = np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0])
    knots_y = knots_x.copy()
    knots_y[1:5] += rng.uniform(-0.1, 0.1, size=4)
    u = np.arange(length, dtype=np.float64) / max(length - 1, 1)
    tau = np.interp(u, knots_x, knots_y)
    x = np.zeros(length)
    for k in range(3):
        x += np.sin(2.0 * np.pi * f[k] * tau + ph[k])
    x += rng.normal(0.0, noise_sd, size=length)
    return znorm(x)


def class_series(rng, templates, n: int, length):
    lens = _lengths(rng, n, length)
    labels = rng.integers(0, len(templates), size=n).astype(np.int32)
    series = [warped_series(rng, templates[c], int(L)) for c, L in zip(labels, lens)]
    return series, labels


# Distance parameters of the measured workloads (paper Section 2.3 names them;
# the values are the ones these workloads fix).
SIX = ("dtw", "cdtw", "wdtw", "erp", "msm", "twe")
DEFAULT_PARAMS = {
    "dtw": dict(kind="dtw"),
    "cdtw": dict(kind="cdtw", window_ratio=0.10),
    "wdtw": dict(kind="wdtw", g=0.05),
    "erp": dict(kind="erp", gap=0.0, window_ratio=float("inf")),
    "msm": dict(kind="msm", c=0.5),
    "twe": dict(kind="twe", nu=0.001, lam=1.0),
}


def make_workload(k: int, n_ref: int | None = None, n_query: int | None = None, length=None):
    """The five measured workloads (k = 1..5); ``n_ref``/``n_query``/``length``
    shrink them for tests.  Returns a dict of numpy arrays and parameters."""
    rng = np.random.default_rng(BASE_SEED + k)
    if k == 1:
        nr, nq, L = 100, 100, 128
        nr, nq = n_ref or nr, n_query or nq
        L = length or L
        r_rng, q_rng = rng.spawn(2)
        refs = random_walks(r_rng, nr, L)
        r_lab = r_rng.integers(0, 3, size=nr).astype(np.int32)
        qs = random_walks(q_rng, nq, L)
        q_lab = q_rng.integers(0, 3, size=nq).astype(np.int32)
        kinds = ("dtw",)
    elif k in (2, 4):
        if k == 2:
            nr, nq, L = 500, 500, 512
        else:
            nr, nq, L = 10000, 1000, (64, 2048)
        nr, nq = n_ref or nr, n_query or nq
        L = length or L
        templates = class_templates(rng, 5)
        r_rng, q_rng = rng.spawn(2)
        refs, r_lab = class_series(r_rng, templates, nr, L)
        qs, q_lab = class_series(q_rng, templates, nq, L)
        kinds = SIX
    elif k == 3:
        n, L = 2000, 1024
        n = n_ref or n
        L = length or L
        (s_rng,) = rng.spawn(1)
        refs = random_walks(s_rng, n, L)
        r_lab = np.zeros(n, dtype=np.int32)
        qs, q_lab = [], np.zeros(0, dtype=np.int32)
        kinds = ("dtw", "cdtw", "msm")
    elif k == 5:
        nr, nq, L = 50000, 2000, (128, 1024)
        nr, nq = n_ref or nr, n_query or nq
        L = length or L
        r_rng, q_rng, a_rng = rng.spawn(3)
        refs = random_walks(r_rng, nr, L)
        r_lab = np.zeros(nr, dtype=np.int32)
        qs = random_walks(q_rng, nq, L)
        q_lab = np.zeros(nq, dtype=np.int32)
        kinds = ("cdtw", "msm")
    else:
        raise ValueError("workload k must be 1..5")
    params = {kd: dict(DEFAULT_PARAMS[kd]) for kd in kinds}
    if k == 3:
        params["cdtw"]["window_ratio"] = 0.05
    if k == 5:
        params["cdtw"]["window_ratio"] = 0.05
    rv, ro = pack(refs)
    out = dict(k=k, refs=rv, ref_off=ro, ref_labels=r_lab, params=params)
    if qs:
        qv, qo = pack(qs)
        out.update(queries=qv, query_off=qo, query_labels=q_lab)
    if k == 5:
        rate = 2000.0
        out["arrivals"] = np.cumsum(a_rng.exponential(1.0 / rate, size=len(qs)))
    return out


def random_pairs(seed: int, n: int, lo: int, hi: int, kind: str = "walk"):
    """Small seeded pair sets for parity tests: ``n`` pairs with lengths drawn
    from [lo, hi]; series are random walks or i.i.d. normals (z-normalised)."""
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for _ in range(n):
        lx, ly = rng.integers(lo, hi + 1, size=2)
        if kind == "walk":
            xs.append(znorm(np.cumsum(rng.standard_normal(int(lx)))))
            ys.append(znorm(np.cumsum(rng.standard_normal(int(ly)))))
        else:
            xs.append(rng.standard_normal(int(lx)))
            ys.append(rng.standard_normal(int(ly)))
    return xs, ys


def subseq_workload(n_windows: int = 1 << 20, m: int = 128, n_query: int = 16):
    """Sub-sequence search input (Section 5.3's task on a synthetic recording):
    a random walk of ``n_windows + m - 1`` values, so that it has ``n_windows``
    windows of ``m``, and ``n_query`` raw queries of ``m`` values.  The first
    half of the queries are windows of the walk at seeded ``starts``, scaled by
    1.5, shifted by 3 and given N(0, 0.1) noise; the rest are fresh random
    walks.  Nothing is normalised here: the search normalises every window and
    query itself."""
    rng = np.random.default_rng(BASE_SEED + 6)
    s = np.cumsum(rng.standard_normal(n_windows + m - 1))
    starts = rng.integers(0, n_windows, n_query // 2)
    qs = [1.5 * s[st:st + m] + 3.0 + 0.1 * rng.standard_normal(m) for st in starts]
    qs += [np.cumsum(rng.standard_normal(m)) for _ in range(n_query - len(qs))]
    return dict(series=s, queries=qs, starts=starts, m=m)

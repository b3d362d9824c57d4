"""The FP32 screen's certified error bound, pinned on the CPU (no GPU).

The FP32 screening sweep of an NN search (precision 1) relies on two
inequalities for every pair: its FP32 result D32 is at most D + eps(D), and
the exact distance D is at most screen_bound(D32), with eps and screen_bound
the library's own (eap_screen_eps / eap_screen_bound, host utilities of the C
ABI).  Here a float32 dynamic programme written in this file evaluates each
distance the way the FP32 sweep does (every operation rounded to float32, no
fused operations; inputs rounded to float32, or, for exact differences, each
difference formed in float64 and rounded once) and is compared with the
float64 oracle on inputs chosen to be hard for the bound: values of large
magnitude, pairs of near-duplicate series whose values straddle float32
rounding boundaries (so that input rounding alone makes up the FP32 result),
constant series, and pairs of up to 2 x 2048 values.
"""
import math

import numpy as np
import pytest

import paper_2102_05221_amd as eap

F = np.float32
INF32 = np.float32(np.inf)


def fma32(a, b, c):
    """float32 fused multiply-add: the product of two float32 values is exact
    in float64, the sum is rounded there and then to float32 (double rounding:
    within the bound's factor 1.01 of a single one)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F)


def fp32_dp(kind, x, y, prm, exact_diff=False, fused=False):
    """float32 DP over anti-diagonals (rows x, columns y).  fused: the squared
    costs' (weighted) square fused with the add, as the FP32 sweeps do."""
    lx, ly = len(x), len(y)
    xs, ys = x.astype(F), y.astype(F)
    M = np.full((lx + 1, ly + 1), INF32, dtype=F)
    M[0, 0] = F(0)
    w = lx + ly
    if kind == "cdtw":
        w = int(math.floor(prm["window_ratio"] * max(lx, ly)))
        if w < abs(lx - ly):
            return math.inf
    if kind == "erp":
        gap = F(prm["gap"])
        for i in range(1, lx + 1):
            M[i, 0] = M[i - 1, 0] + np.abs(xs[i - 1] - gap)
        for j in range(1, ly + 1):
            M[0, j] = M[0, j - 1] + np.abs(ys[j - 1] - gap)
    if kind == "wdtw":
        L = max(lx, ly)
        k = np.arange(L, dtype=np.float64)
        W = (1.0 / (1.0 + np.exp(-prm["g"] * (k - L / 2.0)))).astype(F)
    if kind == "twe":
        nu, lam = F(prm["nu"]), F(prm["lam"])
        nu2 = (prm["nu"] * (2.0 * np.arange(max(lx, ly) + 1, dtype=np.float64))).astype(F)
    if kind == "msm":
        c = F(prm["c"])
    for a in range(2, lx + ly + 1):
        i = np.arange(max(1, a - ly), min(lx, a - 1) + 1)
        j = a - i
        diag, top, left = M[i - 1, j - 1], M[i - 1, j], M[i, j - 1]
        si, tj = xs[i - 1], ys[j - 1]
        if exact_diff:
            d = (x[i - 1] - y[j - 1]).astype(F)
        else:
            d = si - tj
        if kind in ("dtw", "cdtw") and fused:
            v = fma32(d, d, np.minimum(np.minimum(diag, top), left))
        elif kind == "wdtw" and fused:
            v = fma32(W[np.abs(i - j)] * d, d, np.minimum(np.minimum(diag, top), left))
        elif kind in ("dtw", "cdtw"):
            v = d * d + np.minimum(np.minimum(diag, top), left)
        elif kind == "wdtw":
            v = W[np.abs(i - j)] * (d * d) + np.minimum(np.minimum(diag, top), left)
        elif kind == "erp":
            v = np.minimum(np.minimum(diag + np.abs(d), top + np.abs(si - gap)), left + np.abs(tj - gap))
        elif kind == "msm":
            def cost(new, p, q):
                inside = ((p <= new) & (new <= q)) | ((p >= new) & (new >= q))
                return np.where(inside, c, c + np.minimum(np.abs(new - p), np.abs(new - q)))
            sp = xs[np.maximum(i - 2, 0)]
            tp = ys[np.maximum(j - 2, 0)]
            up = np.where(i == 1, INF32, top + cost(si, sp, tj))
            lf = np.where(j == 1, INF32, left + cost(tj, si, tp))
            v = np.minimum(np.minimum(diag + np.abs(d), up), lf)
        elif kind == "twe":
            sp = np.where(i == 1, F(0), xs[np.maximum(i - 2, 0)])
            tp = np.where(j == 1, F(0), ys[np.maximum(j - 2, 0)])
            match = (np.abs(d) + np.abs(sp - tp)) + nu2[np.abs(i - j)]
            v = np.minimum(np.minimum(diag + match, top + ((np.abs(si - sp) + nu) + lam)),
                           left + ((np.abs(tj - tp) + nu) + lam))
        if kind == "cdtw":
            v = np.where(np.abs(i - j) > w, INF32, v)
        M[i, j] = v
    return float(M[lx, ly])


PARAMS = {
    "dtw": dict(kind="dtw"),
    "cdtw": dict(kind="cdtw", window_ratio=0.1),
    "wdtw": dict(kind="wdtw", g=0.05),
    "erp": dict(kind="erp", gap=0.0),
    "msm": dict(kind="msm", c=0.5),
    "twe": dict(kind="twe", nu=0.001, lam=1.0),
}


def straddle(rng, n, scale):
    """Values just below and just above the midpoint between two float32
    neighbours: a pair (x, y) of such series differs by almost nothing in
    float64 but by a whole float32 ulp after rounding."""
    v = (rng.normal(size=n) * scale).astype(F)
    up = np.nextafter(v, F(np.inf))
    mid = (v.astype(np.float64) + up.astype(np.float64)) / 2.0
    gap = (up.astype(np.float64) - v.astype(np.float64))
    x = mid - gap * 1e-3
    y = mid + gap * 1e-3
    return x, y


def cases():
    rng = np.random.default_rng(52210)
    out = []
    # typical z-normalised random walks, up to 2 x 2048 values
    for lx, ly in [(2048, 2048), (2048, 1500), (700, 650), (64, 5), (1, 1)]:
        x = np.cumsum(rng.normal(size=lx))
        y = np.cumsum(rng.normal(size=ly))
        out.append((f"walk{lx}x{ly}", (x - x.mean()) / (x.std() or 1), (y - y.mean()) / (y.std() or 1)))
    # near duplicates straddling float32 rounding: input rounding is the whole FP32 result
    for n, scale in [(2048, 1.0), (600, 1e3), (37, 3e5)]:
        x, y = straddle(rng, n, scale)
        out.append((f"straddle{n}s{scale:g}", x, y))
    # large magnitude, unrelated series
    out.append(("large", rng.normal(size=900) * 1e4, rng.normal(size=1000) * 1e4))
    # constant series (distance 0 or a multiple of one difference)
    out.append(("const", np.full(300, 0.3), np.full(280, 0.3)))
    return out


CASES = cases()


@pytest.mark.parametrize("kind", list(PARAMS))
def test_fp32_dp_within_certified_bound(orc, kind):
    p = PARAMS[kind]
    for name, x, y in CASES:
        if kind in ("twe", "msm", "erp") and len(x) * len(y) > 1600 * 1600:
            x, y = x[:1200], y[:1100]          # keep the L1 kinds' emulation short
        d64 = orc.dp(p, x, y)
        if math.isinf(d64):
            continue
        d32 = fp32_dp(kind, x, y, p)
        A = max(np.abs(x).max(), np.abs(y).max(), abs(p.get("gap", 0.0)))
        N = len(x) + len(y)
        eps = eap.screen_eps(kind, d64, N, A)
        assert d32 <= d64 + eps, (kind, name, d32, d64, eps)
        assert d64 <= eap.screen_bound(kind, d32, N, A), (kind, name, d32, d64)


@pytest.mark.parametrize("kind", ["dtw", "wdtw"])
def test_fp32_dp_exact_differences_within_relative_bound(orc, kind):
    """Differences formed in float64 and rounded once: the bound has no
    magnitude term, so it is relative; WDTW with the weights of long series
    (around 1e-22 near the diagonal) stays within it."""
    p = dict(PARAMS[kind], g=0.05) if kind == "wdtw" else PARAMS[kind]
    for name, x, y in CASES:
        d64 = orc.dp(p, x, y)
        d32 = fp32_dp(kind, x, y, p, exact_diff=True)
        N = len(x) + len(y)
        eps = eap.screen_eps(kind, d64, N, 0.0, exact_diff=True)
        assert d32 <= d64 + eps, (kind, name, d32, d64, eps)
        assert d64 <= eap.screen_bound(kind, d32, N, 0.0, exact_diff=True), (kind, name, d32, d64)
        if d64 > 0:
            assert abs(d32 - d64) <= 1.01 * 2.0 ** -24 * (N + 5) * d64 + N * 4e-38


@pytest.mark.parametrize("kind", ["dtw", "cdtw", "wdtw"])
def test_fp32_dp_fused_within_certified_bound(orc, kind):
    """The FP32 sweeps of the squared costs fuse the (weighted) square with
    the add: one rounding fewer per cell, still inside both bounds (input
    rounding, and exact differences)."""
    p = PARAMS[kind]
    for name, x, y in CASES:
        d64 = orc.dp(p, x, y)
        if math.isinf(d64):
            continue
        N = len(x) + len(y)
        A = max(np.abs(x).max(), np.abs(y).max())
        d32 = fp32_dp(kind, x, y, p, fused=True)
        assert d32 <= d64 + eap.screen_eps(kind, d64, N, A), (kind, name, d32, d64)
        assert d64 <= eap.screen_bound(kind, d32, N, A), (kind, name, d32, d64)
        if kind != "cdtw":
            dx = fp32_dp(kind, x, y, p, exact_diff=True, fused=True)
            assert dx <= d64 + eap.screen_eps(kind, d64, N, 0.0, exact_diff=True), (kind, name, dx, d64)
            assert d64 <= eap.screen_bound(kind, dx, N, 0.0, exact_diff=True), (kind, name, dx, d64)


def test_missing_square_term_would_fail(orc):
    """The straddling near-duplicates are the case the u^2 A^2 N term exists
    for: without it the bound of the squared costs is violated."""
    rng = np.random.default_rng(7)
    x, y = straddle(rng, 2048, 1.0)
    d64 = orc.dp(PARAMS["dtw"], x, y)
    d32 = fp32_dp("dtw", x, y, PARAMS["dtw"])
    A, N, u = max(np.abs(x).max(), np.abs(y).max()), 4096.0, 2.0 ** -24
    without = 1.01 * u * ((N + 5) * d64 + 4 * A * math.sqrt(N * d64)) + N * 4e-38
    assert d32 > d64 + without
    assert d32 <= d64 + eap.screen_eps("dtw", d64, N, A)

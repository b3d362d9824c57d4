"""eap_distance_noalloc (the distance call that allocates nothing) against
eap_distance on the same inputs (GPU required).

Both are called through the C ABI.  Two calls in a row share the library's
static scratch, the second with a smaller input, so that what the first left
in the scratch must not leak into the second; results are compared with the
workspace entry point's bit for bit (same kernels, same cell order) and with
the CPU oracle to the 1e-12 relative tolerance of the contract.
"""
import ctypes
import math
import sys

import numpy as np
import pytest

import paper_2102_05221_amd as eap
from paper_2102_05221_amd import synth

pytestmark = pytest.mark.gpu

INF = math.inf
RTOL = 1e-12

KINDS = [
    dict(kind="dtw"),
    dict(kind="cdtw", window_ratio=0.1),
    dict(kind="wdtw", g=0.05),
    dict(kind="erp", gap=0.0),
    dict(kind="erp", gap=0.3, window_ratio=0.2),
    dict(kind="msm", c=0.5),
    dict(kind="twe", nu=0.001, lam=1.0),
]

# (first call, second call): the second is smaller on both sides
SIZES = [((2048, 1900), (700, 650)), ((700, 650), (90, 33)), ((333, 512), (17, 16)), ((64, 64), (1, 1))]


def pid(p):
    return "-".join(f"{k}={v}" for k, v in p.items())


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def series(rng, n):
    return synth.znorm(np.cumsum(rng.normal(size=n))) if n > 1 else rng.normal(size=1)


def call_noalloc(torch, xd, yd, p, cut):
    """eap_distance_noalloc through ctypes, on torch's current stream."""
    out = torch.full((1,), -1.0, dtype=torch.float64, device=xd.device)
    st = eap.lib().eap_distance_noalloc(xd.data_ptr(), xd.numel(), yd.data_ptr(), yd.numel(),
                                        ctypes.byref(eap.params_from_dict(p)), float(cut), out.data_ptr(),
                                        ctypes.c_void_p(torch.cuda.current_stream(xd.device).cuda_stream))
    assert st == 0, eap.lib().eap_last_error().decode()
    return out


def close(g, o):
    if math.isinf(o) or math.isinf(g):
        return math.isinf(o) and math.isinf(g)
    return abs(g - o) <= RTOL * max(abs(o), 1e-300)


@pytest.mark.parametrize("p", KINDS, ids=pid)
def test_noalloc_equals_workspace_call_twice_in_a_row(torch_dev, orc, p):
    torch, dev = torch_dev
    rng = np.random.default_rng(7000 + synth.SIX.index(p["kind"]))
    for big, small in SIZES:
        pair = {}
        for tag, (lx, ly) in (("big", big), ("small", small)):
            x, y = series(rng, lx), series(rng, ly)
            pair[tag] = (x, y, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), orc.dp(p, x, y))
        # cut-offs: +inf, then just below the distance (abandoned), then the distance itself
        for sel in range(3):
            outs = {}
            for tag in ("big", "small"):   # two calls in a row, the second smaller
                x, y, xd, yd, d = pair[tag]
                cut = [INF, float(np.nextafter(d, -INF)) if d < INF else INF, d][sel]
                print(f"noalloc {pid(p)} {tag} lx={len(x)} ly={len(y)} cut={cut}", flush=True)
                sys.stdout.flush()
                outs[tag] = (call_noalloc(torch, xd, yd, p, cut), cut, d, xd, yd)
            torch.cuda.synchronize()
            for tag, (o, cut, d, xd, yd) in outs.items():
                g = float(o.item())
                ref = float(eap.distance(xd, yd, p, cut).item())
                want = d if d <= cut else INF
                assert g == ref or (math.isinf(g) and math.isinf(ref)), (tag, cut, g, ref)
                assert close(g, want), (tag, cut, g, want)

"""C-ABI checks that need no GPU: the library loads, exports every function
include/eap.h declares, validates its arguments before touching the device,
and computes the same WDTW weights as the oracle, bit for bit."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2102_05221_amd as eap
from paper_2102_05221_amd import build as eap_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eap.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(eap.LIB_PATH):
        eap_build.build()
    return eap.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eap_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_three_paper_calls():
    names = declared_functions()
    for n in ("eap_distance", "eap_nn1", "eap_pairwise", "eap_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name
    assert b"gfx950" in L.eap_version()


def _p(kind="dtw", **kw):
    return eap.params(kind, **kw)


def _off(*lens):
    o = np.zeros(len(lens) + 1, dtype=np.int64)
    o[1:] = np.cumsum(lens)
    return o


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every case below fails validation first


def test_distance_argument_errors(L):
    p = _p()
    ws = ctypes.c_void_p(0x2000)
    need = L.eap_distance_workspace(10, 12, ctypes.byref(p))
    assert need > 0
    cases = [
        (None, 10, FAKE, 12, p, 1.0, FAKE, ws, need),          # NULL x
        (FAKE, 0, FAKE, 12, p, 1.0, FAKE, ws, need),           # empty series
        (FAKE, 10, FAKE, 12, p, float("nan"), FAKE, ws, need), # NaN cut-off
        (FAKE, 10, FAKE, 12, p, -1.0, FAKE, ws, need),         # negative cut-off
        (FAKE, 10, FAKE, 12, _p("cdtw", window_ratio=-0.1), 1.0, FAKE, ws, need),
        (FAKE, 10, FAKE, 12, _p("cdtw", window_ratio=float("nan")), 1.0, FAKE, ws, need),
        (FAKE, 10, FAKE, 12, _p("msm", c=-1.0), 1.0, FAKE, ws, need),
        (FAKE, 10, FAKE, 12, _p("twe", nu=-1.0), 1.0, FAKE, ws, need),
        (FAKE, 10, FAKE, 12, _p("erp", gap=float("inf")), 1.0, FAKE, ws, need),
        (FAKE, 10, FAKE, 12, _p("wdtw", g=float("nan")), 1.0, FAKE, ws, need),
        (FAKE, 5000, FAKE, 12, p, 1.0, FAKE, ws, need),        # longer than supported
    ]
    for x, lx, y, ly, pp, cut, out, w, nb in cases:
        st = L.eap_distance(x, lx, y, ly, ctypes.byref(pp), cut, out, w, nb, None)
        assert st == eap.EAP_EINVAL, (lx, cut, pp.kind)
        assert len(L.eap_last_error()) > 0
    bad_kind = eap.Params(9, 1.0, 0, 0, 0, 0, 0)
    assert L.eap_distance(FAKE, 3, FAKE, 3, ctypes.byref(bad_kind), 1.0, FAKE, ws, need, None) == eap.EAP_EINVAL
    # workspace too small / missing
    assert L.eap_distance(FAKE, 10, FAKE, 12, ctypes.byref(p), 1.0, FAKE, ws, need - 1, None) == eap.EAP_EWORKSPACE
    assert L.eap_distance(FAKE, 10, FAKE, 12, ctypes.byref(p), 1.0, FAKE, None, need, None) == eap.EAP_EWORKSPACE


def test_multivariate_argument_errors(L):
    """Channels: 0..4, and more than one only for DTW and CDTW."""
    ws = ctypes.c_void_p(0x2000)
    for pp in (_p("dtw", dims=5), _p("dtw", dims=-1), _p("erp", dims=2), _p("msm", dims=3), _p("wdtw", dims=2)):
        assert L.eap_distance(FAKE, 10, FAKE, 12, ctypes.byref(pp), 1.0, FAKE, ws, 1 << 20, None) == eap.EAP_EINVAL
    for pp in (_p("dtw", dims=2), _p("cdtw", window_ratio=0.1, dims=4)):
        assert L.eap_distance_workspace(10, 12, ctypes.byref(pp)) > 0


def test_distance_noalloc_argument_errors(L):
    """The call without a workspace rejects the same arguments before it
    touches the device."""
    p = _p()
    cases = [
        (None, 10, FAKE, 12, p, 1.0, FAKE),
        (FAKE, 10, FAKE, 12, p, 1.0, None),                    # NULL output
        (FAKE, 0, FAKE, 12, p, 1.0, FAKE),
        (FAKE, 10, FAKE, 12, p, float("nan"), FAKE),
        (FAKE, 10, FAKE, 12, p, -1.0, FAKE),
        (FAKE, 10, FAKE, 12, _p("cdtw", window_ratio=-0.1), 1.0, FAKE),
        (FAKE, 10, FAKE, 12, _p("twe", lam=-1.0), 1.0, FAKE),
        (FAKE, 10, FAKE, 2049, p, 1.0, FAKE),                  # longer than supported
    ]
    for x, lx, y, ly, pp, cut, out in cases:
        assert L.eap_distance_noalloc(x, lx, y, ly, ctypes.byref(pp), cut, out, None) == eap.EAP_EINVAL, (lx, ly)
        assert len(L.eap_last_error()) > 0


def test_nn1_argument_errors(L):
    p = _p("msm", c=0.5)
    qo, ro = _off(5, 7), _off(4, 4, 9)
    o = eap.NNOpts(0, 1e-4, 0)
    pi = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need = L.eap_nn1_workspace(pi(qo), 2, pi(ro), 3, ctypes.byref(p), ctypes.byref(o))
    assert need > 0
    ws = ctypes.c_void_p(0x2000)

    def call(q=FAKE, qo_=qo, nq=2, r=FAKE, ro_=ro, nr=3, pp=p, oo=o, nb=need, idx=FAKE, dist=FAKE, w=ws):
        return L.eap_nn1(q, pi(qo_), nq, r, pi(ro_), nr, None, ctypes.byref(pp), ctypes.byref(oo), w, nb, idx,
                         dist, None, None)

    assert call(q=None) == eap.EAP_EINVAL
    assert call(idx=None) == eap.EAP_EINVAL
    assert call(nq=0) == eap.EAP_EINVAL
    assert call(qo_=np.array([1, 5, 12], dtype=np.int64)) == eap.EAP_EINVAL      # does not start at 0
    assert call(ro_=np.array([0, 4, 4, 13], dtype=np.int64)) == eap.EAP_EINVAL   # a zero-length series
    assert call(oo=eap.NNOpts(7, 1e-4, 0)) == eap.EAP_EINVAL
    assert call(oo=eap.NNOpts(1, float("nan"), 0)) == eap.EAP_EINVAL
    assert call(oo=eap.NNOpts(0, 1e-4, 64)) == eap.EAP_EINVAL   # unknown flag bit
    assert call(oo=eap.NNOpts(1, 1e-4, eap.FLAG_PRUNE_ONLY)) == eap.EAP_EINVAL   # prune-only is FP64
    assert call(oo=eap.NNOpts(0, 1e-4, 0, None, None, 4)) == eap.EAP_EINVAL      # unknown lb mode
    assert call(oo=eap.NNOpts(0, 1e-4, 0, None, None, -1)) == eap.EAP_EINVAL
    assert call(nb=need - 1) == eap.EAP_EWORKSPACE
    assert call(w=ctypes.c_void_p(0x2008)) == eap.EAP_EWORKSPACE   # not 256-byte aligned


def test_pairwise_argument_errors(L):
    p = _p("cdtw", window_ratio=0.1)
    so = _off(6, 6, 6)
    pi = so.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need = L.eap_pairwise_workspace(pi, 3, ctypes.byref(p))
    assert need > 0
    ws = ctypes.c_void_p(0x2000)
    assert L.eap_pairwise(FAKE, pi, 3, ctypes.byref(p), 2, ws, need, FAKE, None) == eap.EAP_EINVAL   # bad mode
    assert L.eap_pairwise(None, pi, 3, ctypes.byref(p), 0, ws, need, FAKE, None) == eap.EAP_EINVAL
    one = _off(6)
    assert L.eap_pairwise(FAKE, one.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, ctypes.byref(p), 0, ws, need,
                          FAKE, None) == eap.EAP_EINVAL
    assert L.eap_pairwise(FAKE, pi, 3, ctypes.byref(p), 0, ws, need - 8, FAKE, None) == eap.EAP_EWORKSPACE


def test_derivative_argument_errors(L):
    so = _off(6, 1, 9)
    pi = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need = L.eap_derivative_workspace(3)
    assert need >= 4 * 8 and L.eap_derivative_workspace(0) == 0
    ws = ctypes.c_void_p(0x2000)
    out = ctypes.c_void_p(0x100000)
    assert L.eap_derivative(None, pi(so), 3, out, ws, need, None) == eap.EAP_EINVAL
    assert L.eap_derivative(FAKE, pi(so), 3, None, ws, need, None) == eap.EAP_EINVAL
    assert L.eap_derivative(FAKE, pi(so), 0, out, ws, need, None) == eap.EAP_EINVAL
    assert L.eap_derivative(FAKE, pi(_off(6, 0, 9)), 3, out, ws, need, None) == eap.EAP_EINVAL   # zero length
    assert L.eap_derivative(FAKE, pi(so), 3, ctypes.c_void_p(0x1008), ws, need, None) == eap.EAP_EINVAL  # overlap
    assert L.eap_derivative(FAKE, pi(so), 3, out, ws, need - 1, None) == eap.EAP_EWORKSPACE
    assert L.eap_derivative(FAKE, pi(so), 3, out, None, need, None) == eap.EAP_EWORKSPACE


def test_znorm_argument_errors(L):
    so = np.array([0, 4, 4, 9], dtype=np.int64)      # a zero-length series
    pi = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    ok = np.array([0, 4, 9], dtype=np.int64)
    need = L.eap_znorm_workspace(2)
    assert need > 0
    ws = ctypes.c_void_p(0x4000)
    out = ctypes.c_void_p(0x100000)
    assert L.eap_znorm(FAKE, pi(so), 3, out, ws, need, None) == eap.EAP_EINVAL
    assert L.eap_znorm(None, pi(ok), 2, out, ws, need, None) == eap.EAP_EINVAL
    assert L.eap_znorm(FAKE, pi(ok), 2, out, ws, need - 1, None) == eap.EAP_EWORKSPACE
    assert L.eap_znorm(FAKE, pi(ok), 2, FAKE, ws, need, None) == eap.EAP_EINVAL      # out overlaps the input


def test_subseq_windows_argument_errors(L):
    out = ctypes.c_void_p(0x100000)
    assert L.eap_subseq_windows(None, 100, 10, out, None) == eap.EAP_EINVAL
    assert L.eap_subseq_windows(FAKE, 100, 10, None, None) == eap.EAP_EINVAL
    assert L.eap_subseq_windows(FAKE, 100, 0, out, None) == eap.EAP_EINVAL          # empty window
    assert L.eap_subseq_windows(FAKE, 100, 3000, out, None) == eap.EAP_EINVAL       # longer than supported
    assert L.eap_subseq_windows(FAKE, 9, 10, out, None) == eap.EAP_EINVAL           # series shorter than the window
    assert L.eap_subseq_windows(FAKE, 1 << 30, 2048, out, None) == eap.EAP_EINVAL   # over 2^31 - 1 values
    assert L.eap_subseq_windows(FAKE, 100, 10, ctypes.c_void_p(0x1100), None) == eap.EAP_EINVAL  # overlap


def test_workspace_sizes_grow_with_the_problem(L):
    p = _p("twe", nu=0.001, lam=1.0)
    o = eap.NNOpts(0, 1e-4, 0)
    pi = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    small = L.eap_nn1_workspace(pi(_off(8, 8)), 2, pi(_off(8, 8)), 2, ctypes.byref(p), ctypes.byref(o))
    big = L.eap_nn1_workspace(pi(_off(*[100] * 20)), 20, pi(_off(*[100] * 300)), 300, ctypes.byref(p),
                              ctypes.byref(o))
    assert 0 < small < big
    assert big >= 20 * 300 * 8


def test_wdtw_weights_bit_equal_to_oracle(L, orc):
    for g in (0.0, 0.05, 0.3, 1.0, 3.7):
        for n in (1, 2, 7, 128, 511, 512, 1024):
            a = eap.wdtw_weights(g, n)
            b = orc.wdtw_weights(g, n)
            assert a.tobytes() == b.tobytes(), (g, n)
    assert L.eap_wdtw_weights(float("nan"), 4, None) == eap.EAP_EINVAL


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(eap, "_lib", None)
    monkeypatch.setattr(eap, "LIB_PATH", str(tmp_path / "libeap.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        eap.lib()


def test_binding_checks_tensor_sizes_before_any_call():
    """The binding refuses device tensors smaller than the offsets or outputs
    address (the library reads and writes them through raw pointers).  Fake
    "device" tensors: the checks run before anything reaches the library."""
    import torch

    class Fake(torch.Tensor):
        pass

    def dev(n, dtype=torch.float64):
        t = torch.empty(n, dtype=dtype).as_subclass(Fake)
        t.__class__.is_cuda = property(lambda self: True)
        return t

    q, r = dev(10), dev(11)
    with pytest.raises(ValueError, match="offsets address"):
        eap.nn1(q, [0, 5, 12], r, [0, 11], dict(kind="dtw"))
    with pytest.raises(ValueError, match="offsets address"):
        eap.nn1(q, [0, 10], r, [0, 6, 12], dict(kind="dtw"))
    with pytest.raises(ValueError, match="needed"):
        eap.nn1(q, [0, 5, 10], r, [0, 11], dict(kind="dtw"), ws=dev(4096, torch.uint8),
                out=(dev(1, torch.int64), dev(2), None))
    with pytest.raises(TypeError, match="out\\[1\\]"):
        eap.nn1(q, [0, 10], r, [0, 11], dict(kind="dtw"), ws=dev(4096, torch.uint8),
                out=(dev(1, torch.int64), dev(1, torch.float32), None))
    with pytest.raises(TypeError, match="ws must be"):
        eap.nn1(q, [0, 10], r, [0, 11], dict(kind="dtw"), ws=dev(4096))
    with pytest.raises(ValueError, match="needed"):
        eap.subseq_windows(dev(100), 10, out=dev(90 * 10))
    with pytest.raises(ValueError, match="needed"):
        eap.pairwise(dev(30), [0, 10, 20, 30], dict(kind="dtw"), ws=dev(1 << 20, torch.uint8), out=dev(2))
    with pytest.raises(ValueError, match="offsets address"):
        eap.derivative(dev(10), [0, 4, 11], ws=dev(4096, torch.uint8))

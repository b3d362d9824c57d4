"""EAPruned elastic distances on MI355X: thin Python binding of libeap.so.

Every call marshals torch tensors (device values, current HIP stream) and host
offsets into the C ABI of include/eap.h; all of the computation happens in the
library's HIP kernels.  The binding fails loudly when the library is missing:
there is no CPU fallback.

    import torch, paper_2102_05221_amd as eap
    p = eap.params("cdtw", window_ratio=0.1)
    idx, dist, lab = eap.nn1(q_vals, q_off, r_vals, r_off, p, ref_labels=labels)
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = ["params", "distance", "distance_noalloc", "nn1", "pairwise", "workspace", "read_counters", "reset_counters",
           "profile_enable", "profile_take", "wdtw_weights", "EapError", "lib", "KINDS", "FLAG_NO_SEED",
           "FLAG_PLAIN", "FLAG_PREPARED", "FLAG_CANDIDATES", "FLAG_PRUNE_ONLY", "FLAG_NO_PRUNE", "LB_MODES", "derivative", "envelopes", "znorm", "subseq_windows", "subseq_search", "tune_nn1", "tune_set", "tune_reset", "capture_begin", "capture_end", "Graph",
           "Server"]

FLAG_NO_SEED = 1   # skip the seeding sweep (ablation)
FLAG_PLAIN = 2        # plain full DP for every pair: the baseline
FLAG_PREPARED = 4     # offsets and tables already in the workspace: kernels only (graph capture)
FLAG_CANDIDATES = 8   # the workspace holds what an earlier call derived from these same candidates
FLAG_PRUNE_ONLY = 16  # each pair under its own path bound, no shared best-so-far (Section 5's Prune)
FLAG_NO_PRUNE = 32    # early abandoning without pruning (EABase, Alg. 4)
LB_MODES = {"default": 0, "none": 1, "keogh": 2, "keogh2": 3}   # eap_nn_opts.lb (DTW and CDTW)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeap.so")
KINDS = {"dtw": 0, "cdtw": 1, "wdtw": 2, "erp": 3, "msm": 4, "twe": 5}

EAP_OK, EAP_EINVAL, EAP_ENOMEM, EAP_EDEVICE, EAP_EWORKSPACE = 0, -1, -2, -3, -4


class EapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libeap error {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("window_ratio", ctypes.c_double), ("g", ctypes.c_double),
                ("gap", ctypes.c_double), ("c", ctypes.c_double), ("nu", ctypes.c_double),
                ("lam", ctypes.c_double), ("dims", ctypes.c_int32)]


class NNOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("margin_rel", ctypes.c_double), ("flags", ctypes.c_int32),
                ("main_wait", ctypes.c_void_p), ("main_done", ctypes.c_void_p), ("lb", ctypes.c_int32)]


class Counters(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_uint64), ("pairs", ctypes.c_uint64), ("rechecks", ctypes.c_uint64),
                ("overflows", ctypes.c_uint64), ("stage_cells", ctypes.c_uint64 * 8),
                ("stage_pairs", ctypes.c_uint64 * 8), ("lb_pruned", ctypes.c_uint64)]


class ProfileRec(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int32), ("kernel", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("size", ctypes.c_int32), ("fp32", ctypes.c_int32), ("ms", ctypes.c_float),
                ("group", ctypes.c_int32), ("exact_diff", ctypes.c_int32)]


class TuneRec(ctypes.Structure):
    _fields_ = [("g", ctypes.c_int32), ("c", ctypes.c_int32), ("ms", ctypes.c_float), ("chosen", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("max_query_len", ctypes.c_int64),
                ("mem_budget", ctypes.c_size_t), ("precision", ctypes.c_int32), ("margin_rel", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("idx", ctypes.c_int64), ("dist", ctypes.c_double),
                ("label", ctypes.c_int32), ("status", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("queries", ctypes.c_int64), ("max_batch_seen", ctypes.c_int64),
                ("max_inflight", ctypes.c_int64), ("waiting", ctypes.c_int64)]


_lib = None
_vp, _i64, _d, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pP = ctypes.POINTER(Params)
_pO = ctypes.POINTER(NNOpts)


def lib():
    """The loaded libeap.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2102_05221_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.eap_source_hash.restype = ctypes.c_char_p
        L.eap_source_hash.argtypes = []
        from . import srchash
        built, here = L.eap_source_hash().decode(), srchash.source_hash()
        if built != here:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, sources {here}): "
                               "rebuild it with `python -m paper_2102_05221_amd.build`")
        L.eap_last_error.restype = ctypes.c_char_p
        L.eap_version.restype = ctypes.c_char_p
        L.eap_distance_workspace.restype = _sz
        L.eap_distance_workspace.argtypes = [_i64, _i64, _pP]
        L.eap_distance.restype = ctypes.c_int
        L.eap_distance.argtypes = [_vp, _i64, _vp, _i64, _pP, _d, _vp, _vp, _sz, _vp]
        L.eap_envelopes_workspace.restype = _sz
        L.eap_envelopes_workspace.argtypes = [_i64]
        L.eap_envelopes.restype = ctypes.c_int
        L.eap_envelopes.argtypes = [_vp, _pi64, _i64, _i64, _i64, _d, _vp, _vp, _vp, _sz, _vp]
        L.eap_screen_eps.restype = _d
        L.eap_screen_eps.argtypes = [ctypes.c_int32, ctypes.c_int32, _d, _d, _d]
        L.eap_screen_bound.restype = _d
        L.eap_screen_bound.argtypes = [ctypes.c_int32, ctypes.c_int32, _d, _d, _d]
        L.eap_distance_noalloc.restype = ctypes.c_int
        L.eap_distance_noalloc.argtypes = [_vp, _i64, _vp, _i64, _pP, _d, _vp, _vp]
        L.eap_nn1_workspace.restype = _sz
        L.eap_nn1_workspace.argtypes = [_pi64, _i64, _pi64, _i64, _pP, _pO]
        L.eap_nn1.restype = ctypes.c_int
        L.eap_nn1.argtypes = [_vp, _pi64, _i64, _vp, _pi64, _i64, _vp, _pP, _pO, _vp, _sz, _vp, _vp, _vp, _vp]
        L.eap_pairwise_workspace.restype = _sz
        L.eap_pairwise_workspace.argtypes = [_pi64, _i64, _pP]
        L.eap_pairwise.restype = ctypes.c_int
        L.eap_pairwise.argtypes = [_vp, _pi64, _i64, _pP, ctypes.c_int32, _vp, _sz, _vp, _vp]
        L.eap_subseq_windows.restype = ctypes.c_int
        L.eap_subseq_windows.argtypes = [_vp, _i64, _i64, _vp, _vp]
        L.eap_znorm_workspace.restype = _sz
        L.eap_znorm_workspace.argtypes = [_i64]
        L.eap_znorm.restype = ctypes.c_int
        L.eap_znorm.argtypes = [_vp, _pi64, _i64, _vp, _vp, _sz, _vp]
        L.eap_derivative_workspace.restype = _sz
        L.eap_derivative_workspace.argtypes = [_i64]
        L.eap_derivative.restype = ctypes.c_int
        L.eap_derivative.argtypes = [_vp, _pi64, _i64, _vp, _vp, _sz, _vp]
        L.eap_read_counters.restype = ctypes.c_int
        L.eap_read_counters.argtypes = [_vp, _sz, ctypes.POINTER(Counters), _vp]
        L.eap_reset_counters.restype = ctypes.c_int
        L.eap_reset_counters.argtypes = [_vp, _sz, _vp]
        L.eap_profile_enable.restype = ctypes.c_int
        L.eap_profile_enable.argtypes = [ctypes.c_int32]
        L.eap_profile_take.restype = ctypes.c_int
        L.eap_profile_take.argtypes = [ctypes.POINTER(ProfileRec), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.eap_tune_nn1.restype = ctypes.c_int
        L.eap_tune_nn1.argtypes = [_vp, _pi64, _i64, _vp, _pi64, _i64, _pP, _pO, _vp, _sz, _vp, _vp, _vp,
                                   ctypes.POINTER(TuneRec), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.eap_server_create.restype = ctypes.c_int
        L.eap_server_create.argtypes = [_vp, _pi64, _i64, _vp, _pP, ctypes.POINTER(ServerOpts),
                                        ctypes.POINTER(ctypes.c_void_p)]
        L.eap_server_submit.restype = ctypes.c_int
        L.eap_server_submit.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i64, _i64]
        L.eap_server_poll.restype = ctypes.c_int
        L.eap_server_poll.argtypes = [_vp, ctypes.POINTER(Result), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.eap_server_stats_get.restype = ctypes.c_int
        L.eap_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
        L.eap_server_counters.restype = ctypes.c_int
        L.eap_server_counters.argtypes = [_vp, ctypes.POINTER(Counters)]
        L.eap_server_destroy.restype = ctypes.c_int
        L.eap_server_destroy.argtypes = [_vp]
        L.eap_server_last_error.restype = ctypes.c_char_p
        L.eap_capture_begin.restype = ctypes.c_int
        L.eap_capture_begin.argtypes = [_vp]
        L.eap_capture_end.restype = ctypes.c_int
        L.eap_capture_end.argtypes = [_vp, ctypes.POINTER(ctypes.c_void_p)]
        L.eap_graph_launch.restype = ctypes.c_int
        L.eap_graph_launch.argtypes = [_vp, _vp]
        L.eap_graph_destroy.restype = ctypes.c_int
        L.eap_graph_destroy.argtypes = [_vp]
        L.eap_tune_set.restype = ctypes.c_int
        L.eap_tune_set.argtypes = [ctypes.c_int32, ctypes.c_int32, _i64, ctypes.c_int32, ctypes.c_int32]
        L.eap_tune_reset.restype = ctypes.c_int
        L.eap_tune_reset.argtypes = []
        L.eap_wdtw_weights.restype = ctypes.c_int
        L.eap_wdtw_weights.argtypes = [_d, _i64, ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _check(status: int):
    if status != EAP_OK:
        raise EapError(status, lib().eap_last_error().decode(errors="replace"))


def params(kind: str, window_ratio: float = math.inf, g: float = 0.0, gap: float = 0.0, c: float = 0.0,
           nu: float = 0.0, lam: float = 0.0, dims: int = 1) -> Params:
    """Distance parameters (eap_params); `kind` is one of KINDS; dims > 1:
    multivariate DTW / CDTW series of points of `dims` channels, stored point
    after point (offsets count points)."""
    return Params(KINDS[kind], float(window_ratio), float(g), float(gap), float(c), float(nu), float(lam), int(dims))


def params_from_dict(d: dict) -> Params:
    return params(d["kind"], d.get("window_ratio", math.inf), d.get("g", 0.0), d.get("gap", 0.0), d.get("c", 0.0),
                  d.get("nu", 0.0), d.get("lam", d.get("lambda", 0.0)), d.get("dims", 1))


def _as_params(p) -> Params:
    return p if isinstance(p, Params) else params_from_dict(p)


def _offsets(off) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    return a


def _sized(t, off, name, dims: int = 1):
    """The values tensor t must hold the off[-1] points (of `dims` values
    each) its offsets address (the library reads them through a raw pointer)."""
    if len(off) and t.numel() < int(off[-1]) * dims:
        raise ValueError(f"{name}: offsets address {int(off[-1]) * dims} values, the tensor holds {t.numel()}")


def _dims(p) -> int:
    return max(1, int(p.dims))


def _stream(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA/HIP tensor")
    return t


def _dev_buf(t, n, dtype, name):
    """A contiguous device tensor of `dtype` with at least n elements: the
    library writes or reads n of them through a raw pointer."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA/HIP tensor")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")
    return t


def _ws(ws):
    """A workspace: a contiguous device byte tensor (its size in bytes is passed)."""
    import torch
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.element_size() != 1 or not ws.is_contiguous():
        raise TypeError("ws must be a contiguous uint8 CUDA/HIP tensor (see workspace())")
    return ws


def workspace(nbytes: int, device):
    """A device byte buffer usable as a workspace."""
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def distance(x, y, p, cutoff: float = math.inf, ws=None, stream=None):
    """D(x, y) if D <= cutoff else +inf (Alg. 5), as a 1-element float64 tensor."""
    import torch
    _dev_f64(x, "x")
    _dev_f64(y, "y")
    p = _as_params(p)
    d = _dims(p)
    if x.numel() % d or y.numel() % d:
        raise ValueError(f"series of {x.numel()} and {y.numel()} values are not whole points of {d} channels")
    lx, ly = x.numel() // d, y.numel() // d
    need = lib().eap_distance_workspace(lx, ly, ctypes.byref(p))
    ws = workspace(need, x.device) if ws is None else _ws(ws)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib().eap_distance(x.data_ptr(), lx, y.data_ptr(), ly, ctypes.byref(p), float(cutoff),
                              out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, x.device)))
    return out


def distance_noalloc(x, y, p, cutoff: float = math.inf, out=None, stream=None):
    """As distance(), through eap_distance_noalloc: the library's static
    scratch instead of a workspace (calls on one GPU must not overlap)."""
    import torch
    _dev_f64(x, "x")
    _dev_f64(y, "y")
    p = _as_params(p)
    out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else _dev_buf(out, 1, torch.float64,
                                                                                              "out")
    _check(lib().eap_distance_noalloc(x.data_ptr(), x.numel(), y.data_ptr(), y.numel(), ctypes.byref(p),
                                      float(cutoff), out.data_ptr(), _stream(stream, x.device)))
    return out


def _lb_mode(lb) -> int:
    if lb not in LB_MODES:
        raise ValueError(f"lb must be one of {sorted(LB_MODES)}")
    return LB_MODES[lb]


def nn1_workspace_bytes(q_off, r_off, p, precision: int = 0, lb: str = "default") -> int:
    q_off, r_off = _offsets(q_off), _offsets(r_off)
    p = _as_params(p)
    o = NNOpts(precision, 1e-4, 0, None, None, _lb_mode(lb))
    return int(lib().eap_nn1_workspace(q_off.ctypes.data_as(_pi64), len(q_off) - 1, r_off.ctypes.data_as(_pi64),
                                       len(r_off) - 1, ctypes.byref(p), ctypes.byref(o)))


def _event_handle(ev, stream, device):
    """The hipEvent_t of a torch.cuda.Event (None for None); torch creates the
    event at its first record, so an unrecorded one is recorded once first."""
    if ev is None:
        return None
    if not ev.cuda_event:
        import torch
        ev.record(stream if stream is not None else torch.cuda.current_stream(device))
    return ctypes.c_void_p(ev.cuda_event)


def nn1(q, q_off, r, r_off, p, ref_labels=None, precision: int = 0, margin_rel: float = 1e-4, flags: int = 0,
        ws=None, stream=None, out=None, main_wait=None, main_done=None, lb: str = "default"):
    """1-NN search (Alg. 1).  q, r: float64 device tensors of concatenated
    series; q_off, r_off: host int64 offsets.  Returns (idx int64, dist float64,
    label int32 or None) device tensors.  main_wait / main_done: optional
    torch.cuda.Event the main sweep waits for / that is recorded after it, to
    chain several searches on several streams.  lb: lower bounds in front of
    the sweep for DTW and CDTW, one of LB_MODES ('default': LB_Keogh for
    CDTW, none for DTW; 'keogh2' adds the reversed LB_Keogh)."""
    import torch
    _dev_f64(q, "queries")
    _dev_f64(r, "candidates")
    q_off, r_off = _offsets(q_off), _offsets(r_off)
    nq, nr = len(q_off) - 1, len(r_off) - 1
    p = _as_params(p)
    _sized(q, q_off, "queries", _dims(p))
    _sized(r, r_off, "candidates", _dims(p))
    o = NNOpts(int(precision), float(margin_rel), int(flags), _event_handle(main_wait, stream, q.device),
               _event_handle(main_done, stream, q.device), _lb_mode(lb))
    ws = workspace(nn1_workspace_bytes(q_off, r_off, p, precision, lb), q.device) if ws is None else _ws(ws)
    if out is None:
        idx = torch.empty(nq, dtype=torch.int64, device=q.device)
        dist = torch.empty(nq, dtype=torch.float64, device=q.device)
        lab = torch.empty(nq, dtype=torch.int32, device=q.device) if ref_labels is not None else None
    else:
        idx, dist, lab = out
        _dev_buf(idx, nq, torch.int64, "out[0]")
        _dev_buf(dist, nq, torch.float64, "out[1]")
        if lab is not None:
            _dev_buf(lab, nq, torch.int32, "out[2]")
    lab_in = 0
    if ref_labels is not None:
        lab_in = _dev_buf(ref_labels, nr, torch.int32, "ref_labels").data_ptr()
    _check(lib().eap_nn1(q.data_ptr(), q_off.ctypes.data_as(_pi64), nq, r.data_ptr(), r_off.ctypes.data_as(_pi64),
                         nr, lab_in or None, ctypes.byref(p), ctypes.byref(o), ws.data_ptr(), ws.numel(),
                         idx.data_ptr(), dist.data_ptr(), lab.data_ptr() if lab is not None else None,
                         _stream(stream, q.device)))
    return idx, dist, lab


def tune_nn1(q, q_off, r, r_off, p, precision: int = 0, margin_rel: float = 1e-4, ws=None, stream=None) -> list:
    """Autotune the row sweep's shape (lanes per pair, columns per lane) for
    this distance, precision and length class on the given NN problem; later
    calls use the fastest.  Returns one dict per shape timed (g, c, ms,
    chosen); empty for distances the row sweep does not run."""
    import torch
    _dev_f64(q, "queries")
    _dev_f64(r, "candidates")
    q_off, r_off = _offsets(q_off), _offsets(r_off)
    nq, nr = len(q_off) - 1, len(r_off) - 1
    _sized(q, q_off, "queries")
    _sized(r, r_off, "candidates")
    p = _as_params(p)
    o = NNOpts(int(precision), float(margin_rel), 0)
    ws = workspace(nn1_workspace_bytes(q_off, r_off, p, precision), q.device) if ws is None else _ws(ws)
    idx = torch.empty(nq, dtype=torch.int64, device=q.device)
    dist = torch.empty(nq, dtype=torch.float64, device=q.device)
    recs = (TuneRec * 16)()
    n = ctypes.c_int32(0)
    _check(lib().eap_tune_nn1(q.data_ptr(), q_off.ctypes.data_as(_pi64), nq, r.data_ptr(),
                              r_off.ctypes.data_as(_pi64), nr, ctypes.byref(p), ctypes.byref(o), ws.data_ptr(),
                              ws.numel(), idx.data_ptr(), dist.data_ptr(), _stream(stream, q.device), recs, 16,
                              ctypes.byref(n)))
    return [dict(g=x.g, c=x.c, ms=float(x.ms), chosen=bool(x.chosen)) for x in recs[:n.value]]


def tune_set(kind: str, precision: int, lco_max: int, g: int, c: int) -> None:
    """Pin the row-sweep shape g x c for a distance, precision and length class."""
    _check(lib().eap_tune_set(KINDS[kind], int(precision), int(lco_max), int(g), int(c)))


def tune_reset() -> None:
    _check(lib().eap_tune_reset())


class Graph:
    """A HIP graph of NN searches recorded between capture_begin() and
    capture_end(); launch() replays them all with one graph launch."""

    def __init__(self, handle):
        self._h = handle

    def launch(self, stream=None, device=None):
        import torch
        _check(lib().eap_graph_launch(self._h, _stream(stream, device or torch.device("cuda", 0))))

    def close(self):
        if self._h:
            _check(lib().eap_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(status: int):
    if status != EAP_OK:
        raise EapError(status, lib().eap_server_last_error().decode(errors="replace"))


class Server:
    """Request server over a resident candidate set (see eap_server_* in
    include/eap.h): submit() queues a query (host values), poll() returns the
    finished (tag, idx, dist, label) tuples and admits waiting queries into
    free slots without blocking."""

    def __init__(self, refs, r_off, p, ref_labels=None, slots: int = 4, max_batch: int = 32,
                 max_query_len: int = 2048, mem_budget: int = 4 << 30, precision: int = 1,
                 margin_rel: float = 1e-4):
        import torch
        _dev_f64(refs, "candidates")
        self._refs = refs
        self._labels = ref_labels
        self._r_off = _offsets(r_off)
        _sized(refs, self._r_off, "candidates")
        self._p = _as_params(p)
        o = ServerOpts(int(slots), int(max_batch), int(max_query_len), int(mem_budget), int(precision),
                       float(margin_rel))
        lab = None
        if ref_labels is not None:
            lab = _dev_buf(ref_labels, len(self._r_off) - 1, torch.int32, "ref_labels").data_ptr()
        h = ctypes.c_void_p(None)
        _scheck(lib().eap_server_create(refs.data_ptr(), self._r_off.ctypes.data_as(_pi64), len(self._r_off) - 1,
                                        lab, ctypes.byref(self._p), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._buf = (Result * 4096)()

    def submit(self, values, tag: int) -> None:
        v = np.ascontiguousarray(values, dtype=np.float64)
        _scheck(lib().eap_server_submit(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(v),
                                        int(tag)))

    def poll(self) -> list:
        n = ctypes.c_int32(0)
        _scheck(lib().eap_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(n)))
        return [(r.tag, r.idx, r.dist, r.label) for r in self._buf[:n.value]]

    def stats(self) -> dict:
        s = ServerStats()
        _scheck(lib().eap_server_stats_get(self._h, ctypes.byref(s)))
        return dict(batches=s.batches, queries=s.queries, max_batch_seen=s.max_batch_seen,
                    max_inflight=s.max_inflight, waiting=s.waiting)

    def counters(self) -> dict:
        """Sweep counters summed over every batch run (waits for those in flight)."""
        c = Counters()
        _scheck(lib().eap_server_counters(self._h, ctypes.byref(c)))
        return dict(cells=c.cells, pairs=c.pairs, rechecks=c.rechecks, overflows=c.overflows,
                    stage_cells=list(c.stage_cells), stage_pairs=list(c.stage_pairs), lb_pruned=c.lb_pruned)

    def close(self) -> None:
        if self._h:
            _scheck(lib().eap_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture_begin(stream) -> None:
    """Start recording NN searches issued on `stream` (a torch stream other than
    the null stream); each must pass flags=FLAG_PREPARED."""
    _check(lib().eap_capture_begin(ctypes.c_void_p(stream.cuda_stream)))


def capture_end(stream) -> Graph:
    h = ctypes.c_void_p(None)
    _check(lib().eap_capture_end(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    return Graph(h)


def subseq_windows(s, m: int, stream=None, out=None):
    """Every window of length m of the device float64 series s, z-normalised
    on its own (sub-sequence search candidates, eap_subseq_windows), back to
    back: a device tensor of (len(s) - m + 1) * m values."""
    import torch
    _dev_f64(s, "series")
    n = s.numel()
    need = max(n - int(m) + 1, 0) * int(m)
    if out is None:
        out = torch.empty(need, dtype=torch.float64, device=s.device)
    _dev_buf(out, need, torch.float64, "out")
    _check(lib().eap_subseq_windows(s.data_ptr(), n, int(m), out.data_ptr(), _stream(stream, s.device)))
    return out


def subseq_search(query, series, p, precision: int = 0, stream=None, m: int = 0):
    """Sub-sequence search (Section 5.3): for each query, the start of the
    window of `series` closest to it (both device float64), every window and
    every query z-normalised, as one NN search over the windows.  `query` is
    one query, or with m > 0 the concatenation of queries of m values each.
    Returns (starts int64, distances float64) device tensors, one entry per
    query."""
    import numpy as np
    import torch
    m = int(m) if m else query.numel()
    if m < 1 or query.numel() % m:
        raise ValueError(f"query length {query.numel()} is not a multiple of m = {m}")
    nq = query.numel() // m
    q_off = np.arange(nq + 1, dtype=np.int64) * m
    zq = znorm(query, q_off, stream=stream)
    w = subseq_windows(series, m, stream=stream)
    r_off = np.arange(w.numel() // m + 1, dtype=np.int64) * m
    idx, dist, _ = nn1(zq, q_off, w, r_off, p, precision=precision, stream=stream)
    return idx, dist


def znorm(v, off, ws=None, stream=None, out=None):
    """Every series of the concatenated set v (device float64, host offsets
    off) z-normalised on its own, in one launch (eap_znorm): the queries of a
    sub-sequence search.  Returns a device tensor."""
    import torch
    _dev_f64(v, "series")
    off = _offsets(off)
    n = len(off) - 1
    _sized(v, off, "series")
    ws = workspace(int(lib().eap_znorm_workspace(n)), v.device) if ws is None else _ws(ws)
    if out is None:
        out = torch.empty_like(v)
    _dev_buf(out, int(off[-1]) if len(off) else 0, torch.float64, "out")
    _check(lib().eap_znorm(v.data_ptr(), off.ctypes.data_as(_pi64), n, out.data_ptr(), ws.data_ptr(), ws.numel(),
                           _stream(stream, v.device)))
    return out


def derivative(v, off, ws=None, stream=None, out=None):
    """Derivative series of the concatenated series v (device float64) with
    host offsets off, for DDTW / DCDTW / DWDTW (the estimate of Keogh and
    Pazzani; see eap_derivative in include/eap.h).  Returns a device tensor."""
    import torch
    _dev_f64(v, "series")
    off = _offsets(off)
    n = len(off) - 1
    _sized(v, off, "series")
    ws = workspace(int(lib().eap_derivative_workspace(n)), v.device) if ws is None else _ws(ws)
    if out is None:
        out = torch.empty_like(v)
    _dev_buf(out, int(off[-1]) if len(off) else 0, torch.float64, "out")
    _check(lib().eap_derivative(v.data_ptr(), off.ctypes.data_as(_pi64), n, out.data_ptr(), ws.data_ptr(),
                                ws.numel(), _stream(stream, v.device)))
    return out


def envelopes(v, off, npos: int, window_ratio: float, other_max: int = 0, ws=None, stream=None):
    """LB_Keogh envelopes (eap_envelopes): (up, lo), device tensors of shape
    (n, npos) for the series of v (device float64) with host offsets off."""
    import torch
    _dev_f64(v, "series")
    off = _offsets(off)
    n = len(off) - 1
    _sized(v, off, "series")
    ws = workspace(int(lib().eap_envelopes_workspace(n)), v.device) if ws is None else _ws(ws)
    up = torch.empty((n, npos), dtype=torch.float64, device=v.device)
    lo = torch.empty((n, npos), dtype=torch.float64, device=v.device)
    _check(lib().eap_envelopes(v.data_ptr(), off.ctypes.data_as(_pi64), n, int(npos), int(other_max),
                               float(window_ratio), up.data_ptr(), lo.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream(stream, v.device)))
    return up, lo


def pairwise_workspace_bytes(s_off, p) -> int:
    s_off = _offsets(s_off)
    p = _as_params(p)
    return int(lib().eap_pairwise_workspace(s_off.ctypes.data_as(_pi64), len(s_off) - 1, ctypes.byref(p)))


def pairwise(s, s_off, p, mode: str = "prune", ws=None, stream=None, out=None):
    """Condensed all-pairs distances; mode 'prune' (EAPruned with the path upper
    bound, Section 5 "Prune") or 'full' (plain DP)."""
    import torch
    _dev_f64(s, "series")
    s_off = _offsets(s_off)
    n = len(s_off) - 1
    p = _as_params(p)
    _sized(s, s_off, "series", _dims(p))
    ws = workspace(pairwise_workspace_bytes(s_off, p), s.device) if ws is None else _ws(ws)
    if out is None:
        out = torch.empty(max(n * (n - 1) // 2, 1), dtype=torch.float64, device=s.device)
    _dev_buf(out, n * (n - 1) // 2, torch.float64, "out")
    m = {"prune": 0, "full": 1}[mode]
    _check(lib().eap_pairwise(s.data_ptr(), s_off.ctypes.data_as(_pi64), n, ctypes.byref(p), m, ws.data_ptr(),
                              ws.numel(), out.data_ptr(), _stream(stream, s.device)))
    return out


def read_counters(ws, stream=None) -> dict:
    c = Counters()
    _check(lib().eap_read_counters(ws.data_ptr(), ws.numel(), ctypes.byref(c), _stream(stream, ws.device)))
    return dict(cells=c.cells, pairs=c.pairs, rechecks=c.rechecks, overflows=c.overflows,
                stage_cells=list(c.stage_cells), stage_pairs=list(c.stage_pairs), lb_pruned=c.lb_pruned)


def reset_counters(ws, stream=None):
    _check(lib().eap_reset_counters(ws.data_ptr(), ws.numel(), _stream(stream, ws.device)))


def profile_enable(on: bool = True):
    """Time every sweep launch with HIP events (see eap_profile_enable)."""
    _check(lib().eap_profile_enable(1 if on else 0))


def profile_take(cap: int = 4096) -> list:
    """Wait for the timed launches and return them as dicts (stage, kernel
    'rows'/'band', kind, size = strip width or band diagonals, group = lanes
    per pair, fp32, exact_diff, ms)."""
    buf = (ProfileRec * cap)()
    n = ctypes.c_int32(0)
    _check(lib().eap_profile_take(buf, cap, ctypes.byref(n)))
    inv = {v: k for k, v in KINDS.items()}
    return [dict(stage=r.stage, kernel=("band" if r.kernel else "rows"), kind=inv.get(r.kind, r.kind), size=r.size,
                 group=r.group, fp32=int(r.fp32), exact_diff=int(r.exact_diff), ms=float(r.ms))
            for r in buf[:n.value]]


def screen_eps(kind: str, B: float, N: float, A: float, exact_diff: bool = False) -> float:
    """The FP32 screen's certified bound on |V32 - B| (eap_screen_eps)."""
    return lib().eap_screen_eps(KINDS[kind], int(exact_diff), float(B), float(N), float(A))


def screen_bound(kind: str, b: float, N: float, A: float, exact_diff: bool = False) -> float:
    """Largest exact path cost whose FP32 value can be <= b (eap_screen_bound)."""
    return lib().eap_screen_bound(KINDS[kind], int(exact_diff), float(b), float(N), float(A))


def wdtw_weights(g: float, L: int) -> np.ndarray:
    out = np.empty(int(L), dtype=np.float64)
    _check(lib().eap_wdtw_weights(float(g), int(L), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out

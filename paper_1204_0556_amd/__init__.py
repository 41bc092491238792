"""MI355X ADMM LP decoder (arXiv 1204.0556) -- Python binding of liblpdec.so.

Every step of the decoder runs in the HIP library; this module only marshals
arguments through the C ABI declared in include/lpdec.h.  PyTorch supplies
device memory and streams.  If the library is missing the import fails: there
is no CPU fallback.

    import paper_1204_0556_amd as lp
    code = lp.Code(m, n, row_ptr, col_idx)          # H as CSR over checks
    x, iters, flags = lp.decode(code, llr)           # llr: float32 [B, n] on cuda
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "Code", "decode", "decode_noalloc", "decode_state", "decode_multi", "autotune_multi", "project", "default_params", "last_error",
    "LpdecError", "FLAG_CONVERGED", "FLAG_INTEGRAL", "FLAG_CODEWORD", "FLAG_CERTIFIED", "FLAG_INVALID",
    "MODE_AUTO", "MODE_RESIDENT", "MODE_STREAMED", "MODE_PERSISTENT_GLOBAL", "STORAGE_FP32", "STORAGE_FP16",
    "MAX_CHECK_DEGREE", "library_path", "Server", "EXECUTOR_GPU", "EXECUTOR_HOST_NULL",
    "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "decode_dual", "evaluate", "evaluate_multi",
    "EVAL_WORD_ERROR", "EVAL_CODEWORD", "EVAL_ML_ERROR",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "liblpdec.so")

FLAG_CONVERGED, FLAG_INTEGRAL, FLAG_CODEWORD, FLAG_CERTIFIED, FLAG_INVALID = 0x01, 0x02, 0x04, 0x08, 0x80
MODE_AUTO, MODE_RESIDENT, MODE_STREAMED, MODE_PERSISTENT_GLOBAL = 0, 1, 2, 3
STORAGE_FP32, STORAGE_FP16 = 0, 1
STATE_IN, STATE_OUT = 0x1, 0x2
EXECUTOR_GPU, EXECUTOR_HOST_NULL = 0, 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2
EVAL_WORD_ERROR, EVAL_CODEWORD, EVAL_ML_ERROR = 0x01, 0x02, 0x04
MAX_CHECK_DEGREE = 16
TUNE_VARIANTS = 4  # LPDEC_TUNE_VARIANTS

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "EBUSY"}


class LpdecError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lpdec {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_float), ("rho", ctypes.c_float), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_float), ("storage", ctypes.c_int32), ("mode", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("min_check_degree", ctypes.c_int32), ("max_check_degree", ctypes.c_int32),
                ("resident_capable", ctypes.c_int32), ("threads_per_frame", ctypes.c_int32)]


class _LaunchInfo(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threads", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("vgprs", ctypes.c_int32), ("runtime_blocks_per_cu", ctypes.c_int32),
                ("resource_blocks_per_cu", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_batch_frames", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_pending", ctypes.c_int32), ("executor", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("frames_completed", ctypes.c_int64),
                ("bits_completed", ctypes.c_int64), ("inflight_bytes", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("launches", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("peak_device_bytes", ctypes.c_int64), ("peak_concurrent_launches", ctypes.c_int32)]


def _load():
    if not os.path.exists(library_path):
        raise ImportError(f"{library_path} is missing: build it with paper_1204_0556_amd/build.py "
                          "(python -c 'import __graft_entry__; __graft_entry__.build()')")
    # torch brings its own HIP runtime.  Loading it first makes the library bind to
    # that same runtime, so tensors, streams and the library's launches share one;
    # loaded the other way round, the process would hold two HIP runtimes.
    import torch  # noqa: F401
    lib = ctypes.CDLL(library_path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.lpdec_default_params.restype = _Params
    lib.lpdec_last_error.restype = ctypes.c_char_p
    lib.lpdec_code_create.argtypes = [i32, i32, i64, P(i32), P(i32), P(vp)]
    lib.lpdec_code_create.restype = ctypes.c_int
    lib.lpdec_code_destroy.argtypes = [vp]
    lib.lpdec_code_destroy.restype = None
    lib.lpdec_code_get_info.argtypes = [vp, P(_Info)]
    lib.lpdec_code_get_info.restype = ctypes.c_int
    lib.lpdec_decode.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
    lib.lpdec_decode.restype = ctypes.c_int
    lib.lpdec_decode_noalloc.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
    lib.lpdec_decode_noalloc.restype = ctypes.c_int
    lib.lpdec_decode_state.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp, vp, i32, vp]
    lib.lpdec_decode_state.restype = ctypes.c_int
    lib.lpdec_decode_multi.argtypes = [P(vp), i32, i32, P(i32), P(i64), vp, i64, P(_Params), vp, P(i64), i64,
                                       vp, vp, vp]
    lib.lpdec_decode_multi.restype = ctypes.c_int
    lib.lpdec_code_launch_info.argtypes = [vp, P(_Params), P(_LaunchInfo)]
    lib.lpdec_code_launch_info.restype = ctypes.c_int
    lib.lpdec_code_set_tuning.argtypes = [vp, i32, i32, i32]
    lib.lpdec_code_set_tuning.restype = ctypes.c_int
    lib.lpdec_code_set_graph.argtypes = [vp, i32]
    lib.lpdec_code_set_graph.restype = ctypes.c_int
    lib.lpdec_autotune.argtypes = [vp, i32, vp, P(_Params), i32, P(i32), P(ctypes.c_float), vp]
    lib.lpdec_autotune.restype = ctypes.c_int
    lib.lpdec_autotune_multi.argtypes = [P(vp), i32, i32, P(i32), P(i64), vp, i64, P(_Params), i32, P(i32),
                                         P(ctypes.c_float), vp]
    lib.lpdec_autotune_multi.restype = ctypes.c_int
    lib.lpdec_decode_dual.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
    lib.lpdec_decode_dual.restype = ctypes.c_int
    lib.lpdec_evaluate.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lpdec_evaluate.restype = ctypes.c_int
    lib.lpdec_evaluate_multi.argtypes = [P(vp), i32, i32, P(i32), P(i64), vp, i64, vp, P(i64), i64, vp,
                                         vp, vp, vp, vp, vp]
    lib.lpdec_evaluate_multi.restype = ctypes.c_int
    lib.lpdec_project.argtypes = [i32, i32, vp, vp, vp]
    lib.lpdec_project.restype = ctypes.c_int
    lib.lpdec_server_default_config.restype = _ServerConfig
    lib.lpdec_server_create.argtypes = [P(vp), P(i32), i32, P(_Params), P(_ServerConfig), P(vp)]
    lib.lpdec_server_create.restype = ctypes.c_int
    lib.lpdec_server_submit.argtypes = [vp, i32, i32, vp, P(i64)]
    lib.lpdec_server_submit.restype = ctypes.c_int
    lib.lpdec_server_poll.argtypes = [vp, i64, P(i32)]
    lib.lpdec_server_poll.restype = ctypes.c_int
    lib.lpdec_server_wait.argtypes = [vp, i64, ctypes.c_double, vp, vp, vp, P(ctypes.c_double)]
    lib.lpdec_server_wait.restype = ctypes.c_int
    lib.lpdec_server_cancel.argtypes = [vp, i64]
    lib.lpdec_server_cancel.restype = ctypes.c_int
    lib.lpdec_server_get_stats.argtypes = [vp, P(_ServerStats)]
    lib.lpdec_server_get_stats.restype = ctypes.c_int
    lib.lpdec_server_destroy.argtypes = [vp]
    lib.lpdec_server_destroy.restype = None
    return lib


_lib = _load()


def last_error() -> str:
    return _lib.lpdec_last_error().decode()


def _check(status: int):
    if status != 0:
        raise LpdecError(status, last_error())


def default_params() -> dict:
    p = _lib.lpdec_default_params()
    return {k: getattr(p, k) for k, _ in _Params._fields_}


def _params(mu=None, rho=None, max_iter=None, tol=None, storage=None, mode=None) -> _Params:
    p = _lib.lpdec_default_params()
    if mu is not None: p.mu = float(mu)
    if rho is not None: p.rho = float(rho)
    if max_iter is not None: p.max_iter = int(max_iter)
    if tol is not None: p.tol = float(tol)
    if storage is not None: p.storage = int(storage)
    if mode is not None: p.mode = int(mode)
    return p


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Code:
    """A parity-check matrix H resident on the current device (lpdec_code_create)."""

    def __init__(self, m, n=None, row_ptr=None, col_idx=None):
        if n is None:  # a ParityCheckMatrix-like object
            H = m
            m, n, row_ptr, col_idx = H.m, H.n, H.row_ptr, H.col_idx
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        if rp.size != m + 1:
            raise ValueError("row_ptr must have m+1 entries")
        h = ctypes.c_void_p()
        _check(_lib.lpdec_code_create(int(m), int(n), int(ci.size),
                                      rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(h)))
        self._h = h
        self.m, self.n, self.nnz = int(m), int(n), int(ci.size)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("code is closed")
        return self._h

    @property
    def info(self) -> dict:
        inf = _Info()
        _check(_lib.lpdec_code_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def launch_info(self, **params) -> dict:
        """The launch a decode with these parameters (mode, storage) would use."""
        p = _params(**params)
        li = _LaunchInfo()
        _check(_lib.lpdec_code_launch_info(self.handle, ctypes.byref(p), ctypes.byref(li)))
        return {k: getattr(li, k) for k, _ in _LaunchInfo._fields_}

    def set_tuning(self, mode: int, blocks_per_cu: int = 0, variant: int = -1):
        _check(_lib.lpdec_code_set_tuning(self.handle, int(mode), int(blocks_per_cu), int(variant)))

    def set_graph(self, enable: bool):
        """Streamed form: replay blocks of iteration launches from a captured graph."""
        _check(_lib.lpdec_code_set_graph(self.handle, 1 if enable else 0))

    def autotune(self, llr, max_blocks_per_cu: int = 4, stream=None, **params):
        """Time decodes of the sample batch llr (float32 [B, n] CUDA tensor) over the
        launch candidates and keep the fastest.  Returns ((blocks_per_cu, variant),
        {(variant, blocks_per_cu): ms})."""
        torch = _torch()
        B = int(llr.shape[0]) if llr.dim() == 2 else 1
        if llr.numel() != B * self.n:
            raise ValueError("llr must be [batch, n]")
        p = _params(**params)
        mb = int(max_blocks_per_cu)
        best = (ctypes.c_int32 * 2)()
        ms = (ctypes.c_float * (TUNE_VARIANTS * mb))()
        _check(_lib.lpdec_autotune(self.handle, B, _dev_ptr(llr, torch.float32, "llr"), ctypes.byref(p),
                                   mb, best, ms, _stream(stream)))
        # entries of variant v at [v * mb + b]; forms without variants use v = 0 and report -1
        times = {}
        for v in range(TUNE_VARIANTS):
            for b in range(mb):
                if ms[v * mb + b] >= 0:
                    times[(v if best[1] >= 0 else -1, b + 1)] = float(ms[v * mb + b])
        return (best[0], best[1]), times

    def close(self):
        if self._h:
            _lib.lpdec_code_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode(code: Code, llr, out=None, stream=None, **params):
    """Decode llr (float32 [B, n] CUDA tensor).  Returns (x [B,n] f32, iters [B] i32, flags [B] u8)."""
    torch = _torch()
    B = int(llr.shape[0]) if llr.dim() == 2 else 1
    if llr.numel() != B * code.n:
        raise ValueError("llr must be [batch, n]")
    if out is None:
        out = (torch.empty((B, code.n), dtype=torch.float32, device=llr.device),
               torch.empty(B, dtype=torch.int32, device=llr.device),
               torch.empty(B, dtype=torch.uint8, device=llr.device))
    x, it, fl = out
    p = _params(**params)
    _check(_lib.lpdec_decode(code.handle, B, _dev_ptr(llr, torch.float32, "llr"), ctypes.byref(p),
                             _dev_ptr(x, torch.float32, "x"), _dev_ptr(it, torch.int32, "iters"),
                             _dev_ptr(fl, torch.uint8, "flags"), _stream(stream)))
    return x, it, fl


def decode_noalloc(code: Code, llr, out, stream=None, **params):
    """decode() through lpdec_decode_noalloc: the library allocates nothing (its
    scratch is a static device array per GPU); the caller supplies the outputs
    out = (x [B,n] f32, iters [B] i32, flags [B] u8).  Calls that overlap on one
    GPU race on that array.  Persistent forms only (FP32 storage)."""
    torch = _torch()
    B = int(llr.shape[0]) if llr.dim() == 2 else 1
    if llr.numel() != B * code.n:
        raise ValueError("llr must be [batch, n]")
    x, it, fl = out
    p = _params(**params)
    _check(_lib.lpdec_decode_noalloc(code.handle, B, _dev_ptr(llr, torch.float32, "llr"), ctypes.byref(p),
                                     _dev_ptr(x, torch.float32, "x"), _dev_ptr(it, torch.int32, "iters"),
                                     _dev_ptr(fl, torch.uint8, "flags"), _stream(stream)))
    return x, it, fl


def decode_dual(code: Code, llr, out=None, stream=None, mu=None, max_iter=None):
    """Dual subgradient ascent (Appendix A) on llr (float32 [B, n] CUDA tensor) with
    step mu.  Returns (x [B,n] f32 in {0,1}, iters [B] i32, flags [B] u8)."""
    torch = _torch()
    B = int(llr.shape[0]) if llr.dim() == 2 else 1
    if llr.numel() != B * code.n:
        raise ValueError("llr must be [batch, n]")
    if out is None:
        out = (torch.empty((B, code.n), dtype=torch.float32, device=llr.device),
               torch.empty(B, dtype=torch.int32, device=llr.device),
               torch.empty(B, dtype=torch.uint8, device=llr.device))
    x, it, fl = out
    p = _params(mu=mu, max_iter=max_iter)
    _check(_lib.lpdec_decode_dual(code.handle, B, _dev_ptr(llr, torch.float32, "llr"), ctypes.byref(p),
                                  _dev_ptr(x, torch.float32, "x"), _dev_ptr(it, torch.int32, "iters"),
                                  _dev_ptr(fl, torch.uint8, "flags"), _stream(stream)))
    return x, it, fl


def _eval_out(F, dev):
    torch = _torch()
    return (torch.empty(F, dtype=torch.int32, device=dev), torch.empty(F, dtype=torch.float64, device=dev),
            torch.empty(F, dtype=torch.float64, device=dev), torch.empty(F, dtype=torch.uint8, device=dev))


def evaluate(code: Code, llr, x, sent=None, stream=None):
    """Per-frame (bit_errors i32, cost_hat f64, cost_sent f64, outcome u8) of the
    rounded estimate x against the transmitted word (None: all-zero)."""
    torch = _torch()
    B = int(llr.shape[0]) if llr.dim() == 2 else 1
    if llr.numel() != B * code.n or x.numel() != B * code.n:
        raise ValueError("llr and x must be [batch, n]")
    if sent is not None and sent.numel() != B * code.n:
        raise ValueError("sent must be [batch, n]")
    be, ch, cs, oc = _eval_out(B, llr.device)
    sp = _dev_ptr(sent, torch.uint8, "sent") if sent is not None else None
    _check(_lib.lpdec_evaluate(code.handle, B, _dev_ptr(llr, torch.float32, "llr"), _dev_ptr(x, torch.float32, "x"),
                               sp, _dev_ptr(be, torch.int32, "bit_errors"), _dev_ptr(ch, torch.float64, "cost_hat"),
                               _dev_ptr(cs, torch.float64, "cost_sent"), _dev_ptr(oc, torch.uint8, "outcome"),
                               _stream(stream)))
    return be, ch, cs, oc


def evaluate_multi(codes, code_of_frame, llr_offset, llr, x, x_offset, sent=None, stream=None):
    """evaluate() over frames of several codes laid out as for decode_multi."""
    torch = _torch()
    cof = np.ascontiguousarray(code_of_frame, dtype=np.int32)
    lo = np.ascontiguousarray(llr_offset, dtype=np.int64)
    xo = np.ascontiguousarray(x_offset, dtype=np.int64)
    F = int(cof.size)
    be, ch, cs, oc = _eval_out(F, llr.device)
    handles = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
    sp = _dev_ptr(sent, torch.uint8, "sent") if sent is not None else None
    P = ctypes.POINTER
    _check(_lib.lpdec_evaluate_multi(handles, len(codes), F, cof.ctypes.data_as(P(ctypes.c_int32)),
                                     lo.ctypes.data_as(P(ctypes.c_int64)), _dev_ptr(llr, torch.float32, "llr"),
                                     int(llr.numel()), _dev_ptr(x, torch.float32, "x"),
                                     xo.ctypes.data_as(P(ctypes.c_int64)), int(x.numel()), sp,
                                     _dev_ptr(be, torch.int32, "bit_errors"), _dev_ptr(ch, torch.float64, "cost_hat"),
                                     _dev_ptr(cs, torch.float64, "cost_sent"), _dev_ptr(oc, torch.uint8, "outcome"),
                                     _stream(stream)))
    return be, ch, cs, oc


def decode_state(code: Code, llr, z=None, u=None, state_in=False, state_out=True, stream=None, **params):
    """Decode with the ADMM state (z, u = lambda/mu) in CSR edge order, [B, nnz] float32.
    Returns (x, iters, flags, z, u)."""
    torch = _torch()
    B = int(llr.shape[0])
    dev = llr.device
    if z is None:
        z = torch.zeros((B, code.nnz), dtype=torch.float32, device=dev)
    if u is None:
        u = torch.zeros((B, code.nnz), dtype=torch.float32, device=dev)
    x = torch.empty((B, code.n), dtype=torch.float32, device=dev)
    it = torch.empty(B, dtype=torch.int32, device=dev)
    fl = torch.empty(B, dtype=torch.uint8, device=dev)
    flags = (STATE_IN if state_in else 0) | (STATE_OUT if state_out else 0)
    p = _params(**params)
    _check(_lib.lpdec_decode_state(code.handle, B, _dev_ptr(llr, torch.float32, "llr"), ctypes.byref(p),
                                   _dev_ptr(x, torch.float32, "x"), _dev_ptr(it, torch.int32, "iters"),
                                   _dev_ptr(fl, torch.uint8, "flags"), _dev_ptr(z, torch.float32, "z"),
                                   _dev_ptr(u, torch.float32, "u"), flags, _stream(stream)))
    return x, it, fl, z, u


def decode_multi(codes, code_of_frame, llr_offset, llr, x_offset, x_len, stream=None, **params):
    """Frames of several codes in one persistent launch.  code_of_frame, llr_offset,
    x_offset are host int arrays; llr is a flat float32 CUDA tensor.
    Returns (x_flat [x_len], iters [F], flags [F])."""
    torch = _torch()
    cof = np.ascontiguousarray(code_of_frame, dtype=np.int32)
    lo = np.ascontiguousarray(llr_offset, dtype=np.int64)
    xo = np.ascontiguousarray(x_offset, dtype=np.int64)
    F = int(cof.size)
    dev = llr.device
    x = torch.empty(int(x_len), dtype=torch.float32, device=dev)
    it = torch.empty(F, dtype=torch.int32, device=dev)
    fl = torch.empty(F, dtype=torch.uint8, device=dev)
    handles = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
    p = _params(**params)
    _check(_lib.lpdec_decode_multi(handles, len(codes), F, cof.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _dev_ptr(llr, torch.float32, "llr"), int(llr.numel()), ctypes.byref(p),
                                   _dev_ptr(x, torch.float32, "x"),
                                   xo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(x_len),
                                   _dev_ptr(it, torch.int32, "iters"), _dev_ptr(fl, torch.uint8, "flags"),
                                   _stream(stream)))
    return x, it, fl


def autotune_multi(codes, code_of_frame, llr_offset, llr, max_blocks_per_cu=2, stream=None, **params):
    """Time decode_multi launches of this frame set over the fused launch's candidates
    (form x workgroups per CU x frame order) and keep the fastest as the tuning of
    codes[0].  Returns ((mode, blocks_per_cu, order), {(mode, order, blocks): ms})."""
    torch = _torch()
    cof = np.ascontiguousarray(code_of_frame, dtype=np.int32)
    lo = np.ascontiguousarray(llr_offset, dtype=np.int64)
    handles = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
    mb = int(max_blocks_per_cu)
    best = (ctypes.c_int32 * 3)()
    ms = (ctypes.c_float * (4 * mb))()
    p = _params(**params)
    P = ctypes.POINTER
    _check(_lib.lpdec_autotune_multi(handles, len(codes), int(cof.size), cof.ctypes.data_as(P(ctypes.c_int32)),
                                     lo.ctypes.data_as(P(ctypes.c_int64)), _dev_ptr(llr, torch.float32, "llr"),
                                     int(llr.numel()), ctypes.byref(p), mb, best, ms, _stream(stream)))
    times = {}
    for f, mode in enumerate((MODE_RESIDENT, MODE_PERSISTENT_GLOBAL)):
        for o in range(2):
            for b in range(mb):
                v = ms[(2 * f + o) * mb + b]
                if v >= 0:
                    times[(mode, o, b + 1)] = float(v)
    return (best[0], best[1], best[2]), times


def project(v, stream=None):
    """Pi_PPd row-wise for v float32 [count, d] (CUDA)."""
    torch = _torch()
    count, d = int(v.shape[0]), int(v.shape[1])
    z = torch.empty_like(v)
    _check(_lib.lpdec_project(d, count, _dev_ptr(v, torch.float32, "v"), _dev_ptr(z, torch.float32, "z"),
                              _stream(stream)))
    return z


class Server:
    """Continuous-batching request loop (lpdec_server_*).  Requests are host numpy
    arrays of LLRs; results come back as host numpy arrays.

    codes: list of Code (GPU executor), or code_n: list of code lengths with
    executor=EXECUTOR_HOST_NULL (scheduler tests without a GPU)."""

    def __init__(self, codes=None, code_n=None, budget_bytes=None, max_batch_frames=None, max_inflight=None,
                 max_pending=None, executor=EXECUTOR_GPU, **params):
        cfg = _lib.lpdec_server_default_config()
        if budget_bytes is not None: cfg.budget_bytes = int(budget_bytes)
        if max_batch_frames is not None: cfg.max_batch_frames = int(max_batch_frames)
        if max_inflight is not None: cfg.max_inflight = int(max_inflight)
        if max_pending is not None: cfg.max_pending = int(max_pending)
        cfg.executor = int(executor)
        self._codes = list(codes) if codes is not None else None
        if self._codes is not None:
            self.n = [c.n for c in self._codes]
            handles = (ctypes.c_void_p * len(self._codes))(*[c.handle.value for c in self._codes])
            cn = None
            k = len(self._codes)
        else:
            self.n = [int(v) for v in code_n]
            handles = None
            cn = (ctypes.c_int32 * len(self.n))(*self.n)
            k = len(self.n)
        p = _params(**params)
        h = ctypes.c_void_p()
        _check(_lib.lpdec_server_create(handles, cn, k, ctypes.byref(p), ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.config = {k2: getattr(cfg, k2) for k2, _ in _ServerConfig._fields_}

    def submit(self, code: int, llr) -> int:
        a = np.ascontiguousarray(llr, dtype=np.float32)
        frames = a.size // self.n[code]
        if frames * self.n[code] != a.size:
            raise ValueError("llr size is not a multiple of n")
        t = ctypes.c_int64()
        _check(_lib.lpdec_server_submit(self._h, int(code), int(frames), a.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(t)))
        self._last_frames = getattr(self, "_last_frames", {})
        self._last_frames[t.value] = (code, frames)
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32()
        _check(_lib.lpdec_server_poll(self._h, int(ticket), ctypes.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """(x [frames, n], iters [frames], flags [frames], latency_s)."""
        code, frames = self._last_frames[ticket]
        n = self.n[code]
        x = np.empty((frames, n), np.float32)
        it = np.empty(frames, np.int32)
        fl = np.empty(frames, np.uint8)
        lat = ctypes.c_double()
        _check(_lib.lpdec_server_wait(self._h, int(ticket), float(timeout), x.ctypes.data_as(ctypes.c_void_p),
                                      it.ctypes.data_as(ctypes.c_void_p), fl.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(lat)))
        del self._last_frames[ticket]
        return x, it, fl, lat.value

    def cancel(self, ticket: int):
        _check(_lib.lpdec_server_cancel(self._h, int(ticket)))
        self._last_frames.pop(ticket, None)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(_lib.lpdec_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lpdec_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""FP64 CPU oracle for ADMM LP decoding -- TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product: only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP library (``paper_1204_0556_amd``) and neither imports the
other.  The arithmetic lives in ``lpdec_oracle.c`` (plain C, FP64, no
fast-math); this module only marshals numpy arrays through ctypes.

Functions
  project(v)            Pi_PPd(v) by Algorithm 2's steps (Sec. 4.4), FP64.
  project_info(v)       the same plus (r, beta_opt, branch).
  max_linear(c)         Algorithm 3 (Appendix A): argmax c^T z over PP_d.
  decode(H, llr, ...)   Algorithm 1 with over-relaxation (Sec. 3.3, Sec. 5.2).
  dual_decode(H, llr, ...)  dual subgradient ascent with Algorithm 3 (Appendix A).
  evaluate(H, llr, x, sent)  word/bit errors and the ML lower-bound test (Sec. 5.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpdec_oracle.c")
_LIB = os.path.join(_HERE, "liblpdec_oracle.so")

BRANCH_ALL_ONE, BRANCH_BOX, BRANCH_SEARCH = 0, 1, 2
FLAG_CONVERGED, FLAG_INTEGRAL, FLAG_CODEWORD, FLAG_CERTIFIED, FLAG_INVALID = 0x01, 0x02, 0x04, 0x08, 0x80
EVAL_WORD_ERROR, EVAL_CODEWORD, EVAL_ML_ERROR = 0x01, 0x02, 0x04


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread", "-D_GNU_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.lpo_project.argtypes = [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int),
                                    P(ctypes.c_double), P(ctypes.c_int)]
        lib.lpo_project.restype = ctypes.c_int
        lib.lpo_max_linear.argtypes = [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
        lib.lpo_max_linear.restype = ctypes.c_int
        lib.lpo_decode_batch.argtypes = [
            ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), ctypes.c_int, P(ctypes.c_float),
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double, P(ctypes.c_double), P(ctypes.c_int),
            P(ctypes.c_ubyte), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int, ctypes.c_int,
            P(ctypes.c_longlong)]
        lib.lpo_decode_batch.restype = ctypes.c_int
        lib.lpo_dual_decode_batch.argtypes = [
            ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), ctypes.c_int, P(ctypes.c_float),
            ctypes.c_double, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_ubyte)]
        lib.lpo_dual_decode_batch.restype = ctypes.c_int
        lib.lpo_evaluate.argtypes = [
            ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), ctypes.c_int, P(ctypes.c_float),
            P(ctypes.c_double), P(ctypes.c_ubyte), P(ctypes.c_int), P(ctypes.c_double), P(ctypes.c_double),
            P(ctypes.c_ubyte)]
        lib.lpo_evaluate.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def project_info(v):
    """(z, r, beta_opt, branch) for one vector v (any length 1..64)."""
    lib = _load()
    v = np.ascontiguousarray(v, dtype=np.float64)
    z = np.empty_like(v)
    r = ctypes.c_int()
    beta = ctypes.c_double()
    br = ctypes.c_int()
    if lib.lpo_project(v.size, _ptr(v, ctypes.c_double), _ptr(z, ctypes.c_double), ctypes.byref(r),
                       ctypes.byref(beta), ctypes.byref(br)) != 0:
        raise ValueError("bad degree")
    return z, r.value, beta.value, br.value


def project(v):
    """Pi_PPd(v); v may be [d] or [k, d] (row-wise)."""
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 1:
        return project_info(v)[0]
    return np.stack([project_info(row)[0] for row in v])


def max_linear(c):
    lib = _load()
    c = np.ascontiguousarray(c, dtype=np.float64)
    z = np.empty_like(c)
    if lib.lpo_max_linear(c.size, _ptr(c, ctypes.c_double), _ptr(z, ctypes.c_double)) != 0:
        raise ValueError("bad degree")
    return z


def host_threads(cap: int = 16) -> int:
    """Worker threads for batch decodes: the cores this process may run on (its CPU
    affinity, which can be fewer than the machine has), at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


class Result:
    def __init__(self, x, iters, flags, z=None, u=None, proj_counts=None):
        self.x, self.iters, self.flags, self.z, self.u, self.proj_counts = x, iters, flags, z, u, proj_counts

    @property
    def hard(self):
        return (self.x >= 0.5).astype(np.uint8)


def decode(H, llr, mu=3.0, rho=1.9, max_iter=1000, tol=1e-5, state=False, z0=None, u0=None,
           nthreads=None) -> Result:
    """Decode frames of one code.  llr: float32 [frames, n].  With state=True the
    final replicas z and scaled duals u = lambda/mu ([frames, nnz], CSR edge order)
    are returned; z0/u0 warm-start the iteration."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    B, n = llr.shape
    if n != H.n:
        raise ValueError("llr width != code length")
    E = H.nnz
    rp = np.ascontiguousarray(H.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(H.col_idx, dtype=np.int32)
    x = np.empty((B, n), np.float64)
    it = np.empty(B, np.int32)
    fl = np.empty(B, np.uint8)
    warm = z0 is not None
    if warm or state:
        z = np.zeros((B, E), np.float64) if z0 is None else np.array(z0, dtype=np.float64, copy=True).reshape(B, E)
        u = np.zeros((B, E), np.float64) if u0 is None else np.array(u0, dtype=np.float64, copy=True).reshape(B, E)
        zp, up = _ptr(z, ctypes.c_double), _ptr(u, ctypes.c_double)
    else:
        z = u = None
        zp = up = None
    counts = np.zeros(3, np.int64)
    if nthreads is None:
        nthreads = host_threads()
    rc = lib.lpo_decode_batch(H.m, n, _ptr(rp, ctypes.c_int), _ptr(ci, ctypes.c_int), B,
                              _ptr(llr, ctypes.c_float), float(mu), float(rho), int(max_iter), float(tol),
                              _ptr(x, ctypes.c_double), _ptr(it, ctypes.c_int), _ptr(fl, ctypes.c_ubyte),
                              zp, up, int(warm), int(nthreads), _ptr(counts, ctypes.c_longlong))
    if rc != 0:
        raise ValueError(f"oracle decode failed ({rc})")
    return Result(x, it, fl, z, u, counts)


def dual_decode(H, llr, mu=3.0, max_iter=1000) -> Result:
    """Dual subgradient ascent (Appendix A) on frames of one code; mu is the step size."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    B, n = llr.shape
    if n != H.n:
        raise ValueError("llr width != code length")
    rp = np.ascontiguousarray(H.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(H.col_idx, dtype=np.int32)
    x = np.empty((B, n), np.float64)
    it = np.empty(B, np.int32)
    fl = np.empty(B, np.uint8)
    rc = lib.lpo_dual_decode_batch(H.m, n, _ptr(rp, ctypes.c_int), _ptr(ci, ctypes.c_int), B,
                                   _ptr(llr, ctypes.c_float), float(mu), int(max_iter),
                                   _ptr(x, ctypes.c_double), _ptr(it, ctypes.c_int), _ptr(fl, ctypes.c_ubyte))
    if rc != 0:
        raise ValueError(f"lpo_dual_decode_batch failed ({rc})")
    return Result(x, it, fl)


def evaluate(H, llr, x, sent=None) -> dict:
    """Per-frame bit errors, costs gamma^T xhat and gamma^T sent (FP64), and outcome
    bits (EVAL_WORD_ERROR, EVAL_CODEWORD, EVAL_ML_ERROR); sent=None is all-zero."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    B, n = llr.shape
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    if x.shape != (B, n) or n != H.n:
        raise ValueError("llr and x must be [frames, n]")
    sp = None
    if sent is not None:
        sent = np.ascontiguousarray(np.atleast_2d(sent), dtype=np.uint8)
        if sent.shape != (B, n):
            raise ValueError("sent must be [frames, n]")
        sp = _ptr(sent, ctypes.c_ubyte)
    rp = np.ascontiguousarray(H.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(H.col_idx, dtype=np.int32)
    be = np.empty(B, np.int32)
    ch = np.empty(B, np.float64)
    cs = np.empty(B, np.float64)
    oc = np.empty(B, np.uint8)
    rc = lib.lpo_evaluate(H.m, n, _ptr(rp, ctypes.c_int), _ptr(ci, ctypes.c_int), B, _ptr(llr, ctypes.c_float),
                          _ptr(x, ctypes.c_double), sp, _ptr(be, ctypes.c_int), _ptr(ch, ctypes.c_double),
                          _ptr(cs, ctypes.c_double), _ptr(oc, ctypes.c_ubyte))
    if rc != 0:
        raise ValueError(f"lpo_evaluate failed ({rc})")
    return {"bit_errors": be, "cost_hat": ch, "cost_sent": cs, "outcome": oc}

"""CPU oracle for the CG / SpMV path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg load
this package; the GPU library never imports, links or calls it, and it
imports nothing from the GPU library.

* ``cg_oracle.c`` (built into ``liborc.so``): plain serial FP64 SpMV for CSR,
  symmetric CSR (upper) and CSC, the format conversions, structure
  validation and the CG iteration of section III of the paper; plus a timing
  mode of the CSR iteration over OpenMP threads (``cg_csr_omp``), used only
  for the CPU baseline of the benchmark.
* ``exact.py``: the same SpMV and CG in exact rational arithmetic for tiny
  inputs.
* ``fem.py``: the finite-element operator A(nu) = sum_e nu_e K_e, the
  adjoint solve and the gradients dL/db, dL/dA (on the pattern) and dL/dnu
  (numpy FP64; pinned in ``tests/test_oracle_fem.py``).

Parity status: every function is pinned by the CPU tests (closed forms,
exact arithmetic, library routines, invariants); see the test module
``tests/test_oracle_pins.py``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

FMT_CSR, FMT_SYM_CSR, FMT_CSC = 0, 1, 2
OK, NOT_CONVERGED, ERR_ARG, ERR_STRUCTURE, ERR_BREAKDOWN, ERR_NONFINITE, ERR_NOMEM = 0, 1, -1, -2, -3, -4, -5
CHECK_SYMMETRY = 1


class OrcInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("ms_loop", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p


def load(path=None):
    """Load liborc.so, compiling it first if it is not there."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        _build.build(p)
    lib = ctypes.CDLL(p)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    for nm in ("orc_spmv_csr", "orc_spmv_csc", "orc_spmv_symcsr"):
        getattr(lib, nm).argtypes = [i64, _P, _P, _P, _P, _P]
        getattr(lib, nm).restype = None
    lib.orc_spmv.argtypes = [ctypes.c_int, i64, _P, _P, _P, _P, _P]
    lib.orc_dot.argtypes = [i64, _P, _P]
    lib.orc_dot.restype = ctypes.c_double
    lib.orc_dot_plain.argtypes = [i64, _P, _P]
    lib.orc_dot_plain.restype = ctypes.c_double
    lib.orc_dot_pairwise.argtypes = [i64, _P, _P]
    lib.orc_dot_pairwise.restype = ctypes.c_double
    lib.orc_dot_fused.argtypes = [i64, _P, _P]
    lib.orc_dot_fused.restype = ctypes.c_double
    lib.orc_transpose.argtypes = [i64, _P, _P, _P, _P, _P, _P]
    lib.orc_transpose.restype = ctypes.c_int
    lib.orc_csr_upper.argtypes = [i64, _P, _P, _P, _P, _P, _P]
    lib.orc_csr_upper.restype = i64
    lib.orc_sym_expand.argtypes = [i64, _P, _P, _P, _P, _P, _P]
    lib.orc_sym_expand.restype = i64
    lib.orc_validate.argtypes = [ctypes.c_int, i64, _P, _P, _P, ctypes.c_int, ctypes.c_uint32]
    lib.orc_validate.restype = ctypes.c_int
    lib.orc_cg.argtypes = [ctypes.c_int, i64, _P, _P, _P, _P, _P, ctypes.c_double, i32,
                           ctypes.POINTER(OrcInfo), _P, _P, _P, i32, _P, i32, i32, i32, ctypes.c_int]
    lib.orc_cg.restype = ctypes.c_int
    lib.orc_cg_csr_omp.argtypes = [i64, _P, _P, _P, _P, _P, ctypes.c_double, i32, ctypes.POINTER(OrcInfo),
                                   ctypes.POINTER(i32)]
    lib.orc_cg_csr_omp.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def spmv(fmt, ptr, idx, val, x, lib=None):
    """y = A x with A given 0-based in format fmt (plain definition)."""
    lib = lib or load()
    ptr, idx, val, x = _i32(ptr), _i32(idx), _f64(val), _f64(x)
    n = ptr.size - 1
    y = np.empty(n)
    lib.orc_spmv(fmt, n, _p(ptr), _p(idx), _p(val), _p(x), _p(y))
    return y


DOT_MODES = {"exact": 0, "plain": 1, "pairwise": 2, "fused": 3}


def dot(a, b, lib=None, plain=False, mode=None):
    """a'b: the exact value rounded once (default), the plain left-to-right
    loop (plain=True or mode="plain"), pairwise summation (mode="pairwise")
    or left-to-right fused multiply-adds (mode="fused")."""
    lib = lib or load()
    a, b = _f64(a), _f64(b)
    mode = mode or ("plain" if plain else "exact")
    fn = {"exact": lib.orc_dot, "plain": lib.orc_dot_plain, "pairwise": lib.orc_dot_pairwise,
          "fused": lib.orc_dot_fused}[mode]
    return fn(a.size, _p(a), _p(b))


def transpose(ptr, idx, val, lib=None):
    lib = lib or load()
    ptr, idx, val = _i32(ptr), _i32(idx), _f64(val)
    n = ptr.size - 1
    tp, ti, tv = np.empty(n + 1, np.int32), np.empty(idx.size, np.int32), np.empty(idx.size)
    if lib.orc_transpose(n, _p(ptr), _p(idx), _p(val), _p(tp), _p(ti), _p(tv)) != OK:
        raise MemoryError
    return tp, ti, tv


def csr_upper(ptr, col, val, lib=None):
    lib = lib or load()
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    n = ptr.size - 1
    up, uc, uv = np.empty(n + 1, np.int32), np.empty(col.size, np.int32), np.empty(col.size)
    m = lib.orc_csr_upper(n, _p(ptr), _p(col), _p(val), _p(up), _p(uc), _p(uv))
    return up, uc[:m].copy(), uv[:m].copy()


def sym_expand(uptr, ucol, uval, lib=None):
    lib = lib or load()
    uptr, ucol, uval = _i32(uptr), _i32(ucol), _f64(uval)
    n = uptr.size - 1
    cap = 2 * ucol.size
    p, c, v = np.empty(n + 1, np.int32), np.empty(max(cap, 1), np.int32), np.empty(max(cap, 1))
    m = lib.orc_sym_expand(n, _p(uptr), _p(ucol), _p(uval), _p(p), _p(c), _p(v))
    if m < 0:
        raise MemoryError
    return p, c[:m].copy(), v[:m].copy()


def validate(fmt, ptr, idx, val, base=0, flags=0, n=None, lib=None):
    lib = lib or load()
    ptr = None if ptr is None else _i32(ptr)
    idx = None if idx is None else _i32(idx)
    val = None if val is None else _f64(val)
    if n is None:
        n = ptr.size - 1
    return lib.orc_validate(fmt, n, _p(ptr), _p(idx), _p(val), base, flags)


def cg(fmt, ptr, idx, val, b, x0=None, tol=1e-10, maxit=None, history=0, x_stride=0, x_cap=0, lib=None,
       plain_dots=False, dots=None, x_first=None):
    """Run the oracle CG; returns (x, info dict, history dict or None).
    dots selects the arithmetic: "exact" scalar products (default, the
    reference), "plain" (the literal left-to-right loop; also
    plain_dots=True), "pairwise", or "fused" (fused multiply-adds in the
    scalar products and the three vector updates).
    x_stride / x_cap / x_first: snapshots of x after iterations x_first
    (default x_stride), x_first + x_stride, ... (x_cap of them) in hist["x"]."""
    dot_mode = DOT_MODES[dots or ("plain" if plain_dots else "exact")]
    lib = lib or load()
    ptr, idx, val, b = _i32(ptr), _i32(idx), _f64(val), _f64(b)
    n = ptr.size - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    if maxit is None:
        maxit = max(n, 1)
    info = OrcInfo()
    ah = bh = rh = xh = None
    if history:
        ah, bh, rh = np.zeros(history), np.zeros(history), np.zeros(history)
    if x_stride and x_cap:
        xh = np.zeros((x_cap, n))
    lib.orc_cg(fmt, n, _p(ptr), _p(idx), _p(val), _p(b), _p(x), tol, maxit, ctypes.byref(info),
               _p(ah), _p(bh), _p(rh), history, _p(xh), x_stride, x_cap,
               x_stride if x_first is None else x_first, dot_mode)
    d = dict(iters=info.iters, status=info.status, relres=info.relres, relres_true=info.relres_true,
             ms_loop=info.ms_loop)
    hist = None
    if history or xh is not None:
        k = min(info.iters, history) if history else 0
        hist = dict(alpha=None if ah is None else ah[:k], beta=None if bh is None else bh[:k],
                    res=None if rh is None else rh[:k], x=xh)
    return x, d, hist


def cg_csr_omp(ptr, col, val, b, x0=None, tol=1e-10, maxit=None, lib=None):
    """TIMING MODE of the CSR iteration on all OpenMP threads (not the
    correctness reference, which is ``cg``).  Returns (x, info dict with
    'threads')."""
    lib = lib or load()
    ptr, col, val, b = _i32(ptr), _i32(col), _f64(val), _f64(b)
    n = ptr.size - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    if maxit is None:
        maxit = max(n, 1)
    info = OrcInfo()
    nt = ctypes.c_int32(0)
    lib.orc_cg_csr_omp(n, _p(ptr), _p(col), _p(val), _p(b), _p(x), tol, maxit, ctypes.byref(info), ctypes.byref(nt))
    return x, dict(iters=info.iters, status=info.status, relres=info.relres, ms_loop=info.ms_loop,
                   threads=nt.value)

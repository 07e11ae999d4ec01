"""Python binding of libcgmi.so (ctypes; argument marshalling only).

Every function of include/cgmi.h is exposed under the same name.  Device
buffers are torch tensors on a ROCm device (float64, contiguous); their
``data_ptr()`` is passed straight through, and the work is ordered on the
caller's current torch stream.  Nothing here computes: if the library is not
built, or a tensor is not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcgmi.so")

CG_FMT_CSR, CG_FMT_SYM_CSR, CG_FMT_CSC = 0, 1, 2
FORMATS = {"csr": CG_FMT_CSR, "symcsr": CG_FMT_SYM_CSR, "csc": CG_FMT_CSC}
CG_OK, CG_NOT_CONVERGED = 0, 1
CG_ERR_ARG, CG_ERR_STRUCTURE, CG_ERR_BREAKDOWN, CG_ERR_NONFINITE = -1, -2, -3, -4
CG_ERR_NOMEM, CG_ERR_HIP, CG_ERR_UNSUPPORTED = -5, -6, -7
CG_CHECK_SYMMETRY = 1
CG_MIXED = 2
CG_LOWER = 4

# every symbol declared in include/cgmi.h
EXPORTS = ("cg_create", "cg_set_stream", "cg_set_batch", "cg_solve", "cg_solve_mixed", "cg_spmv", "cg_get_stats",
           "cg_destroy", "cg_status_string", "cg_last_error", "cg_analyze", "cg_analyze_export",
           "cg_batch_create", "cg_batch_set_stream", "cg_batch_spmm", "cg_batch_autotune", "cg_batch_solve",
           "cg_batch_destroy", "cg_batch_last_error", "cg_set_values", "cg_pattern_grad", "cg_fem_create",
           "cg_fem_set_stream", "cg_fem_pattern", "cg_fem_assemble", "cg_fem_nu_grad", "cg_fem_destroy",
           "cg_fem_last_error", "cg_analyze_panels", "cg_analyze_compact", "cg_spmv_static")


class cg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("ms", ctypes.c_double), ("outer", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class cg_plan_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("format", ctypes.c_int32),
                ("lanes_per_line", ctypes.c_int32), ("spmv_blocks", ctypes.c_int32),
                ("vec_blocks", ctypes.c_int32), ("colors", ctypes.c_int32),
                ("scatter_blocks", ctypes.c_int32), ("max_block_entries", ctypes.c_int32),
                ("slices", ctypes.c_int32),
                ("cached_loads", ctypes.c_int32), ("compact", ctypes.c_int32), ("slots", ctypes.c_int64),
                ("plan_bytes", ctypes.c_int64), ("parked", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class CgError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{cg_status_string(status)} ({status}): {detail}")
        self.status = status


_lib = None
_VP = ctypes.c_void_p


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes the dynamic linker bind this library to that
    # runtime, so the process has ONE HIP runtime and torch's device pointers
    # and streams are valid handles here.  Loaded the other way round, two
    # runtimes would compete for the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    lib.cg_create.argtypes = [ctypes.POINTER(_VP), ctypes.c_int, i64, _VP, _VP, _VP, ctypes.c_int, u32]
    lib.cg_set_stream.argtypes = [_VP, _VP]
    lib.cg_set_batch.argtypes = [_VP, i32]
    lib.cg_solve.argtypes = [_VP, _VP, _VP, dbl, i32, ctypes.POINTER(cg_info)]
    lib.cg_solve_mixed.argtypes = [_VP, _VP, _VP, dbl, i32, dbl, i32, ctypes.POINTER(cg_info)]
    lib.cg_spmv.argtypes = [_VP, _VP, _VP]
    lib.cg_spmv_static.argtypes = [_VP, _VP, _VP]
    lib.cg_get_stats.argtypes = [_VP, ctypes.POINTER(cg_plan_stats)]
    lib.cg_destroy.argtypes = [_VP]
    lib.cg_destroy.restype = None
    lib.cg_status_string.argtypes = [ctypes.c_int]
    lib.cg_status_string.restype = ctypes.c_char_p
    lib.cg_last_error.argtypes = [_VP]
    lib.cg_last_error.restype = ctypes.c_char_p
    lib.cg_analyze.argtypes = [ctypes.c_int, i64, _VP, _VP, _VP, ctypes.c_int, u32, ctypes.POINTER(cg_plan_stats)]
    lib.cg_analyze_export.argtypes = [ctypes.c_int, i64, _VP, _VP, ctypes.c_int] + [_VP] * 9
    lib.cg_batch_create.argtypes = [ctypes.POINTER(_VP), i32, _VP, _VP, _VP, _VP, i32, ctypes.c_int]
    lib.cg_batch_set_stream.argtypes = [_VP, _VP]
    lib.cg_batch_spmm.argtypes = [_VP, _VP, _VP]
    lib.cg_batch_autotune.argtypes = [_VP, _VP, _VP, _VP, _VP]
    lib.cg_batch_solve.argtypes = [_VP, _VP, _VP, dbl, i32, _VP, _VP, ctypes.POINTER(cg_info)]
    lib.cg_batch_destroy.argtypes = [_VP]
    lib.cg_batch_destroy.restype = None
    lib.cg_batch_last_error.argtypes = [_VP]
    lib.cg_batch_last_error.restype = ctypes.c_char_p
    lib.cg_analyze_panels.argtypes = [i64, _VP, _VP, ctypes.c_int] + [_VP] * 7
    lib.cg_analyze_compact.argtypes = [i64, _VP, _VP, ctypes.c_int] + [_VP] * 5
    lib.cg_set_values.argtypes = [_VP, _VP]
    lib.cg_pattern_grad.argtypes = [_VP, _VP, _VP, _VP]
    lib.cg_fem_create.argtypes = [ctypes.POINTER(_VP), i64, _VP, i64, _VP, _VP, i64]
    lib.cg_fem_set_stream.argtypes = [_VP, _VP]
    lib.cg_fem_pattern.argtypes = [_VP, ctypes.POINTER(i64), _VP, _VP]
    lib.cg_fem_assemble.argtypes = [_VP, _VP, _VP]
    lib.cg_fem_nu_grad.argtypes = [_VP, _VP, _VP, _VP]
    lib.cg_fem_destroy.argtypes = [_VP]
    lib.cg_fem_destroy.restype = None
    lib.cg_fem_last_error.argtypes = [_VP]
    lib.cg_fem_last_error.restype = ctypes.c_char_p
    for nm in ("cg_batch_create", "cg_batch_set_stream", "cg_batch_spmm", "cg_batch_autotune", "cg_batch_solve",
               "cg_set_values", "cg_pattern_grad", "cg_fem_create", "cg_fem_set_stream", "cg_fem_pattern",
               "cg_fem_assemble", "cg_fem_nu_grad", "cg_analyze_panels", "cg_analyze_compact"):
        getattr(lib, nm).restype = ctypes.c_int
    for nm in ("cg_create", "cg_set_stream", "cg_set_batch", "cg_solve", "cg_solve_mixed", "cg_spmv",
               "cg_spmv_static", "cg_get_stats",
               "cg_analyze", "cg_analyze_export"):
        getattr(lib, nm).restype = ctypes.c_int
    _lib = lib
    return lib


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_VP)


def _host_i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _host_f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _dev(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU (no CPU fallback)")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise TypeError(f"{name} must be a contiguous float64 tensor of {n} elements")
    return ctypes.c_void_p(t.data_ptr())


def _fmt(fmt):
    return FORMATS[fmt] if isinstance(fmt, str) else int(fmt)


# ----------------------------------------------------------- C names
def cg_status_string(status):
    return load().cg_status_string(int(status)).decode()


def cg_last_error(handle=None):
    return load().cg_last_error(handle).decode()


def cg_create(fmt, n, ptr, idx, vals, index_base=0, flags=0):
    """Returns (status, handle or None).  ptr / idx / vals are host arrays."""
    lib = load()
    ptr, idx, vals = _host_i32(ptr), _host_i32(idx), _host_f64(vals)
    h = _VP()
    st = lib.cg_create(ctypes.byref(h), _fmt(fmt), int(n), _np_ptr(ptr), _np_ptr(idx), _np_ptr(vals),
                       int(index_base), int(flags))
    return st, (h if st == CG_OK else None)


def cg_set_stream(handle, stream_ptr):
    return load().cg_set_stream(handle, _VP(stream_ptr))


def cg_set_batch(handle, iters):
    return load().cg_set_batch(handle, int(iters))


def cg_solve(handle, b_ptr, x_ptr, tol, maxit):
    """Raw call on device addresses; returns (status, info dict)."""
    info = cg_info()
    st = load().cg_solve(handle, _VP(b_ptr), _VP(x_ptr), float(tol), int(maxit), ctypes.byref(info))
    return st, info.as_dict()


def cg_solve_mixed(handle, b_ptr, x_ptr, tol, maxit, inner_tol, max_outer):
    """Raw call on device addresses; returns (status, info dict)."""
    info = cg_info()
    st = load().cg_solve_mixed(handle, _VP(b_ptr), _VP(x_ptr), float(tol), int(maxit), float(inner_tol),
                               int(max_outer), ctypes.byref(info))
    return st, info.as_dict()


def cg_spmv(handle, x_ptr, y_ptr):
    return load().cg_spmv(handle, _VP(x_ptr), _VP(y_ptr))


def cg_get_stats(handle):
    s = cg_plan_stats()
    st = load().cg_get_stats(handle, ctypes.byref(s))
    return st, s.as_dict()


def cg_destroy(handle):
    if handle:
        load().cg_destroy(handle)


def cg_analyze(fmt, n, ptr, idx, vals=None, index_base=0, flags=0):
    """Host-only validation + plan summary: returns (status, stats dict)."""
    ptr, idx, vals = _host_i32(ptr), _host_i32(idx), _host_f64(vals)
    s = cg_plan_stats()
    st = load().cg_analyze(_fmt(fmt), int(n), _np_ptr(ptr), _np_ptr(idx), _np_ptr(vals), int(index_base),
                           int(flags), ctypes.byref(s))
    return st, s.as_dict()


def cg_analyze_export(fmt, n, ptr, idx, index_base=0):
    """Host-only export of the scatter plan: returns (status, dict of arrays)."""
    st, stats = cg_analyze(fmt, n, ptr, idx, None, index_base)
    if st != CG_OK:
        return st, None
    nb, ns = stats["scatter_blocks"], stats["slots"]
    out = dict(color=np.zeros(nb, np.int32), line0=np.zeros(nb, np.int32), line1=np.zeros(nb, np.int32),
               entry0=np.zeros(nb, np.int32), entry1=np.zeros(nb, np.int32), slot0=np.zeros(nb + 1, np.int64),
               target=np.zeros(ns, np.int32), flags=np.zeros(ns, np.uint8), count=np.zeros(ns, np.int32))
    ptr, idx = _host_i32(ptr), _host_i32(idx)
    st = load().cg_analyze_export(_fmt(fmt), int(n), _np_ptr(ptr), _np_ptr(idx), int(index_base),
                                  *[_np_ptr(out[k]) for k in ("color", "line0", "line1", "entry0", "entry1",
                                                              "slot0", "target", "flags", "count")])
    out["stats"] = stats
    return st, out


def cg_analyze_compact(n, ptr, idx, index_base=0):
    """Host-only compact-block plan of a symmetric (upper) matrix; returns
    (status, dict of numpy arrays)."""
    lib = load()
    st, stats = cg_analyze(CG_FMT_SYM_CSR, n, ptr, idx, None, index_base)
    if st != CG_OK:
        return st, None
    nb, ns = stats["scatter_blocks"], stats["slots"]
    out = dict(block_of=np.zeros(max(n, 1), np.int32), slot0=np.zeros(nb + 1, np.int64),
               lines=np.zeros(max(nb, 1), np.int32), target=np.zeros(max(ns, 1), np.int32),
               count=np.zeros(max(ns, 1), np.int32))
    p = np.ascontiguousarray(ptr, dtype=np.int32)
    i = np.ascontiguousarray(idx, dtype=np.int32)
    st = lib.cg_analyze_compact(int(n), _np_ptr(p), _np_ptr(i), int(index_base),
                                *[_np_ptr(out[k]) for k in ("block_of", "slot0", "lines", "target", "count")])
    out["block_of"], out["lines"] = out["block_of"][:n], out["lines"][:nb]
    out["target"], out["count"] = out["target"][:ns], out["count"][:ns]
    out["stats"] = stats
    return st, out


def cg_analyze_panels(n, ptr, idx, index_base=0):
    """Host-only CSC panel plan; returns (status, dict of numpy arrays)."""
    lib = load()
    st, stats = cg_analyze(CG_FMT_CSC, n, ptr, idx, None, index_base)
    if st != CG_OK:
        return st, None
    p, i = _host_i32(ptr), _host_i32(idx)
    nnz, ns, nch = int(stats["nnz"]), int(stats["slots"]), int(stats["scatter_blocks"])
    out = dict(stats=stats, entry_src=np.empty(max(nnz, 1), np.int32), target=np.empty(max(ns, 1), np.int32),
               slot_ptr=np.empty(ns + 1, np.int32), panel=np.empty(max(ns, 1), np.int32),
               chunk_slot=np.empty(nch + 1, np.int32))
    w, fp = ctypes.c_int64(), ctypes.c_int32()
    st = lib.cg_analyze_panels(n, _np_ptr(p), _np_ptr(i), index_base, ctypes.byref(w), _np_ptr(out["entry_src"]),
                               _np_ptr(out["target"]), _np_ptr(out["slot_ptr"]), _np_ptr(out["panel"]),
                               _np_ptr(out["chunk_slot"]), ctypes.byref(fp))
    out["entry_src"], out["target"], out["panel"] = out["entry_src"][:nnz], out["target"][:ns], out["panel"][:ns]
    out["width"], out["first_parked"] = w.value, fp.value
    return st, out


# ------------------------------------------------------- convenience
class Solver:
    """A matrix on the device with its CG / SpMV entry points.

    Solver(fmt, ptr, idx, vals): host arrays (numpy), fmt in {"csr",
    "symcsr", "csc"} or CG_FMT_*.  solve(b, x0, tol, maxit) and spmv(x) take
    and return float64 GPU tensors.
    """

    def __init__(self, fmt, ptr, idx, vals, index_base=0, flags=0, batch=None, mixed=False):
        self.n = len(ptr) - 1
        self.nnz = len(idx)
        self.fmt = _fmt(fmt)
        if mixed:
            flags |= CG_MIXED
        st, h = cg_create(fmt, self.n, ptr, idx, vals, index_base, flags)
        if st != CG_OK:
            raise CgError(st, cg_last_error(None))
        self.h = h
        if batch is not None:
            cg_set_batch(h, batch)

    def _stream(self):
        import torch
        cg_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def solve(self, b, x0=None, tol=1e-10, maxit=None, check=True):
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        bp, xp = _dev(b, self.n, "b"), _dev(x, self.n, "x")
        self._stream()
        info = cg_info()
        st = load().cg_solve(self.h, bp, xp, float(tol), int(self.n if maxit is None else maxit),
                             ctypes.byref(info))
        d = info.as_dict()
        if check and st < 0 and st != CG_ERR_BREAKDOWN:
            raise CgError(st, cg_last_error(self.h))
        return x, d

    def solve_mixed(self, b, x0=None, tol=1e-10, maxit=None, inner_tol=1e-2, max_outer=50, check=True):
        """FP64 refinement around FP32 inner CG (handle created with mixed=True)."""
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        bp, xp = _dev(b, self.n, "b"), _dev(x, self.n, "x")
        self._stream()
        info = cg_info()
        st = load().cg_solve_mixed(self.h, bp, xp, float(tol), int(10 * self.n if maxit is None else maxit),
                                   float(inner_tol), int(max_outer), ctypes.byref(info))
        d = info.as_dict()
        if check and st < 0 and st != CG_ERR_BREAKDOWN:
            raise CgError(st, cg_last_error(self.h))
        return x, d

    def spmv(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        xp, yp = _dev(x, self.n, "x"), _dev(y, self.n, "y")
        self._stream()
        st = load().cg_spmv(self.h, xp, yp)
        if st != CG_OK:
            raise CgError(st, cg_last_error(self.h))
        return y

    def spmv_static(self, x, y=None):
        """y = A x through cg_spmv_static (scratch in the library's static
        device array; the library allocates nothing)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        xp, yp = _dev(x, self.n, "x"), _dev(y, self.n, "y")
        self._stream()
        st = load().cg_spmv_static(self.h, xp, yp)
        if st != CG_OK:
            raise CgError(st, cg_last_error(self.h))
        return y

    def set_values(self, vals):
        """New values (GPU float64 tensor, nnz, the entry order given at creation)."""
        vp = _dev(vals, self.nnz, "vals")
        self._stream()
        st = load().cg_set_values(self.h, vp)
        if st != CG_OK:
            raise CgError(st, cg_last_error(self.h))

    def pattern_grad(self, lam, x, out=None):
        """dL/d(stored values) from the adjoint lam and the solution x."""
        import torch
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=x.device)
        lp, xp, gp = _dev(lam, self.n, "lam"), _dev(x, self.n, "x"), _dev(out, self.nnz, "grad")
        self._stream()
        st = load().cg_pattern_grad(self.h, lp, xp, gp)
        if st != CG_OK:
            raise CgError(st, cg_last_error(self.h))
        return out

    def stats(self):
        return cg_get_stats(self.h)[1]

    def close(self):
        if self.h:
            cg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------- C-named thin wrappers
def cg_set_values(handle, vals_ptr):
    return load().cg_set_values(handle, _VP(vals_ptr))


def cg_pattern_grad(handle, lam_ptr, x_ptr, grad_ptr):
    return load().cg_pattern_grad(handle, _VP(lam_ptr), _VP(x_ptr), _VP(grad_ptr))


def cg_fem_last_error(handle=None):
    return (load().cg_fem_last_error(handle) or b"").decode()


def cg_fem_create(coords, tets, dof, n):
    """Host arrays coords (npts, 3) f64, tets (nelem, 4) int32, dof (npts,) int32."""
    lib = load()
    c = _host_f64(np.asarray(coords).reshape(-1))
    t = _host_i32(np.asarray(tets).reshape(-1))
    d = _host_i32(dof)
    h = _VP()
    st = lib.cg_fem_create(ctypes.byref(h), d.size, _np_ptr(c), t.size // 4, _np_ptr(t), _np_ptr(d), int(n))
    return st, h


def cg_fem_set_stream(handle, stream_ptr):
    return load().cg_fem_set_stream(handle, _VP(stream_ptr))


def cg_fem_pattern(handle, n):
    lib = load()
    nnz = ctypes.c_int64()
    st = lib.cg_fem_pattern(handle, ctypes.byref(nnz), None, None)
    if st != CG_OK:
        return st, None, None
    rp, col = np.empty(n + 1, np.int32), np.empty(max(nnz.value, 1), np.int32)
    st = lib.cg_fem_pattern(handle, ctypes.byref(nnz), _np_ptr(rp), _np_ptr(col))
    return st, rp, col[:nnz.value].copy()


def cg_fem_assemble(handle, nu_ptr, vals_ptr):
    return load().cg_fem_assemble(handle, _VP(nu_ptr), _VP(vals_ptr))


def cg_fem_nu_grad(handle, lam_ptr, x_ptr, grad_ptr):
    return load().cg_fem_nu_grad(handle, _VP(lam_ptr), _VP(x_ptr), _VP(grad_ptr))


def cg_fem_destroy(handle):
    load().cg_fem_destroy(handle)


class FemOperator:
    """Linear-tetrahedron operator A(nu) = sum_e nu_e K_e on the device.

    FemOperator(coords, tets, dof, n): host mesh arrays.  pattern() gives the
    full-CSR structure (host numpy), assemble(nu) the values, nu_grad(lam, x)
    the gradient -lam_e' K_e x_e, all on float64 GPU tensors.
    """

    def __init__(self, coords, tets, dof, n):
        self.n = int(n)
        self.nelem = int(np.asarray(tets).size // 4)
        st, h = cg_fem_create(coords, tets, dof, n)
        if st != CG_OK:
            raise CgError(st, cg_fem_last_error(None))
        self.h = h
        st, self.rowptr, self.col = cg_fem_pattern(h, self.n)
        if st != CG_OK:
            raise CgError(st, cg_fem_last_error(h))
        self.nnz = int(self.col.size)

    def _stream(self):
        import torch
        cg_fem_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def pattern(self):
        return self.rowptr, self.col

    def assemble(self, nu, out=None):
        import torch
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=nu.device)
        np_, vp = _dev(nu, self.nelem, "nu"), _dev(out, self.nnz, "vals")
        self._stream()
        st = load().cg_fem_assemble(self.h, np_, vp)
        if st != CG_OK:
            raise CgError(st, cg_fem_last_error(self.h))
        return out

    def nu_grad(self, lam, x, out=None):
        import torch
        if out is None:
            out = torch.empty(self.nelem, dtype=torch.float64, device=x.device)
        lp, xp, gp = _dev(lam, self.n, "lam"), _dev(x, self.n, "x"), _dev(out, self.nelem, "grad")
        self._stream()
        st = load().cg_fem_nu_grad(self.h, lp, xp, gp)
        if st != CG_OK:
            raise CgError(st, cg_fem_last_error(self.h))
        return out

    def close(self):
        if self.h:
            cg_fem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------- batches
def cg_batch_last_error(handle=None):
    return load().cg_batch_last_error(handle).decode()


def cg_batch_create(sys_off, ptr, idx, vals, nrhs=4, index_base=0):
    """Returns (status, handle or None); host arrays of the block-diagonal CSR."""
    lib = load()
    so = np.ascontiguousarray(sys_off, dtype=np.int64)
    ptr, idx, vals = _host_i32(ptr), _host_i32(idx), _host_f64(vals)
    h = _VP()
    st = lib.cg_batch_create(ctypes.byref(h), len(so) - 1, _np_ptr(so), _np_ptr(ptr), _np_ptr(idx), _np_ptr(vals),
                             int(nrhs), int(index_base))
    return st, (h if st == CG_OK else None)


class Batch:
    """Many independent systems (block-diagonal CSR) x nrhs right-hand sides.

    Vectors are torch float64 GPU tensors of shape (N, nrhs) (row-major, so
    entry (i, r) sits at i*nrhs + r)."""

    def __init__(self, sys_off, ptr, idx, vals, nrhs=4, index_base=0):
        st, h = cg_batch_create(sys_off, ptr, idx, vals, nrhs, index_base)
        if st != CG_OK:
            raise CgError(st, cg_batch_last_error(None))
        self.h, self.nrhs = h, nrhs
        self.N = int(sys_off[-1])
        self.nsys = len(sys_off) - 1

    def _stream(self):
        import torch
        load().cg_batch_set_stream(self.h, _VP(torch.cuda.current_stream().cuda_stream))

    def _check(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() \
                or tuple(t.shape) != (self.N, self.nrhs):
            raise TypeError(f"{name} must be a contiguous float64 GPU tensor of shape ({self.N}, {self.nrhs})")
        return _VP(t.data_ptr())

    def autotune(self):
        e, ln, w, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        self._stream()
        st = load().cg_batch_autotune(self.h, ctypes.byref(e), ctypes.byref(ln), ctypes.byref(w), ctypes.byref(us))
        if st != CG_OK:
            raise CgError(st, cg_batch_last_error(self.h))
        return dict(entries_per_block=e.value, lanes_per_row=ln.value, workgroups=w.value, us=us.value)

    def spmm(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        xp, yp = self._check(X, "X"), self._check(Y, "Y")
        self._stream()
        st = load().cg_batch_spmm(self.h, xp, yp)
        if st != CG_OK:
            raise CgError(st, cg_batch_last_error(self.h))
        return Y

    def solve(self, B, X0=None, tol=1e-10, maxit=None):
        """Returns (X, info dict, iters[nsys, nrhs], status[nsys, nrhs])."""
        import torch
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        bp, xp = self._check(B, "B"), self._check(X, "X")
        it = np.zeros((self.nsys, self.nrhs), np.int32)
        stv = np.zeros((self.nsys, self.nrhs), np.int32)
        info = cg_info()
        self._stream()
        load().cg_batch_solve(self.h, bp, xp, float(tol), int(10 * self.N if maxit is None else maxit),
                              _np_ptr(it), _np_ptr(stv), ctypes.byref(info))
        return X, info.as_dict(), it, stv

    def close(self):
        if self.h:
            load().cg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

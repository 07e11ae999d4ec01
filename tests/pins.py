"""Pins of the CPU oracle against facts that do not come from the oracle.

Every pin takes the oracle's shared library handle, so the same checks can be
run against copies of the oracle compiled with a planted mistake (see
``test_oracle_mutants.py``): a pin set is only trusted if every planted
mistake makes at least one pin fail.

Sources of truth used here: exact rational arithmetic (``oracle.exact`` and
``fractions``), LAPACK through numpy (Cholesky, eigenvalues), scipy.sparse
format conversions and products, closed-form spectra, and the floating-point
error bound |fl(sum) - sum| <= gamma_m sum |terms| (Higham, Accuracy and
Stability of Numerical Algorithms, section 3.1).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

import oracle
from oracle import exact
from paper_1010_4639_amd import workload as W

U = 2.0 ** -53


def gamma(m):
    return m * U / (1.0 - m * U)


def _csr(ptr, col, val, n=None, m=None):
    n = len(ptr) - 1 if n is None else n
    m = n if m is None else m
    return sp.csr_matrix((val, col, ptr), shape=(n, m))


def _csc_arrays(A):
    C = A.tocsc()
    C.sort_indices()
    return C.indptr.astype(np.int32), C.indices.astype(np.int32), C.data.copy()


def _upper_arrays(A):
    T = sp.triu(A, format="csr")
    T.sort_indices()
    return T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.copy()


def _row_bound(A, x):
    """gamma_m * sum_j |a_ij x_j| per row (m = row length, at least 1)."""
    absy = abs(A) @ np.abs(x)
    m = np.maximum(np.diff(A.indptr), 1)
    return gamma(m) * absy


# ----------------------------------------------------------------- SpMV
def pin_spmv_exact(lib):
    """CSR / CSC / symmetric-CSR products vs the exact rational product,
    within the rounding bound of an m-term sum."""
    for seed in range(3):
        ptr, col, val = W.random_sparse(14, density=0.3, seed=seed, empty_rows=2, long_rows=1)
        x = W.uniform_vector(14, seed=100 + seed)
        A = _csr(ptr, col, val)
        yex = np.array([float(t) for t in exact.spmv_csr_exact(ptr, col, val, x)])
        bound = _row_bound(A, x)
        y = oracle.spmv(oracle.FMT_CSR, ptr, col, val, x, lib=lib)
        assert np.all(np.abs(y - yex) <= bound + 1e-300), "CSR product off the exact value"
        cp, ri, cv = _csc_arrays(A)
        y = oracle.spmv(oracle.FMT_CSC, cp, ri, cv, x, lib=lib)
        assert np.all(np.abs(y - yex) <= bound + 1e-300), "CSC product off the exact value"
        # symmetric input for the triangle format
        sptr, scol, sval = W.random_spd_sparse(14, density=0.4, seed=seed)
        S = _csr(sptr, scol, sval)
        yex = np.array([float(t) for t in exact.spmv_csr_exact(sptr, scol, sval, x)])
        up, uc, uv = _upper_arrays(S)
        y = oracle.spmv(oracle.FMT_SYM_CSR, up, uc, uv, x, lib=lib)
        assert np.all(np.abs(y - yex) <= _row_bound(S, x) + 1e-300), "SymCSR product off the exact value"


def pin_spmv_library(lib):
    """Larger ragged non-symmetric products vs scipy's, rounding-bounded."""
    ptr, col, val = W.random_sparse(400, density=0.02, seed=7, empty_rows=5, long_rows=3)
    A = _csr(ptr, col, val)
    x = W.uniform_vector(400, seed=8)
    ref = A @ x
    bound = 2 * _row_bound(A, x)
    assert np.all(np.abs(oracle.spmv(oracle.FMT_CSR, ptr, col, val, x, lib=lib) - ref) <= bound + 1e-300)
    cp, ri, cv = _csc_arrays(A)
    assert np.all(np.abs(oracle.spmv(oracle.FMT_CSC, cp, ri, cv, x, lib=lib) - ref) <= bound + 1e-300)


def pin_three_formats_bitwise(lib):
    """For an exactly symmetric A with sorted indices, CSR, CSC and symmetric
    CSR products are bitwise equal: each y_i is the same left-to-right sum."""
    s = W.fem_p1_system(6, 5, 4, seed=11)
    A = _csr(s.rowptr, s.col, s.val)
    x = W.uniform_vector(s.n, seed=12)
    y1 = oracle.spmv(oracle.FMT_CSR, s.rowptr, s.col, s.val, x, lib=lib)
    cp, ri, cv = _csc_arrays(A)
    y2 = oracle.spmv(oracle.FMT_CSC, cp, ri, cv, x, lib=lib)
    up, uc, uv = _upper_arrays(A)
    y3 = oracle.spmv(oracle.FMT_SYM_CSR, up, uc, uv, x, lib=lib)
    assert np.array_equal(y1, y2) and np.array_equal(y1, y3), "formats differ bitwise"
    assert np.all(np.abs(y1 - A @ x) <= 2 * _row_bound(A, x) + 1e-300)


def _exact_dot(a, b):
    s = Fraction(0)
    for u, v in zip(a, b):
        s += Fraction(float(u)) * Fraction(float(v))
    return s


def pin_dot_exact(lib):
    """Scalar products: the default is the exact inner product rounded once
    (within 2 u of it even under heavy cancellation); the plain loop obeys the
    gamma_n bound of a left-to-right sum, the pairwise sum the gamma bound of
    its tree depth (Higham, ch. 4)."""
    rng = np.random.default_rng(17)
    for cancel in (False, True, "inexact"):
        a = rng.uniform(-1, 1, 600)
        b = rng.uniform(-1, 1, 600)
        if cancel == "inexact":          # inexact products that nearly cancel pairwise
            a = np.concatenate([a, -a])
            b = np.concatenate([b, b * (1 + 2.0 ** -20)])
        elif cancel:                       # condition number ~1e12: big terms that cancel exactly
            big = rng.uniform(-1, 1, 300) * 2.0 ** 40
            a = np.concatenate([a, big, -big])
            b = np.concatenate([b, np.full(300, 3.0), np.full(300, 3.0)])
            perm = rng.permutation(a.size)
            a, b = a[perm], b[perm]
        ex = _exact_dot(a, b)
        got = oracle.dot(a, b, lib=lib)
        assert abs(Fraction(got) - ex) <= 2 * U * abs(ex), "dot not within 2u of the exact value"
        plain = oracle.dot(a, b, lib=lib, plain=True)
        assert abs(Fraction(plain) - ex) <= Fraction(gamma(a.size)) * Fraction(float(np.sum(np.abs(a * b))) * 1.01)
        fu = oracle.dot(a, b, lib=lib, mode="fused")
        assert abs(Fraction(fu) - ex) <= Fraction(gamma(a.size)) * Fraction(float(np.sum(np.abs(a * b))) * 1.01)
        # pairwise: the depth of the summation tree, not n, bounds the error
        pw = oracle.dot(a, b, lib=lib, mode="pairwise")
        depth = int(np.ceil(np.log2(a.size))) + 8
        assert abs(Fraction(pw) - ex) <= Fraction(gamma(depth)) * Fraction(float(np.sum(np.abs(a * b))) * 1.01)
    # every term counts: a dropped product shows at once against the exact value
    for m in (1, 2, 7, 8, 9, 16, 17, 1000, 1023):
        a = rng.uniform(0.5, 1.0, m)
        b = rng.uniform(0.5, 1.0, m)
        ex = _exact_dot(a, b)
        pw = oracle.dot(a, b, lib=lib, mode="pairwise")
        assert abs(Fraction(pw) - ex) <= Fraction(gamma(int(np.ceil(np.log2(m))) + 8)) * ex, m
        fu = oracle.dot(a, b, lib=lib, mode="fused")
        assert abs(Fraction(fu) - ex) <= Fraction(gamma(m)) * ex, m


# ----------------------------------------------------------- conversions
def pin_conversions(lib):
    """Transpose / triangle / expansion vs scipy, integer- and bit-exact."""
    ptr, col, val = W.random_sparse(60, density=0.1, seed=3, empty_rows=3)
    A = _csr(ptr, col, val)
    tp, ti, tv = oracle.transpose(ptr, col, val, lib=lib)
    cp, ri, cv = _csc_arrays(A)
    assert np.array_equal(tp, cp) and np.array_equal(ti, ri) and np.array_equal(tv, cv), "transpose != scipy CSC"
    # T3: transposing twice is the identity
    p2, i2, v2 = oracle.transpose(tp, ti, tv, lib=lib)
    assert np.array_equal(p2, ptr) and np.array_equal(i2, col) and np.array_equal(v2, val)
    s = W.fem_p1_system(5, 4, 3, seed=5)
    S = _csr(s.rowptr, s.col, s.val)
    # T1: CSC of a symmetric A is its CSR
    tp, ti, tv = oracle.transpose(s.rowptr, s.col, s.val, lib=lib)
    assert np.array_equal(tp, s.rowptr) and np.array_equal(ti, s.col) and np.array_equal(tv, s.val)
    # upper triangle vs scipy.triu
    up, uc, uv = oracle.csr_upper(s.rowptr, s.col, s.val, lib=lib)
    rp, rc, rv = _upper_arrays(S)
    assert np.array_equal(up, rp) and np.array_equal(uc, rc) and np.array_equal(uv, rv), "upper != triu"
    # T2: expanding the stored triangle gives the full matrix back
    fp, fc, fv = oracle.sym_expand(up, uc, uv, lib=lib)
    assert np.array_equal(fp, s.rowptr) and np.array_equal(fc, s.col) and np.array_equal(fv, s.val)
    # T4: CSR of the upper triangle == CSC of the lower triangle
    L = sp.tril(S, format="csr")
    lp, li, lv = _csc_arrays(L)
    assert np.array_equal(lp, up) and np.array_equal(li, uc) and np.array_equal(lv, uv)


# ------------------------------------------------------------ validation
def malformed_cases():
    """(name, fmt, ptr, idx, val, base, flags, expected status)."""
    C, S, K = oracle.FMT_CSR, oracle.FMT_SYM_CSR, oracle.FMT_CSC
    p = np.array([0, 2, 3, 5], np.int32)
    i = np.array([0, 2, 1, 0, 2], np.int32)
    v = np.ones(5)
    sym_p = np.array([0, 2, 3, 4], np.int32)
    sym_i = np.array([0, 2, 1, 2], np.int32)
    sv = np.ones(4)
    cases = [
        ("ok_csr", C, p, i, v, 0, 0, oracle.OK),
        ("ok_csc", K, p, i, v, 0, 0, oracle.OK),
        ("ok_sym", S, sym_p, sym_i, sv, 0, 0, oracle.OK),
        ("ok_one_based", C, p + 1, i + 1, v, 1, 0, oracle.OK),
        ("bad_format", 7, p, i, v, 0, 0, oracle.ERR_ARG),
        ("bad_base", C, p, i, v, 2, 0, oracle.ERR_ARG),
        ("ptr0_not_base", C, p + 1, i, v, 0, 0, oracle.ERR_STRUCTURE),
        ("ptr_decreasing", C, np.array([0, 3, 2, 5], np.int32), i, v, 0, 0, oracle.ERR_STRUCTURE),
        ("idx_out_of_range", C, p, np.array([0, 3, 1, 0, 2], np.int32), v, 0, 0, oracle.ERR_STRUCTURE),
        ("idx_negative", C, p, np.array([0, 2, -1, 0, 2], np.int32), v, 0, 0, oracle.ERR_STRUCTURE),
        ("unsorted", C, p, np.array([2, 0, 1, 0, 2], np.int32), v, 0, 0, oracle.ERR_STRUCTURE),
        ("duplicate", C, p, np.array([0, 0, 1, 0, 2], np.int32), v, 0, 0, oracle.ERR_STRUCTURE),
        ("sym_lower_entry", S, np.array([0, 1, 3, 4], np.int32), np.array([0, 0, 1, 2], np.int32),
         sv, 0, 0, oracle.ERR_STRUCTURE),
        ("sym_missing_diag", S, np.array([0, 1, 2, 3], np.int32), np.array([0, 2, 2], np.int32),
         np.ones(3), 0, 0, oracle.ERR_STRUCTURE),
        ("sym_empty_row", S, np.array([0, 1, 1, 2], np.int32), np.array([0, 2], np.int32),
         np.ones(2), 0, 0, oracle.ERR_STRUCTURE),
        ("nan_value", C, p, i, np.array([1, np.nan, 1, 1, 1]), 0, 0, oracle.ERR_NONFINITE),
        ("inf_value", K, p, i, np.array([1, 1, np.inf, 1, 1]), 0, 0, oracle.ERR_NONFINITE),
        ("asym_pattern_flagged", C, p, np.array([0, 1, 1, 0, 2], np.int32), v, 0, oracle.CHECK_SYMMETRY,
         oracle.ERR_STRUCTURE),
        ("asym_pattern_unflagged", C, p, np.array([0, 1, 1, 0, 2], np.int32), v, 0, 0, oracle.OK),
        ("sym_pattern_flagged", C, np.array([0, 2, 3, 5], np.int32), np.array([0, 2, 1, 0, 2], np.int32),
         np.array([1.0, 2.0, 1.0, 2.0, 1.0]), 0, oracle.CHECK_SYMMETRY, oracle.OK),
        ("asym_values_flagged", C, np.array([0, 2, 3, 5], np.int32), np.array([0, 2, 1, 0, 2], np.int32),
         np.array([1.0, 2.0, 1.0, 3.0, 1.0]), 0, oracle.CHECK_SYMMETRY, oracle.ERR_STRUCTURE),
    ]
    return cases


def pin_validate(lib):
    for name, fmt, p, i, v, base, flags, want in malformed_cases():
        got = oracle.validate(fmt, p, i, v, base=base, flags=flags, lib=lib)
        assert got == want, f"validate {name}: {got} != {want}"


# -------------------------------------------------------------------- CG
def pin_cg_cholesky(lib):
    """CG solution vs LAPACK Cholesky on SPD systems, from zero and from a
    random start: ||x_cg - x_chol|| / ||x_chol|| <= 10 kappa tol."""
    cases = [W.random_spd_dense(48, seed=1)[:3], W.random_spd_sparse(300, density=0.02, seed=2)]
    for c, (ptr, col, val) in enumerate(cases):
        n = len(ptr) - 1
        M = _csr(ptr, col, val).toarray()
        b = W.uniform_vector(n, seed=20 + c) * 3.0
        Lc = np.linalg.cholesky(M)
        xs = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
        kappa = np.linalg.cond(M)
        tol = 1e-12
        for x0 in (None, W.uniform_vector(n, seed=30 + c)):
            x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, b, x0=x0, tol=tol, maxit=10 * n, lib=lib)
            assert info["status"] == oracle.OK, info
            err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
            assert err <= 10 * kappa * tol, (err, kappa)
            # the reported true residual is the residual of the returned x
            rt = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
            assert abs(rt - info["relres_true"]) <= 1e-3 * rt + 1e-15
            assert info["relres"] <= tol


def _laplacian_7pt(nx, ny, nz):
    s = W.fem_p1_system(nx, ny, nz, jitter=0.0, iron_frac=0.0, seed=9, with_rhs=False)
    # drop the structural zeros of the diagonal couplings: integer stencil
    A = _csr(s.rowptr, s.col, np.round(s.val))
    return A


def pin_cg_exact_termination(lib):
    """Exact CG on the 7-point Laplacian of a 3^3 / 4^3 grid ends after as
    many steps as the matrix has distinct eigenvalues, with x exact; the
    FP64 oracle reaches a tiny residual at that same step."""
    for g in (3, 4):
        A = _laplacian_7pt(g, g, g)
        A.eliminate_zeros()
        ptr, col, val = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
        n = A.shape[0]
        xt = np.random.default_rng(g).integers(-8, 9, size=n).astype(np.float64)
        b = A @ xt                     # integers: exact in FP64
        lam = np.linalg.eigvalsh(A.toarray())
        distinct = 1 + int(np.sum(np.diff(np.sort(lam)) > 1e-9))
        x_ex, steps = exact.cg_exact(ptr, col, val, b)
        assert steps == distinct, (g, steps, distinct)
        assert all(xe == Fraction(float(t)) for xe, t in zip(x_ex, xt))
        x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, b, tol=0.0, maxit=steps, lib=lib)
        assert info["iters"] == steps
        assert info["relres_true"] <= 1e-14, info
        assert np.linalg.norm(x - xt) / np.linalg.norm(xt) <= 1e-14


def _lanczos_ritz(alpha, beta):
    """Ritz values of the CG-Lanczos tridiagonal built from alpha_k, beta_k."""
    k = len(alpha)
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    d[0] = 1.0 / alpha[0]
    for j in range(1, k):
        d[j] = 1.0 / alpha[j] + beta[j - 1] / alpha[j - 1]
        e[j - 1] = math.sqrt(beta[j - 1]) / alpha[j - 1]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    return np.linalg.eigvalsh(T)


def pin_cg_lanczos_spectrum(lib):
    """On the 7-point Laplacian the extreme Ritz values of the CG recurrence
    converge to the closed-form extreme eigenvalues
    4[sin^2(p pi / 2(nx+1)) + sin^2(q pi / 2(ny+1)) + sin^2(r pi / 2(nz+1))]."""
    nx, ny, nz = 10, 12, 14
    A = _laplacian_7pt(nx, ny, nz)
    ptr, col, val = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
    b = W.uniform_vector(A.shape[0], seed=5)

    def lam(p, q, r):
        return 4 * (math.sin(p * math.pi / (2 * (nx + 1))) ** 2 + math.sin(q * math.pi / (2 * (ny + 1))) ** 2
                    + math.sin(r * math.pi / (2 * (nz + 1))) ** 2)
    lo, hi = lam(1, 1, 1), lam(nx, ny, nz)
    _, info, h = oracle.cg(oracle.FMT_CSR, ptr, col, val, b, tol=1e-13, maxit=2000, history=2000, lib=lib)
    assert info["status"] == oracle.OK
    ritz = _lanczos_ritz(h["alpha"], h["beta"])
    assert abs(ritz[0] - lo) <= 1e-8 * lo, (ritz[0], lo)
    assert abs(ritz[-1] - hi) <= 1e-8 * hi, (ritz[-1], hi)
    assert np.all(h["alpha"] > 0) and np.all(h["beta"] > 0)


def pin_cg_invariants(lib):
    """On a jittered FEM system with iron: the A-norm of the error never
    grows, consecutive true residuals are orthogonal in the first steps, the
    stop is at the FIRST step whose recursive residual meets tol*||b||, and
    the error vs x_true respects kappa_est * relres_true."""
    s = W.fem_p1_system(9, 8, 7, nu_iron=1e-2, seed=4)
    A = _csr(s.rowptr, s.col, s.val)
    b = s.b * 7.5                      # ||b|| far from 1: the criterion is relative
    xt = s.x_true * 7.5
    tol = 1e-10
    x, info, h = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, b, tol=tol, maxit=5000,
                           history=5000, x_stride=1, x_cap=5000, lib=lib)
    assert info["status"] == oracle.OK
    k = info["iters"]
    nb = np.linalg.norm(b)
    res = h["res"]
    assert res[k - 1] <= tol * nb and res[k - 2] > tol * nb, "not the first step meeting the criterion"
    X = h["x"][:k]
    from scipy.sparse.linalg import spsolve
    xs = spsolve(A.tocsc(), b)          # direct solution (SuperLU), not the oracle
    E = X - xs
    # A-norm via the true residual route, independent of the oracle's product
    an = np.einsum("ij,ij->i", E, (A @ E.T).T)
    assert np.all(np.diff(an) <= 1e-12 * an[:-1] + 1e-28), "A-norm error increased"
    R = b[None, :] - (A @ X.T).T
    for j in range(min(8, k - 1)):
        c = abs(R[j + 1] @ R[j]) / (np.linalg.norm(R[j + 1]) * np.linalg.norm(R[j]))
        assert c <= 1e-8, (j, c)
    assert np.all(h["alpha"] > 0) and np.all(h["beta"] > 0)
    ritz = _lanczos_ritz(h["alpha"], h["beta"])
    kappa_est = ritz[-1] / ritz[0]
    err = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    assert err <= 2 * kappa_est * info["relres_true"] + 1e-14, (err, kappa_est, info)
    assert info["relres_true"] <= 2 * tol


def pin_cg_alternative_evaluations(lib):
    """The iteration in every alternative arithmetic (plain, pairwise or
    fused scalar products; fused vector updates) is still CG: it converges
    on a jittered FEM system with iron to the direct solution (energy norm,
    SuperLU), meets the tolerance on the true residual, takes the first
    steps of the exactly rounded run to rounding level, and its iterates
    snapshot where asked (from a chosen step)."""
    s = W.fem_p1_system(9, 8, 7, nu_iron=1e-2, seed=4)
    A = _csr(s.rowptr, s.col, s.val)
    from scipy.sparse.linalg import spsolve
    xs = spsolve(A.tocsc(), s.b)
    ea = float(np.sqrt(xs @ (A @ xs)))
    _, i0, h0 = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=1e-10, maxit=5000, history=8, lib=lib)
    for mode in ("plain", "pairwise", "fused"):
        x, info, h = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=1e-10, maxit=5000, history=8,
                               lib=lib, dots=mode)
        assert info["status"] == oracle.OK and info["relres_true"] <= 2e-10, (mode, info)
        e = x - xs
        assert np.sqrt(e @ (A @ e)) <= 1e-8 * ea, mode
        assert np.allclose(h["alpha"][:5], h0["alpha"][:5], rtol=1e-12, atol=0), mode
        assert np.allclose(h["beta"][:5], h0["beta"][:5], rtol=1e-11, atol=0), mode
        assert abs(info["iters"] - i0["iters"]) <= 0.1 * i0["iters"], (mode, info, i0)
    # fused updates are single roundings: x1 = fl(alpha p0 + x0) exactly
    # (Fraction arithmetic, one rounding), which for a generic x0 differs
    # from the twice-rounded x0 + fl(alpha p0) in some entries
    n = 64
    rng = np.random.default_rng(23)
    d = rng.uniform(1.0, 3.0, n)
    ip, ic = np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    x1, _, h = oracle.cg(oracle.FMT_CSR, ip, ic, d, b, x0=x0, tol=0.0, maxit=1, history=1, lib=lib, dots="fused")
    p0 = b - d * x0                        # r0 = b - A x0 (one product and one subtraction per entry)
    al = Fraction(float(h["alpha"][0]))
    want = np.array([float(al * Fraction(float(p0[i])) + Fraction(float(x0[i]))) for i in range(n)])
    assert np.array_equal(x1, want), "fused x update is not one rounding"
    assert np.any(want != x0 + float(al) * p0)
    # snapshots from a chosen step: x after steps 5, 8, 11 == runs stopped there
    _, _, h = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=0.0, maxit=11, x_stride=3, x_cap=3,
                        x_first=5, lib=lib)
    for j, k in enumerate((5, 8, 11)):
        xk, _, _ = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=0.0, maxit=k, lib=lib)
        assert np.array_equal(h["x"][j], xk), k


def pin_cg_statuses(lib):
    """Early exits: b = 0, non-finite b, maxit exhaustion, breakdown on an
    indefinite matrix, x0 already the solution, and the empty system."""
    ptr, col, val = W.random_spd_sparse(50, density=0.1, seed=3)
    n = 50
    x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, np.zeros(n), x0=np.ones(n), lib=lib)
    assert info["status"] == oracle.OK and info["iters"] == 0 and np.all(x == 0)
    bad = W.uniform_vector(n, seed=1)
    bad[7] = np.nan
    x0 = W.uniform_vector(n, seed=2)
    x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, bad, x0=x0, lib=lib)
    assert info["status"] == oracle.ERR_NONFINITE and np.array_equal(x, x0)
    b = W.uniform_vector(n, seed=4)
    x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, b, tol=1e-14, maxit=3, lib=lib)
    assert info["status"] == oracle.NOT_CONVERGED and info["iters"] == 3
    # indefinite: diag(1, -1, 1, ...) -> p'Ap <= 0 at some step
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    ip = np.arange(n + 1, dtype=np.int32)
    ic = np.arange(n, dtype=np.int32)
    x, info, _ = oracle.cg(oracle.FMT_CSR, ip, ic, d, np.ones(n), lib=lib)      # p'Ap = 0 at step 1
    assert info["status"] == oracle.ERR_BREAKDOWN and info["iters"] == 0 and np.all(x == 0)
    e1 = np.zeros(n)
    e1[1] = 1.0                                                                   # p'Ap = -1 < 0
    x, info, _ = oracle.cg(oracle.FMT_CSR, ip, ic, d, e1, lib=lib)
    assert info["status"] == oracle.ERR_BREAKDOWN and info["iters"] == 0 and np.all(x == 0)
    # x0 = exact solution of a diagonal system -> zero residual, no iteration
    dv = np.arange(1, n + 1, dtype=np.float64)
    x, info, _ = oracle.cg(oracle.FMT_CSR, ip, ic, dv, dv * 2.0, x0=np.full(n, 2.0), lib=lib)
    assert info["status"] == oracle.OK and info["iters"] == 0
    # a diagonal system: one step of CG is exact when b is an eigenvector
    x, info, _ = oracle.cg(oracle.FMT_CSR, ip, ic, np.full(n, 4.0), np.ones(n), lib=lib)
    assert info["iters"] == 1 and np.allclose(x, 0.25, rtol=0, atol=1e-16)
    x, info, _ = oracle.cg(oracle.FMT_CSR, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0),
                           np.zeros(0), lib=lib)
    assert info["status"] == oracle.OK and x.size == 0


def pin_cg_formats_agree(lib):
    """CG on the same SPD system stored three ways: identical bits (the
    products are bitwise equal, the rest of the iteration is shared)."""
    s = W.fem_p1_system(7, 6, 5, seed=6)
    A = _csr(s.rowptr, s.col, s.val)
    cp, ri, cv = _csc_arrays(A)
    up, uc, uv = _upper_arrays(A)
    r1 = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, lib=lib)
    r2 = oracle.cg(oracle.FMT_CSC, cp, ri, cv, s.b, lib=lib)
    r3 = oracle.cg(oracle.FMT_SYM_CSR, up, uc, uv, s.b, lib=lib)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[0], r3[0])
    assert r1[1]["iters"] == r2[1]["iters"] == r3[1]["iters"]
    assert r1[1]["status"] == oracle.OK


ALL_PINS = [pin_dot_exact, pin_spmv_exact, pin_spmv_library, pin_three_formats_bitwise, pin_conversions, pin_validate,
            pin_cg_cholesky, pin_cg_exact_termination, pin_cg_lanczos_spectrum, pin_cg_invariants,
            pin_cg_alternative_evaluations, pin_cg_statuses, pin_cg_formats_agree]


def run_all(lib_path):
    """Run every pin against the oracle library at lib_path; returns the
    names of the pins that failed (used on planted-mistake builds)."""
    lib = oracle.load(lib_path)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except Exception as e:             # noqa: BLE001 - any failure counts
            failed.append(f"{pin.__name__}: {type(e).__name__}")
    return failed


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(run_all(sys.argv[1])))

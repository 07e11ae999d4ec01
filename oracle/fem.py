"""CPU oracle for the differentiable solve -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy, written from the definitions; shares nothing with the GPU
library (which it never imports) and is loaded only by the tests, the smoke
check and the benchmark's CPU leg.

The finite-element operator the paper's systems come from (abstract and
section I: finite-element discretisations of Maxwell's equations; section
III: the resulting SPD matrix A) is, for linear tetrahedra,

    A(nu) = sum_e nu_e K_e,    K_e[a, b] = |T_e| grad(phi_a) . grad(phi_b),

restricted to the unknowns (Dirichlet vertices dropped).  For the solve
x = A^-1 b and a loss L(x):

    lambda = A^-1 dL/dx                       (A symmetric: the adjoint solve)
    dL/db       = lambda
    dL/dA_ij    = -lambda_i x_j               (on the stored pattern)
    dL/dnu_e    = -lambda_e' K_e x_e

Functions:
* ``element_matrices``: K_e of every element.  The barycentric functions are
  found from their defining property phi_a(P_b) = delta_ab: with the 4x4
  matrix M whose rows are [1, P_b - P_0] (coordinates measured from the
  first vertex), the coefficients of phi_a are column a of M^-1, so its
  gradient is rows 1..3 of that column; |T_e| = |det M| / 6.
* ``assemble``: A(nu) on a given CSR pattern (sum of element contributions).
* ``nu_grad``, ``pattern_grad``: the formulas above, element by element and
  entry by entry.
* ``solve_grad``: forward solve, loss ||x - x_obs||^2, adjoint solve and all
  three gradients, with the oracle CG of ``oracle`` or a dense solve.

Parity status: pinned in ``tests/test_oracle_fem.py`` (textbook element
matrix, patch test, agreement with the generator's independently assembled
matrix, central finite differences with dense solves, the homogeneity
identity sum_e nu_e dL/dnu_e = -lambda' b).
"""
import numpy as np

# pair order of the 10 distinct entries of a symmetric 4x4 element matrix
PAIRS = [(a, b) for a in range(4) for b in range(a, 4)]


def element_matrices(coords, tets):
    """K_e (nelem, 4, 4) without the coefficient, from vertex coordinates."""
    P = np.asarray(coords, dtype=np.float64)[np.asarray(tets)]          # (e, 4, 3)
    # the basis functions of an element do not depend on where the origin is:
    # measuring from the first vertex keeps M as well conditioned as the element
    P = P - P[:, :1, :]
    M = np.concatenate([np.ones(P.shape[:2] + (1,)), P], axis=2)       # rows [1, P_b - P_0]
    C = np.linalg.inv(M)                                               # column a: coefficients of phi_a
    grads = C[:, 1:, :]                                                # (e, 3, 4): column a = grad phi_a
    vol = np.abs(np.linalg.det(M)) / 6.0
    return vol[:, None, None] * np.einsum("eka,ekb->eab", grads, grads)


def cauchy_schwarz_scale(K):
    """|T_e| |grad phi_a| |grad phi_b| = sqrt(K_aa K_bb): the size against
    which the rounding error of K_e[a, b] is measured (an off-diagonal entry
    can be much smaller than this by cancellation)."""
    d = np.sqrt(np.maximum(np.einsum("eaa->ea", K), 0.0))
    return d[:, :, None] * d[:, None, :]


def _pattern_positions(rowptr, col, rows, cols):
    """Index into the CSR arrays of each (row, col) pair; all must be stored."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = rowptr.size - 1
    key = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr)) * (n + 1) + col
    want = rows.astype(np.int64) * (n + 1) + cols.astype(np.int64)
    pos = np.searchsorted(key, want)
    if np.any(pos >= key.size) or np.any(key[np.minimum(pos, key.size - 1)] != want):
        raise ValueError("element pair outside the CSR pattern")
    return pos


def assemble(nu, K, tets, dof, rowptr, col):
    """Values of A(nu) = sum_e nu_e K_e on a column-sorted full CSR pattern."""
    nu = np.asarray(nu, dtype=np.float64)
    d = np.asarray(dof)[np.asarray(tets)]                              # (e, 4) unknown ids or -1
    vals = np.zeros(np.asarray(col).size)
    for a in range(4):
        for b in range(4):
            m = (d[:, a] >= 0) & (d[:, b] >= 0)
            pos = _pattern_positions(rowptr, col, d[m, a], d[m, b])
            np.add.at(vals, pos, nu[m] * K[m, a, b])
    return vals


def _gather(v, d):
    out = np.zeros(d.shape)
    m = d >= 0
    out[m] = v[d[m]]
    return out


def nu_grad(K, tets, dof, lam, x):
    """dL/dnu_e = -lambda_e' K_e x_e (Dirichlet components are zero)."""
    d = np.asarray(dof)[np.asarray(tets)]
    le, xe = _gather(np.asarray(lam, dtype=np.float64), d), _gather(np.asarray(x, dtype=np.float64), d)
    return -np.einsum("ea,eab,eb->e", le, K, xe)


def pattern_grad(fmt, ptr, idx, lam, x):
    """dL/d(stored value) for every stored entry, in storage order.

    fmt 0 (CSR, line = row i, index = column j): -lambda_i x_j.
    fmt 2 (CSC, line = column j, index = row i): -lambda_i x_j.
    fmt 1 (symmetric CSR, upper triangle: the stored u_ij is both A_ij and
    A_ji): -(lambda_i x_j + lambda_j x_i) off the diagonal, -lambda_i x_i on it.
    """
    ptr = np.asarray(ptr, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    lam = np.asarray(lam, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    line = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    if fmt == 0:
        return -lam[line] * x[idx]
    if fmt == 2:
        return -lam[idx] * x[line]
    g = -(lam[line] * x[idx] + lam[idx] * x[line])
    diag = line == idx
    g[diag] = -lam[line[diag]] * x[idx[diag]]
    return g


def dense(rowptr, col, vals, n):
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(np.asarray(rowptr)))
    np.add.at(A, (rows, np.asarray(col)), vals)
    return A


def solve_grad(nu, b, x_obs, K, tets, dof, rowptr, col, *, tol=1e-13, dense_solve=False, maxit=None):
    """Forward x = A(nu)^-1 b, L = ||x - x_obs||^2 and the adjoint gradients.

    Returns dict(x, L, lam, g_b, g_nu, g_vals, vals, info)."""
    import oracle
    n = np.asarray(rowptr).size - 1
    vals = assemble(nu, K, tets, dof, rowptr, col)
    if dense_solve:
        A = dense(rowptr, col, vals, n)
        x = np.linalg.solve(A, b)
        r = x - x_obs
        lam = np.linalg.solve(A.T, 2.0 * r)
        info = None
    else:
        x, i1, _ = oracle.cg(oracle.FMT_CSR, rowptr, col, vals, b, tol=tol, maxit=maxit or 20 * n)
        r = x - x_obs
        lam, i2, _ = oracle.cg(oracle.FMT_CSR, rowptr, col, vals, 2.0 * r, tol=tol, maxit=maxit or 20 * n)
        info = (i1, i2)
    return dict(x=x, L=float(r @ r), lam=lam, g_b=lam, g_nu=nu_grad(K, tets, dof, lam, x),
                g_vals=pattern_grad(0, rowptr, col, lam, x), vals=vals, info=info)

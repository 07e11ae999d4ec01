"""Exact rational SpMV and CG for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Python ``fractions.Fraction`` throughout, so there is no rounding at all:

* ``spmv_csr_exact`` is the definition y_i = sum_j a_ij x_j (section III, the
  "trivial" row product), used to bound the floating-point products;
* ``cg_exact`` is the CG recurrence of section III (alpha = r'r / p'Ap,
  x += alpha p, r -= alpha Ap, beta = r_k'r_k / r_{k-1}'r_{k-1},
  p = r + beta p) run until r == 0 exactly.  In exact arithmetic CG ends in
  at most as many steps as A has distinct eigenvalues (for the b used),
  which pins the step count and the solution.
"""
from fractions import Fraction


def to_frac(v):
    return [Fraction(float(t)) for t in v]


def spmv_csr_exact(ptr, col, val, x):
    n = len(ptr) - 1
    vf, xf = to_frac(val), [t if isinstance(t, Fraction) else Fraction(float(t)) for t in x]
    y = []
    for i in range(n):
        s = Fraction(0)
        for k in range(int(ptr[i]), int(ptr[i + 1])):
            s += vf[k] * xf[int(col[k])]
        y.append(s)
    return y


def _dot(a, b):
    s = Fraction(0)
    for u, v in zip(a, b):
        s += u * v
    return s


def cg_exact(ptr, col, val, b, maxit=None):
    """Exact CG from x0 = 0.  Returns (x, steps) where steps is the number of
    products A p needed until the residual is exactly zero."""
    n = len(ptr) - 1
    vf = to_frac(val)
    bf = [t if isinstance(t, Fraction) else Fraction(float(t)) for t in b]

    def matvec(v):
        out = []
        for i in range(n):
            s = Fraction(0)
            for k in range(int(ptr[i]), int(ptr[i + 1])):
                s += vf[k] * v[int(col[k])]
            out.append(s)
        return out

    x = [Fraction(0)] * n
    r = list(bf)
    p = list(r)
    rho = _dot(r, r)
    if rho == 0:
        return x, 0
    maxit = n if maxit is None else maxit
    for k in range(1, maxit + 1):
        q = matvec(p)
        alpha = rho / _dot(p, q)
        x = [xi + alpha * pi for xi, pi in zip(x, p)]
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        rho_new = _dot(r, r)
        if rho_new == 0:
            return x, k
        beta = rho_new / rho
        p = [ri + beta * pi for ri, pi in zip(r, p)]
        rho = rho_new
    raise RuntimeError("exact CG did not terminate within maxit")

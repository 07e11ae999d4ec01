"""Pins of the finite-element / adjoint oracle (``oracle/fem.py``).

Each pin takes the oracle module as an argument, so the same checks can run
against copies of it with a planted mistake (``test_oracle_fem.py``).

Sources of truth: the hand-derived element matrix of the reference
tetrahedron (``tests/golden/p1_reference_tet.txt``); the patch test (a linear
field u has energy sum_e u_e' K_e u_e = |Omega| |grad u|^2 exactly, and
constants are in the kernel of every K_e); the generator's matrix, assembled by
an independent route (3x3 Jacobian inverse, upper keys, bincount); central
finite differences of the loss with LAPACK dense solves; and the identity
sum_e nu_e dL/dnu_e = -lambda' A x = -lambda' b (A is linear in nu).
"""
from __future__ import annotations

import os

import numpy as np

from paper_1010_4639_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p1_reference_tet.txt")


def _small(nx=4, ny=3, nz=3, seed=7, nu_iron=1e-2):
    s = W.fem_p1_system(nx, ny, nz, nu_iron=nu_iron, seed=seed)
    coords, tets, dof, nu = W.fem_mesh(s)
    return s, coords, tets, dof, nu


def pin_reference_tet(F):
    K6 = np.loadtxt(GOLDEN)
    P = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    K = F.element_matrices(P, np.array([[0, 1, 2, 3]]))[0]
    assert np.allclose(6.0 * K, K6, rtol=0, atol=1e-14), K * 6
    # translation + rotation leave K unchanged; scaling by s multiplies it by s
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    P2 = 2.5 * P @ Q.T + np.array([3.0, -1.0, 7.0])
    K2 = F.element_matrices(P2, np.array([[0, 1, 2, 3]]))[0]
    assert np.allclose(K2, 2.5 * K, rtol=0, atol=1e-13)
    # vertex order reversed (negative orientation): same matrix, permuted
    K3 = F.element_matrices(P, np.array([[3, 2, 1, 0]]))[0]
    assert np.allclose(K3, K[::-1, ::-1], rtol=0, atol=1e-14)


def pin_patch_test(F):
    s, coords, tets, dof, nu = _small(5, 4, 3, seed=11)
    K = F.element_matrices(coords, tets)
    scale = np.abs(K).max()
    assert np.abs(K.sum(axis=2)).max() <= 1e-13 * scale          # constants in the kernel
    c = np.array([0.3, -1.1, 0.7])
    u = coords @ c + 2.0
    ue = u[tets]
    energy = np.einsum("ea,eab,eb->", ue, K, ue)
    vol = (s.nx + 1) * (s.ny + 1) * (s.nz + 1)                  # the jittered mesh still tiles the box
    assert abs(energy - vol * (c @ c)) <= 1e-12 * vol * (c @ c), (energy, vol * (c @ c))


def pin_matches_generator(F):
    for (nx, ny, nz, seed) in [(4, 3, 3, 7), (6, 5, 4, 8)]:
        s, coords, tets, dof, nu = _small(nx, ny, nz, seed=seed)
        K = F.element_matrices(coords, tets)
        v = F.assemble(nu, K, tets, dof, s.rowptr, s.col)
        scale = np.abs(s.val).max()
        assert np.abs(v - s.val).max() <= 1e-13 * scale, np.abs(v - s.val).max() / scale


def _setup_grad(seed=7):
    s, coords, tets, dof, _ = _small(4, 3, 3, seed=seed)
    rng = np.random.default_rng(seed + 100)
    nu = rng.uniform(0.5, 1.5, size=tets.shape[0])
    return s, coords, tets, dof, nu, rng


def pin_fd_nu(F):
    s, coords, tets, dof, nu, rng = _setup_grad()
    K = F.element_matrices(coords, tets)
    xo = W.observation(s)
    base = F.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)
    # elements touching at least one unknown, drawn at random
    touch = np.nonzero((dof[tets] >= 0).any(axis=1))[0]
    for e in rng.choice(touch, size=12, replace=False):
        h = 1e-5 * nu[e]
        Lp = F.solve_grad(np.where(np.arange(nu.size) == e, nu + h, nu), s.b, xo, K, tets, dof, s.rowptr, s.col,
                          dense_solve=True)["L"]
        Lm = F.solve_grad(np.where(np.arange(nu.size) == e, nu - h, nu), s.b, xo, K, tets, dof, s.rowptr, s.col,
                          dense_solve=True)["L"]
        fd = (Lp - Lm) / (2 * h)
        g = base["g_nu"][e]
        assert abs(fd - g) <= 1e-6 * abs(g) + 1e-8 * base["L"] / nu[e], (e, fd, g)


def pin_fd_b(F):
    s, coords, tets, dof, nu, rng = _setup_grad(9)
    K = F.element_matrices(coords, tets)
    xo = W.observation(s)
    base = F.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)
    for i in rng.choice(s.n, size=8, replace=False):
        h = 1e-4
        bp, bm = s.b.copy(), s.b.copy()
        bp[i] += h
        bm[i] -= h
        Lp = F.solve_grad(nu, bp, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)["L"]
        Lm = F.solve_grad(nu, bm, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)["L"]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - base["g_b"][i]) <= 1e-6 * abs(base["g_b"][i]) + 1e-9 * base["L"], (i, fd, base["g_b"][i])


def pin_fd_pattern(F):
    """dL/d(stored value) against central differences of a dense solve, in all
    three storage formats (symmetric storage perturbs A_ij and A_ji together)."""
    s, coords, tets, dof, nu, rng = _setup_grad(13)
    n = s.n
    K = F.element_matrices(coords, tets)
    vals = F.assemble(nu, K, tets, dof, s.rowptr, s.col)
    A = F.dense(s.rowptr, s.col, vals, n)
    xo = W.observation(s)
    x = np.linalg.solve(A, s.b)
    lam = np.linalg.solve(A.T, 2.0 * (x - xo))

    def loss(M):
        y = np.linalg.solve(M, s.b)
        return float((y - xo) @ (y - xo))

    up, uc, uv = W.upper_triangle(s.rowptr, s.col, vals)
    cp, ci, cv = W.transpose_csr(n, n, s.rowptr, s.col, vals)
    cases = [(0, s.rowptr, s.col, lambda l, j: [(l, j)]),
             (2, cp, ci, lambda l, i: [(i, l)]),
             (1, up, uc, lambda l, j: [(l, j)] if l == j else [(l, j), (j, l)])]
    for fmt, ptr, idx, where in cases:
        g = F.pattern_grad(fmt, ptr, idx, lam, x)
        line = np.repeat(np.arange(n), np.diff(ptr))
        ks = list(rng.choice(idx.size, size=10, replace=False))
        ks += list(np.nonzero(line == idx)[0][:2])               # some diagonal entries
        for k in ks:
            h = 1e-6
            Ap, Am = A.copy(), A.copy()
            for (i, j) in where(int(line[k]), int(idx[k])):
                Ap[i, j] += h
                Am[i, j] -= h
            fd = (loss(Ap) - loss(Am)) / (2 * h)
            assert abs(fd - g[k]) <= 1e-5 * abs(g[k]) + 1e-8 * np.abs(g).max(), (fmt, k, fd, g[k])


def pin_homogeneity(F):
    s, coords, tets, dof, nu, rng = _setup_grad(17)
    K = F.element_matrices(coords, tets)
    xo = W.observation(s)
    r = F.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)
    lhs = float(nu @ r["g_nu"])
    rhs = -float(r["lam"] @ s.b)
    assert abs(lhs - rhs) <= 1e-10 * (abs(nu) @ np.abs(r["g_nu"])), (lhs, rhs)
    # and -lambda' b = -2 (x - x_obs)' x (lambda = A^-1 2 (x - x_obs), A symmetric)
    rhs2 = -2.0 * float((r["x"] - xo) @ r["x"])
    assert abs(rhs - rhs2) <= 1e-9 * abs(rhs2), (rhs, rhs2)


def pin_cg_path_matches_dense(F):
    s, coords, tets, dof, _ = _small(8, 7, 6, seed=21)
    rng = np.random.default_rng(5)
    nu = rng.uniform(0.2, 2.0, size=tets.shape[0])
    K = F.element_matrices(coords, tets)
    xo = W.observation(s)
    d = F.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)
    c = F.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, tol=1e-13)
    for k in ("x", "lam", "g_nu", "g_vals"):
        err = np.linalg.norm(c[k] - d[k]) / np.linalg.norm(d[k])
        assert err <= 1e-9, (k, err)


ALL_PINS = [pin_reference_tet, pin_patch_test, pin_matches_generator, pin_fd_nu, pin_fd_b, pin_fd_pattern,
            pin_homogeneity, pin_cg_path_matches_dense]


def run_all(F):
    """Names of the pins that fail (or raise) for oracle module F."""
    bad = []
    for p in ALL_PINS:
        try:
            p(F)
        except Exception:                       # noqa: BLE001 -- a crash is a failed pin
            bad.append(p.__name__)
    return bad

"""Differentiable CG solves (adjoint method) through the HIP library.

For x = A^-1 b and a scalar loss L(x), with A symmetric positive definite
(the systems of the paper, section III):

    lam = A^-1 dL/dx                  (a second CG solve on the same matrix)
    dL/db = lam,   dL/dA_ij = -lam_i x_j on the stored pattern,
    dL/dnu_e = -lam_e' K_e x_e        when A(nu) = sum_e nu_e K_e.

The backward pass recomputes: it keeps x (and the inputs), not the forward
iterates, and re-sends the matrix values to the handle before the adjoint
solve, so one handle can serve several forward passes before their backward
passes.  Every step runs in the library's kernels (assembly, product, CG,
gradients); torch only holds the tensors and the stream.

    sparse_solve(vals, b, solver)     -> x, differentiable in vals and b
    fem_solve(nu, b, fem, solver)     -> x, differentiable in nu and b
    FemSolve(coords, tets, dof, n)    owns both handles: FemSolve(...)(nu, b)
"""
from __future__ import annotations

import torch

from . import cgmi


def _solve(solver, rhs, tol, maxit):
    x, info = solver.solve(rhs.detach().contiguous(), tol=tol, maxit=maxit, check=False)
    if info["status"] != cgmi.CG_OK:
        raise cgmi.CgError(info["status"], f"CG solve inside the differentiable solve: {info}")
    return x, info


class _SparseSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, solver, tol, maxit):
        v = vals.detach().contiguous()
        solver.set_values(v)
        x, _ = _solve(solver, b, tol, maxit)
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        ctx.save_for_backward(v, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        v, x = ctx.saved_tensors
        solver = ctx.solver
        solver.set_values(v)
        lam, _ = _solve(solver, gx, ctx.tol, ctx.maxit)
        g_vals = solver.pattern_grad(lam, x) if ctx.needs_input_grad[0] else None
        g_b = lam if ctx.needs_input_grad[1] else None
        return g_vals, g_b, None, None, None


class _FemSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nu, b, fem, solver, tol, maxit):
        nu_d = nu.detach().contiguous()
        solver.set_values(fem.assemble(nu_d))
        x, _ = _solve(solver, b, tol, maxit)
        ctx.fem, ctx.solver, ctx.tol, ctx.maxit = fem, solver, tol, maxit
        ctx.save_for_backward(nu_d, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        nu_d, x = ctx.saved_tensors
        fem, solver = ctx.fem, ctx.solver
        solver.set_values(fem.assemble(nu_d))           # recomputed, not stored
        lam, _ = _solve(solver, gx, ctx.tol, ctx.maxit)
        g_nu = fem.nu_grad(lam, x) if ctx.needs_input_grad[0] else None
        g_b = lam if ctx.needs_input_grad[1] else None
        return g_nu, g_b, None, None, None, None


def sparse_solve(vals, b, solver, tol=1e-10, maxit=None):
    """x = A(vals)^-1 b on the structure of `solver` (a cgmi.Solver)."""
    return _SparseSolve.apply(vals, b, solver, float(tol), maxit)


def fem_solve(nu, b, fem, solver, tol=1e-10, maxit=None):
    """x = A(nu)^-1 b with A(nu) assembled by `fem` (a cgmi.FemOperator) and
    solved by `solver` (a cgmi.Solver built on fem's CSR pattern)."""
    return _FemSolve.apply(nu, b, fem, solver, float(tol), maxit)


class FemSolve:
    """The operator and a CSR solver on its pattern, created together.

    FemSolve(coords, tets, dof, n): host mesh arrays.  The solver is planned
    on the operator's pattern (only the structure matters there: every call
    sends the assembled values first).  Calling it with (nu, b) returns x.
    """

    def __init__(self, coords, tets, dof, n, batch=None):
        import numpy as np
        self.fem = cgmi.FemOperator(coords, tets, dof, n)
        rp, col = self.fem.pattern()
        # structure-only placeholder values; fem_solve sends the real ones
        self.solver = cgmi.Solver(cgmi.CG_FMT_CSR, rp, col, np.ones(col.size), batch=batch)
        self.n, self.nelem, self.nnz = self.fem.n, self.fem.nelem, self.fem.nnz

    def __call__(self, nu, b, tol=1e-10, maxit=None):
        return fem_solve(nu, b, self.fem, self.solver, tol=tol, maxit=maxit)

    def close(self):
        self.solver.close()
        self.fem.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

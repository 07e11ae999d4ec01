"""Mixed precision (FP32 product and search directions inside FP64 iterative
refinement) through the C-ABI vs the FP64 oracle.

The refinement stops on the TRUE residual ||b - A x|| <= tol ||b|| computed
with the FP64 product, so the bar is the FP64 one: true residual (oracle
product) <= 2 tol, energy-norm difference to the oracle's FP64 CG solution
<= 1e-8, and a 2-norm error against the exact solution no larger than the
FP64 oracle's own (within 4x); the 2-norm difference to the oracle's
solution is recorded per result.
"""
import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import fem_cached, say, to_dev, true_relres
from tests import parity
from tests.test_gpu_cg import a_norm, formats_of

pytestmark = pytest.mark.gpu

CSR, SYM, CSC = cgmi.CG_FMT_CSR, cgmi.CG_FMT_SYM_CSR, cgmi.CG_FMT_CSC


def run_mixed(fmt, arrs, b, tol=1e-10, inner_tol=1e-4, label=""):
    with cgmi.Solver(fmt, *arrs, mixed=True) as S:
        x, info = S.solve_mixed(to_dev(b), tol=tol, maxit=200000, inner_tol=inner_tol, max_outer=60, check=False)
    say(f"mixed {label} fmt={fmt}: status={info['status']} inner iters={info['iters']} outer={info['outer']} "
        f"relres_true={info['relres_true']:.3e} ms={info['ms']:.1f}")
    return x.cpu().numpy(), info


def check_vs_fp64(fmt, arrs, b, xg, info, x_true, tol=1e-10, label=""):
    """The refinement is another algorithm than the oracle's CG: it stops on
    the true residual, after whole inner solves, usually well below tol, so
    its x does not sit where the oracle's FP64 CG stops (~kappa tol away from
    the solution).  Asserted: the energy-norm difference to the oracle's
    solution (<= 1e-8, the FP64 bar), and the 2-norm error against the exact
    solution x_true no larger than the FP64 oracle's own (within 4x, floor
    1e-8).  The 2-norm difference to the oracle's solution is recorded."""
    assert info["status"] == cgmi.CG_OK, info
    rt = true_relres(fmt, *arrs, b, xg)
    assert rt <= 2 * tol and abs(rt - info["relres_true"]) <= 1e-2 * rt
    xo, oinfo, _ = oracle.cg(fmt, *arrs, b, tol=tol, maxit=200000)
    assert oinfo["status"] == oracle.OK
    d = xg - xo
    err_a = a_norm(fmt, arrs, d) / a_norm(fmt, arrs, xo)
    err = np.linalg.norm(d) / np.linalg.norm(xo)
    nt = np.linalg.norm(x_true)
    e_orc, e_mx = np.linalg.norm(xo - x_true) / nt, np.linalg.norm(xg - x_true) / nt
    say(f"   vs FP64 oracle ({oinfo['iters']} it): 2-norm {err:.3e}  A-norm {err_a:.3e}; error vs x_true: "
        f"mixed {e_mx:.3e}, oracle {e_orc:.3e}")
    parity.record(test="mixed " + label, fmt=int(fmt), n=len(arrs[0]) - 1, err2=err, errA=err_a,
                  err2_vs_true=e_mx, oracle_err2_vs_true=e_orc, inner_iters=info["iters"], outer=info["outer"],
                  relres_true=rt)
    assert err_a <= parity.X_TOL, err_a
    assert e_mx <= max(parity.X_TOL, 4 * e_orc), (e_mx, e_orc)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_mixed_paper_sized(fmt):
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info = run_mixed(fmt, arrs, s.b, label="fem32x32x30")
    check_vs_fp64(fmt, arrs, s.b, xg, info, s.x_true, label="fem32x32x30 inner 1e-4")


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_mixed_row_blocks(monkeypatch, fmt):
    # the FP32 product through the row-block / panel-chunk layout (FEM
    # matrices default to slices)
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "rows")
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info = run_mixed(fmt, arrs, s.b, label="fem32x32x30 row blocks")
    check_vs_fp64(fmt, arrs, s.b, xg, info, s.x_true, label="fem32x32x30 row blocks")


@pytest.mark.parametrize("restart", ["0", "1"])
@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_mixed_loose_inner_tolerance(monkeypatch, fmt, restart):
    # inner tolerance 1e-2: several refinement steps, each continuing with the
    # previous inner solve's direction (restart = 0, the default) or starting
    # over from p = r (restart = 1); both must meet the FP64 bar
    monkeypatch.setenv("CGMI_MIXED_RESTART", restart)
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info = run_mixed(fmt, arrs, s.b, inner_tol=1e-2, label=f"fem32x32x30 inner 1e-2 restart={restart}")
    assert info["outer"] >= 3
    check_vs_fp64(fmt, arrs, s.b, xg, info, s.x_true, label=f"fem32x32x30 inner 1e-2 restart={restart}")


@pytest.mark.parametrize("fmt", [CSR, SYM])
def test_mixed_high_contrast(fmt):
    # iron contrast 1e-4: kappa * u_fp32 would exceed 1 without the diagonal scaling
    s = W.fem_p1_system(20, 20, 18, nu_iron=1e-4, seed=3)
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info = run_mixed(fmt, arrs, s.b, label="fem20x20x18 nu=1e-4")
    check_vs_fp64(fmt, arrs, s.b, xg, info, s.x_true, label="fem20x20x18 nu=1e-4")


def test_mixed_statuses():
    import torch
    ptr, col, val = W.random_spd_sparse(80, density=0.1, seed=4)
    n = 80
    with cgmi.Solver(CSR, ptr, col, val) as S:          # no FP32 copy
        st, _ = cgmi.cg_solve_mixed(S.h, to_dev(np.ones(n)).data_ptr(), to_dev(np.zeros(n)).data_ptr(),
                                    1e-10, 100, 1e-4, 10)
        assert st == cgmi.CG_ERR_ARG
    with cgmi.Solver(CSR, ptr, col, val, mixed=True) as S:
        x, info = S.solve_mixed(to_dev(np.zeros(n)), to_dev(np.ones(n)))
        assert info["status"] == cgmi.CG_OK and torch.all(x == 0)
        bad = W.uniform_vector(n, seed=5)
        bad[3] = np.inf
        x0 = to_dev(W.uniform_vector(n, seed=6))
        x, info = S.solve_mixed(to_dev(bad), x0, check=False)
        assert info["status"] == cgmi.CG_ERR_NONFINITE and torch.equal(x, x0)
        b = W.uniform_vector(n, seed=7)
        x, info = S.solve_mixed(to_dev(b), tol=1e-14, maxit=2, check=False)
        assert info["status"] == cgmi.CG_NOT_CONVERGED and info["iters"] <= 2
        for bad_args in ((1e-10, 10, 0.0, 5), (1e-10, 10, 1.0, 5), (1e-10, 10, 1e-3, 0), (-1.0, 10, 1e-3, 5)):
            st, _ = cgmi.cg_solve_mixed(S.h, to_dev(b).data_ptr(), x.data_ptr(), *bad_args)
            assert st == cgmi.CG_ERR_ARG
        x, info = S.solve_mixed(to_dev(b), tol=1e-12)
        assert info["status"] == cgmi.CG_OK and info["outer"] >= 2
    # CG_MIXED needs a positive diagonal
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    st, h = cgmi.cg_create(CSR, n, np.arange(n + 1), np.arange(n), d, 0, cgmi.CG_MIXED)
    assert st == cgmi.CG_ERR_ARG and h is None and "diagonal" in cgmi.cg_last_error(None)

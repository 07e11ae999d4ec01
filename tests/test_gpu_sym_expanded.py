"""Symmetric CSR on small systems, planned as expanded full rows (the
library's default where the vector kernels have at most 256 workgroups,
n <= 65 536): each off-diagonal stored entry serves positions (i, j) and
(j, i), and the rows are sliced like CSR.  Checked against the oracle's
symmetric product and CG like the other plans; the CG runs the two-kernel
iteration there and must give the bits of the three-kernel one.
"""
import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import check_spmv, fem_cached, say, to_dev
from tests.test_gpu_cg import check_contract, run_pair

pytestmark = [pytest.mark.gpu, pytest.mark.sym_expanded]

SYM = cgmi.CG_FMT_SYM_CSR


def expanded(n, *arrs, **kw):
    st, stats = cgmi.cg_analyze(SYM, n, *arrs, **kw)
    assert st == 0 and stats["compact"] == 0 and stats["slices"] >= 1 and stats["parked"] == 0, stats
    return stats


@pytest.mark.parametrize("case", ["fem", "random_spd", "diagonal", "one_row"])
def test_expanded_products(case, monkeypatch):
    # (random rows pad their slices beyond the default limit: slices forced)
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "slices")
    if case == "fem":
        s = W.fem_p1_system(20, 18, 16, seed=31)
        up = W.upper_triangle(s.rowptr, s.col, s.val)
    elif case == "random_spd":
        ptr, col, val = W.random_spd_sparse(700, density=0.02, seed=32)
        up = W.upper_triangle(ptr, col, val)
    elif case == "diagonal":
        n = 129
        up = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), W.uniform_vector(n, seed=33) + 2.0)
    else:
        up = (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0]))
    n = len(up[0]) - 1
    expanded(n, *up)
    check_spmv(SYM, *up, W.uniform_vector(n, seed=34), label=f"expanded {case}")


def test_expanded_lower_and_one_based_input(monkeypatch):
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "slices")  # (a 504-row grid pads its slices beyond the default limit)
    s = W.fem_p1_system(9, 8, 7, seed=35)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    x = W.uniform_vector(s.n, seed=36)
    expanded(s.n, *up)
    y0, _ = check_spmv(SYM, *up, x, label="expanded upper")
    # the same matrix given as its lower triangle, 1-based
    import scipy.sparse as sp
    L = sp.tril(sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)), format="csr")
    L.sort_indices()
    with cgmi.Solver(SYM, L.indptr.astype(np.int32) + 1, L.indices.astype(np.int32) + 1, L.data, index_base=1,
                     flags=cgmi.CG_LOWER) as S:
        assert S.stats()["compact"] == 0 and S.stats()["slices"] >= 1
        y1 = S.spmv(to_dev(x)).cpu().numpy()
    assert np.array_equal(y0, y1)


def test_expanded_cg_paper_sized():
    s = fem_cached("fem32x32x30")
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    expanded(s.n, *up)
    xg, info, xo, oinfo = run_pair(SYM, up, s.b, label="fem32x32x30 expanded")
    check_contract(SYM, up, s.b, xg, info, xo, oinfo, strict_2norm=False, label="fem32x32x30 symcsr expanded")


def test_expanded_two_kernel_iteration_same_bits(monkeypatch):
    s = W.fem_p1_system(14, 13, 12, nu_iron=1e-3, seed=37)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    expanded(s.n, *up)
    out = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("CGMI_FUSED", fused)
        with cgmi.Solver(SYM, *up) as S:
            x, info = S.solve(to_dev(s.b), tol=1e-10, maxit=5000)
            out[fused] = (x.cpu().numpy(), info["iters"], info["relres"])
    assert np.array_equal(out["1"][0], out["0"][0]) and out["1"][1:] == out["0"][1:]


def test_expanded_set_values_and_mixed():
    s = W.fem_p1_system(12, 11, 10, nu_iron=1e-3, seed=38)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    expanded(s.n, *up)
    x = W.uniform_vector(s.n, seed=39)
    # new values, still SPD: the diagonal raised by up to 50 % (the upper
    # triangle stores each row's diagonal entry first)
    v2 = up[2].copy()
    v2[up[0][:-1]] *= 1.25 + 0.25 * W.uniform_vector(s.n, seed=40)
    assert np.all(up[1][up[0][:-1]] == np.arange(s.n))
    with cgmi.Solver(SYM, *up, mixed=True) as S:
        S.set_values(to_dev(v2))
        y = S.spmv(to_dev(x)).cpu().numpy()
        # b = A(v2) s.b: the exact solution is s.b
        xm, info = S.solve_mixed(to_dev(oracle.spmv(SYM, up[0], up[1], v2, s.b)), tol=1e-10, maxit=100000)
    with cgmi.Solver(SYM, up[0], up[1], v2) as S2:
        assert np.array_equal(y, S2.spmv(to_dev(x)).cpu().numpy())
    assert info["status"] == cgmi.CG_OK
    err = np.linalg.norm(xm.cpu().numpy() - s.b) / np.linalg.norm(s.b)
    say(f"expanded mixed: {info}, error vs the exact solution {err:.2e}")
    assert err <= 1e-6

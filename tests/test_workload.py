"""Pins of the synthetic FEM input generator (no GPU).

The generator is not the method; it only has to produce what it claims: the
P1 stiffness matrix of a Kuhn-split, jittered box with an iron region.  The
checks are closed forms (nonzero counts, the 7-point Laplacian special case),
exact symmetry, the stiffness row-sum property, an independent element-energy
route for x'Ax, positive definiteness, and the orientation guard.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1010_4639_amd import workload as W


def closed_form_nnz(nx, ny, nz):
    """n + 2 * (pairs along the 7 positive directions {0,1}^3 \\ 0)."""
    n = nx * ny * nz
    pairs = 0
    for d in range(1, 8):
        dx, dy, dz = d & 1, (d >> 1) & 1, (d >> 2) & 1
        pairs += (nx - dx) * (ny - dy) * (nz - dz)
    return n + 2 * pairs, n + pairs


def _A(s):
    return sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))


@pytest.fixture(scope="module")
def c1():
    return W.fem_config("fem32x32x30")


def test_closed_form_counts_paper_sized(c1):
    nnz, nnz_u = closed_form_nnz(32, 32, 30)
    assert c1.n == 30720 and c1.nnz == nnz == 437622
    up = W.upper_triangle(c1.rowptr, c1.col, c1.val)
    assert up[0][-1] == nnz_u == 234171


@pytest.mark.parametrize("dims,expect", [((100, 100, 100), (14761198, 7880599)),
                                         ((160, 160, 160), (60827518, 32461759))])
def test_closed_form_counts_large(dims, expect):
    assert closed_form_nnz(*dims) == expect


def test_pattern_builder_matches_closed_form_1m():
    # pattern-only assembly (all values zero) of the 100^3 grid
    rp, col, _ = W._upper_keys_to_csr(np.zeros(100 ** 3 * 8), 100, 100, 100)
    assert int(rp[-1]) == closed_form_nnz(100, 100, 100)[0]
    rows = np.repeat(np.arange(100 ** 3), np.diff(rp))
    same = np.diff(rows) == 0
    assert np.all(np.diff(col)[same] > 0)


def test_paper_sized_shape_and_iron(c1):
    rows_len = np.diff(c1.rowptr)
    assert rows_len.max() == 15 and rows_len.min() == 5     # corners like (nx, 1, 1)
    assert abs(c1.iron_fraction - 0.392) < 5e-3          # box of round(0.4^(1/3) C_d) cells
    assert c1.min_orient_det > 0


def test_exact_symmetry_and_sorted(c1):
    A = _A(c1)
    assert (A != A.T).nnz == 0
    rows = np.repeat(np.arange(c1.n), np.diff(c1.rowptr))
    assert np.all(np.diff(c1.col)[np.diff(rows) == 0] > 0)
    assert c1.rowptr.dtype == np.int32 and c1.col.dtype == np.int32


def test_undistorted_unit_coefficient_is_7pt_laplacian():
    s = W.fem_p1_system(6, 5, 4, jitter=0.0, iron_frac=0.0, seed=3)
    A = _A(s).toarray()
    n = s.n
    off = W.direction_offsets(6, 5)
    ref = np.zeros((n, n))
    ids = np.arange(n).reshape(4, 5, 6)
    for k in range(4):
        for j in range(5):
            for i in range(6):
                a = ids[k, j, i]
                ref[a, a] = 6.0
                for (di, dj, dk) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if ii < 6 and jj < 5 and kk < 4:
                        ref[a, ids[kk, jj, ii]] = ref[ids[kk, jj, ii], a] = -1.0
    assert np.max(np.abs(A - ref)) <= 1e-14
    # the diagonal-neighbour couplings are structurally present although zero
    assert _A(s).nnz == closed_form_nnz(6, 5, 4)[0]
    assert off[7] == 1 + 6 + 30


def test_row_sums_vanish_away_from_boundary(c1):
    A = _A(c1)
    rs = np.asarray(A.sum(axis=1)).ravel()
    absrs = np.asarray(abs(A).sum(axis=1)).ravel()
    k, j, i = np.meshgrid(np.arange(30), np.arange(32), np.arange(32), indexing="ij")
    inner = ((i > 0) & (i < 31) & (j > 0) & (j < 31) & (k > 0) & (k < 29)).ravel()
    assert np.all(np.abs(rs[inner]) <= 32 * 2.0 ** -53 * absrs[inner])
    # Dirichlet rows lose couplings; A SPD still gives 1'A1 > 0
    assert rs.sum() > 0 and np.any(np.abs(rs[~inner]) > 1e-3)


def _element_energy(s, xfull):
    """sum_e nu_e |T_e| |grad u_e|^2 with the barycentric gradients taken from
    the inverse of the 4x4 matrix [1 x y z] of each tetrahedron."""
    P = s.coords
    nz1, ny1, nx1 = s.nu_cell.shape
    total = 0.0
    for perm in W.PERMS:
        offs = [np.zeros(3, int)]
        for ax in perm:
            o = offs[-1].copy()
            o[ax] += 1
            offs.append(o)
        cz, cy, cx = np.meshgrid(np.arange(nz1), np.arange(ny1), np.arange(nx1), indexing="ij")
        cz, cy, cx = cz.ravel(), cy.ravel(), cx.ravel()
        M = np.ones((cz.size, 4, 4))
        u = np.empty((cz.size, 4))
        for a, o in enumerate(offs):
            M[:, a, 1:] = P[cz + o[2], cy + o[1], cx + o[0]]
            u[:, a] = xfull[cz + o[2], cy + o[1], cx + o[0]]
        C = np.linalg.inv(M)                 # columns: coefficients of phi_a
        grad = np.einsum("eka,ea->ek", C[:, 1:, :], u)
        vol = np.abs(np.linalg.det(M)) / 6.0
        nu = s.nu_cell[cz, cy, cx]
        total += np.sum(nu * vol * np.einsum("ek,ek->e", grad, grad))
    return total


def test_energy_identity_independent_route():
    s = W.fem_p1_system(6, 5, 4, nu_iron=1e-2, seed=13)
    x = W.uniform_vector(s.n, seed=14)
    xfull = np.zeros((6, 7, 8))
    xfull[1:-1, 1:-1, 1:-1] = x.reshape(4, 5, 6)
    e_ref = _element_energy(s, xfull)
    e_orc = x @ oracle.spmv(oracle.FMT_CSR, s.rowptr, s.col, s.val, x)
    assert abs(e_orc - e_ref) <= 1e-12 * abs(e_ref)
    # the right-hand side is A x_true (formed element by element)
    assert np.max(np.abs(_A(s) @ s.x_true - s.b)) <= 1e-13 * np.max(np.abs(s.b))


def test_positive_definite_small():
    s = W.fem_p1_system(8, 8, 8, seed=15)
    A = _A(s).toarray()
    assert np.all(np.diag(A) > 0)
    np.linalg.cholesky(A)             # raises if not SPD


def test_orientation_guard():
    with pytest.raises(ValueError):
        W.fem_p1_system(8, 8, 8, jitter=0.49, seed=1, with_rhs=False)


def test_seeded_reproducible():
    a = W.fem_p1_system(5, 4, 3, seed=21)
    b = W.fem_p1_system(5, 4, 3, seed=21)
    c = W.fem_p1_system(5, 4, 3, seed=22)
    assert np.array_equal(a.val, b.val) and np.array_equal(a.b, b.b)
    assert not np.array_equal(a.val, c.val)


def test_format_helpers_match_scipy():
    ptr, col, val = W.random_sparse(50, density=0.1, seed=2, empty_rows=4)
    A = sp.csr_matrix((val, col, ptr), shape=(50, 50))
    cp, ri, cv = W.transpose_csr(50, 50, ptr, col, val)
    C = A.tocsc()
    C.sort_indices()
    assert np.array_equal(cp, C.indptr) and np.array_equal(ri, C.indices) and np.array_equal(cv, C.data)
    up, uc, uv = W.upper_triangle(ptr, col, val)
    T = sp.triu(A, format="csr")
    T.sort_indices()
    assert np.array_equal(up, T.indptr) and np.array_equal(uc, T.indices) and np.array_equal(uv, T.data)

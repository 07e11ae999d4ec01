"""Matrix Market reading (the paper-format input path) on the host.

Pinned against scipy.io's reader on the same files, and by round trips of
the generator's matrices through every storage the library accepts."""
import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp

from paper_1010_4639_amd import cgmi, mmio
from paper_1010_4639_amd import workload as W


def _fem(tmp_path, symmetric):
    s = W.fem_p1_system(5, 4, 4, seed=12)
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    T = sp.tril(A).tocoo() if symmetric else A.tocoo()
    path = tmp_path / ("sym.mtx" if symmetric else "gen.mtx")
    mmio.write_matrix(path, s.n, T.row, T.col, T.data, symmetric=symmetric, comment="test")
    return s, A, path


@pytest.mark.parametrize("symmetric", [False, True])
def test_read_matches_scipy_and_generator(tmp_path, symmetric):
    s, A, path = _fem(tmp_path, symmetric)
    M = mmio.read_matrix(path)
    B = scipy.io.mmread(str(path)).tocsr()
    assert M.n == s.n and M.symmetric == symmetric
    p, c, v = M.csr()
    assert np.array_equal(p, s.rowptr) and np.array_equal(c, s.col) and np.array_equal(v, s.val)
    assert abs(sp.csr_matrix((v, c, p), shape=A.shape) - B).max() == 0
    # upper triangle by rows = the generator's upper triangle
    up, uc, uv = M.upper()
    eu = W.upper_triangle(s.rowptr, s.col, s.val)
    assert all(np.array_equal(a, b) for a, b in zip((up, uc, uv), eu))
    # the paper's storage: lower triangle by rows, 1-based
    lp, lc, lv = M.lower_one_based()
    L = sp.tril(A).tocsr()
    L.sort_indices()
    assert np.array_equal(lp - 1, L.indptr) and np.array_equal(lc - 1, L.indices) and np.array_equal(lv, L.data)
    # by columns: for a symmetric matrix the same arrays as by rows
    cp, ci, cv = M.csc()
    assert np.array_equal(cp, s.rowptr) and np.array_equal(ci, s.col) and np.array_equal(cv, s.val)


def test_csc_of_nonsymmetric(tmp_path):
    ptr, col, val = W.random_sparse(40, density=0.1, seed=3)
    A = sp.csr_matrix((val, col, ptr), shape=(40, 40)).tocoo()
    path = tmp_path / "ns.mtx"
    mmio.write_matrix(path, 40, A.row, A.col, A.data)
    cp, ci, cv = mmio.read_matrix(path).csc()
    C = A.tocsc()
    C.sort_indices()
    assert np.array_equal(cp, C.indptr) and np.array_equal(ci, C.indices) and np.array_equal(cv, C.data)


def test_library_accepts_every_storage(tmp_path):
    s, A, path = _fem(tmp_path, True)
    M = mmio.read_matrix(path)
    for fmt, arrs, base, flags in [("csr", M.csr(), 0, 0), ("csc", M.csc(), 0, 0), ("symcsr", M.upper(), 0, 0),
                                   ("symcsr", M.lower_one_based(), 1, cgmi.CG_LOWER)]:
        st, stats = cgmi.cg_analyze(cgmi.FORMATS[fmt], M.n, *arrs, index_base=base, flags=flags)
        assert st == cgmi.CG_OK, (fmt, cgmi.cg_last_error(None))


def test_vectors_round_trip(tmp_path):
    v = W.uniform_vector(17, seed=4)
    mmio.write_vector(tmp_path / "v.mtx", v)
    assert np.array_equal(mmio.read_vector(tmp_path / "v.mtx"), v)
    V = np.stack([v, 2 * v, -v], axis=1)
    mmio.write_vector(tmp_path / "V.mtx", V)
    assert np.array_equal(mmio.read_vector(tmp_path / "V.mtx"), V)
    assert np.array_equal(scipy.io.mmread(str(tmp_path / "V.mtx")), V)


@pytest.mark.parametrize("text,msg", [
    ("%%NotMatrixMarket matrix coordinate real general\n1 1 1\n1 1 1.0\n", "not a Matrix Market"),
    ("%%MatrixMarket matrix coordinate complex general\n1 1 1\n1 1 1.0 0.0\n", "field"),
    ("%%MatrixMarket matrix coordinate real general\n2 3 1\n1 1 1.0\n", "square"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 2\n1 1 1.0\n", "expected 2 entries"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 1\n3 1 1.0\n", "outside"),
    ("%%MatrixMarket matrix coordinate real symmetric\n2 2 2\n1 2 1.0\n2 1 1.0\n", "one triangle"),
    ("%%MatrixMarket matrix coordinate real general\n2 2 2\n1 1 1.0\n1 1 2.0\n", "twice"),
])
def test_malformed_files(tmp_path, text, msg):
    p = tmp_path / "bad.mtx"
    p.write_text(text)
    with pytest.raises(mmio.MatrixFileError, match=msg):
        mmio.read_matrix(p).csr()

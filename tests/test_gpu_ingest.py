"""Paper-format input end to end: a symmetric Matrix Market file (one
triangle, 1-based) with b, solved in each storage the library accepts,
against the oracle's solution of the same arrays."""
import json

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1010_4639_amd import mmio, solve_file
from paper_1010_4639_amd import workload as W
from tests.gpu_util import say, true_relres

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["paper", "symcsr", "csr", "csc"])
def test_solve_file(tmp_path, capsys, storage):
    s = W.fem_p1_system(12, 11, 10, seed=31)
    L = sp.tril(sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))).tocoo()
    mmio.write_matrix(tmp_path / "A.mtx", s.n, L.row, L.col, L.data, symmetric=True)
    mmio.write_vector(tmp_path / "b.mtx", s.b)
    rc = solve_file.main([str(tmp_path / "A.mtx"), "--rhs", str(tmp_path / "b.mtx"), "--storage", storage,
                          "--out", str(tmp_path / "x.mtx")])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    say(f"{storage}: {out}")
    assert rc == 0 and out["status"] == 0
    x = mmio.read_vector(tmp_path / "x.mtx")
    assert true_relres(0, s.rowptr, s.col, s.val, s.b, x) <= 2e-10
    xo, oi, _ = oracle.cg(0, s.rowptr, s.col, s.val, s.b, tol=1e-10)
    assert abs(out["iters"] - oi["iters"]) <= max(2, 0.03 * oi["iters"])

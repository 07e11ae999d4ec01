"""The oracle's OpenMP timing mode runs the same CSR iteration as the serial
oracle: same iteration count and solution to rounding level (its scalar
products are exactly rounded per thread chunk and combined exactly, so they
agree with the serial exact products to the last bit almost always)."""
import os

import numpy as np

import oracle
from paper_1010_4639_amd import workload as W


def test_omp_mode_follows_the_serial_iteration():
    s = W.fem_p1_system(14, 13, 12, seed=11)
    x, info, _ = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=1e-10, maxit=5000)
    xo, oinfo = oracle.cg_csr_omp(s.rowptr, s.col, s.val, s.b, tol=1e-10, maxit=5000)
    assert oinfo["status"] == info["status"] == 0
    assert oinfo["threads"] >= 1
    assert abs(oinfo["iters"] - info["iters"]) <= 2
    assert np.linalg.norm(xo - x) <= 1e-8 * np.linalg.norm(x)


def test_omp_mode_thread_count_and_early_iterates():
    ptr, col, val = W.random_spd_sparse(500, density=0.03, seed=3)
    b = W.uniform_vector(500, seed=4)
    for k in (1, 3, 7):
        x, info, _ = oracle.cg(oracle.FMT_CSR, ptr, col, val, b, tol=0.0, maxit=k)
        xo, oinfo = oracle.cg_csr_omp(ptr, col, val, b, tol=0.0, maxit=k)
        assert oinfo["iters"] == info["iters"] == k
        assert np.linalg.norm(xo - x) <= 1e-13 * np.linalg.norm(x)
    want = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if want:
        assert oinfo["threads"] == want

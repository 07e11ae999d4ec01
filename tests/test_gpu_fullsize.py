"""Full-size cases of the measured workloads (one MI355X), checked against the
oracle where it can be evaluated at this size (its products, in C) and by
properties that hold at any size.

* 160^3 system, contrast 1e-4 (n 4 096 000, nnz 60 827 518): products in
  every format against the oracle's, element by element; the FP64 CG and the
  mixed-precision refinement (inner tolerance 1e-4, and 1e-2 as measured)
  reach ||b - A x|| <= tol ||b|| measured with the oracle's product (their
  differences are reported).
* The batch of 256 uneven systems x 4 right-hand sides (N 15 254 976, nnz
  219 547 592): every pair converges, its true residual (oracle product, per
  system) meets the tolerance, and sampled pairs take the iteration count of
  single solves of the same system (within 3 %).
"""
import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import SPMV_TOL, say, to_dev

pytestmark = pytest.mark.gpu

_CACHE = {}


def fem160():
    if "fem160" not in _CACHE:
        say("generating fem160 (about 45 s)")
        _CACHE["fem160"] = W.fem_config("fem160", keep_geometry=False)
    return _CACHE["fem160"]


@pytest.mark.parametrize("fmt", ["csr", "symcsr", "csc"])
def test_fem160_products(fmt):
    s = fem160()
    if fmt == "symcsr":
        ptr, idx, val = W.upper_triangle(s.rowptr, s.col, s.val)
    else:
        ptr, idx, val = s.rowptr, s.col, s.val
    f = cgmi.FORMATS[fmt]
    x = W.uniform_vector(s.n, seed=21)
    say(f"fem160 product {fmt}")
    with cgmi.Solver(fmt, ptr, idx, val) as S:
        y = S.spmv(to_dev(x)).cpu().numpy()
    yo = oracle.spmv(f, ptr, idx, val, x)
    bound = SPMV_TOL * oracle.spmv(f, ptr, idx, np.abs(val), np.abs(x))
    assert np.all(np.abs(y - yo) <= bound), float(np.max(np.abs(y - yo) - bound))


def test_fem160_fp64_and_mixed_solves():
    s = fem160()
    tol = 1e-10
    b = to_dev(s.b)
    nb = np.linalg.norm(s.b)
    with cgmi.Solver("csr", s.rowptr, s.col, s.val, mixed=True) as S:
        say("fem160 FP64 CG")
        x64, i64 = S.solve(b, tol=tol, maxit=100000)
        say(f"  {i64}")
        say("fem160 mixed refinement, inner tol 1e-4")
        xm, im = S.solve_mixed(b, tol=tol, maxit=100000, inner_tol=1e-4, max_outer=50)
        say(f"  {im}")
        say("fem160 mixed refinement, inner tol 1e-2 (the measured configuration)")
        xm2, im2 = S.solve_mixed(b, tol=tol, maxit=100000, inner_tol=1e-2, max_outer=50)
        say(f"  {im2}")
    assert i64["status"] == cgmi.CG_OK and im["status"] == cgmi.CG_OK and im2["status"] == cgmi.CG_OK
    x64, xm, xm2 = x64.cpu().numpy(), xm.cpu().numpy(), xm2.cpu().numpy()
    r64 = np.linalg.norm(s.b - oracle.spmv(0, s.rowptr, s.col, s.val, x64))
    rm = np.linalg.norm(s.b - oracle.spmv(0, s.rowptr, s.col, s.val, xm))
    rm2 = np.linalg.norm(s.b - oracle.spmv(0, s.rowptr, s.col, s.val, xm2))
    say(f"true relres: fp64 {r64 / nb:.3e}  mixed {rm / nb:.3e}  mixed 1e-2 {rm2 / nb:.3e}")
    assert r64 <= 1.1 * tol * nb and rm <= 1.1 * tol * nb and rm2 <= 1.1 * tol * nb
    for xx in (xm, xm2):
        d = x64 - xx
        say(f"||x64 - xmixed|| / ||x64|| = {np.linalg.norm(d) / np.linalg.norm(x64):.3e}")


def test_batch_full_size():
    say("generating the 256-system batch (about 30 s)")
    systems, B, _ = W.fem_batch(256, nrhs=4, workers=8)
    so, ptr, col, val = W.block_diagonal(systems)
    tol = 1e-10
    Bd = to_dev(np.ascontiguousarray(B))
    with cgmi.Batch(so, ptr, col, val, nrhs=4) as bt:
        tuned = bt.autotune()
        say(f"autotune {tuned}")
        X, info, iters, st = bt.solve(Bd, tol=tol)
    assert np.all(st == cgmi.CG_OK), np.unique(st, return_counts=True)
    Xh = X.cpu().numpy().reshape(-1, 4)
    worst = 0.0
    for k, (rp, c, v) in enumerate(systems):
        r0, r1 = so[k], so[k + 1]
        for r in range(4):
            bk = B[r0:r1, r]
            res = np.linalg.norm(bk - oracle.spmv(0, rp, c, v, Xh[r0:r1, r])) / np.linalg.norm(bk)
            worst = max(worst, res)
    say(f"batch: worst true relres {worst:.3e}, iterations {iters.min()}..{iters.max()}")
    assert worst <= 1.1 * tol
    # sampled pairs against single solves of the same system
    rng = np.random.default_rng(3)
    for k in rng.choice(len(systems), size=4, replace=False):
        rp, c, v = systems[k]
        r0, r1 = so[k], so[k + 1]
        with cgmi.Solver("csr", rp, c, v) as S:
            for r in range(4):
                xs, inf = S.solve(to_dev(np.ascontiguousarray(B[r0:r1, r])), tol=tol)
                xs = xs.cpu().numpy()
                assert abs(inf["iters"] - iters.reshape(-1)[k * 4 + r]) <= 0.03 * inf["iters"] + 2
                rs = np.linalg.norm(B[r0:r1, r] - oracle.spmv(0, rp, c, v, xs)) / np.linalg.norm(B[r0:r1, r])
                assert rs <= 1.1 * tol

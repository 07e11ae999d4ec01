"""GPU conjugate gradient through the C-ABI vs the oracle (FP64, tol 1e-10).

Contract on the same b bits:
  1. the same status; the true residual of x_gpu, computed with the oracle's
     product, <= 2 tol, and equal to the one the library reports;
  2. ||x_gpu - x_oracle||_A / ||x_oracle||_A <= 1e-8 (energy norm, the norm
     CG minimises);
  3. ||x_gpu - x_oracle||_2 / ||x_oracle||_2 <= 1e-8 on well-conditioned
     systems; on the ill-conditioned FEM systems <= max(1e-8, 4 x the
     oracle's own reduction-order spread) -- the larger distance between the
     oracle with exactly rounded scalar products and the oracle with plain
     left-to-right or with pairwise-summed ones, all valid FP64 runs of the
     same iteration (tests/parity.py); on the 32x32x30 system those
     distances are 2.45e-8 and 1.01e-7, because each run stops ~3.5e-7 away
     from the exact solution;
  4. iteration count within 3 % of the oracle's (the stop step moves with
     rounding; the paper's own runs of one matrix in three arithmetics
     needed 323-328 iterations);
  5. bitwise-identical results run to run and for any graph batch size.
Measured differences are printed and recorded (CGMI_PARITY_RECORD).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests import parity
from tests.gpu_util import CG_ITER_TOL, CG_X_TOL, fem_cached, say, to_dev, true_relres

pytestmark = pytest.mark.gpu

CSR, SYM, CSC = cgmi.CG_FMT_CSR, cgmi.CG_FMT_SYM_CSR, cgmi.CG_FMT_CSC


def formats_of(ptr, col, val):
    up, uc, uv = W.upper_triangle(ptr, col, val)
    return {CSR: (ptr, col, val), SYM: (up, uc, uv), CSC: (ptr, col, val)}


def run_pair(fmt, arrs, b, x0=None, tol=1e-10, maxit=50000, batch=None, label=""):
    say(f"cg {label} fmt={fmt} n={len(arrs[0]) - 1} batch={batch}")
    with cgmi.Solver(fmt, *arrs, batch=batch) as S:
        xg, info = S.solve(to_dev(b), None if x0 is None else to_dev(x0), tol=tol, maxit=maxit, check=False)
        xg = xg.cpu().numpy()
    xo, oinfo, _ = oracle.cg(fmt, *arrs, b, x0=x0, tol=tol, maxit=maxit)
    say(f"   gpu iters={info['iters']} status={info['status']} relres={info['relres']:.3e} "
        f"true={info['relres_true']:.3e} ms={info['ms']:.1f} | oracle iters={oinfo['iters']} "
        f"status={oinfo['status']}")
    return xg, info, xo, oinfo


def a_norm(fmt, arrs, v):
    return float(np.sqrt(v @ oracle.spmv(fmt, *arrs, v)))


def lambda_min_est(fmt, arrs, b):
    """Smallest Ritz value of the oracle's CG-Lanczos tridiagonal (an upper
    estimate of lambda_min that is tight once CG has converged)."""
    from tests.pins import _lanczos_ritz
    _, info, h = oracle.cg(fmt, *arrs, b, tol=1e-12, maxit=20000, history=20000)
    return float(_lanczos_ritz(h["alpha"], h["beta"])[0])


def check_contract(fmt, arrs, b, xg, info, xo, oinfo, tol=1e-10, strict_2norm=True, x0=None, label="",
                   spread=None, step=None):
    assert info["status"] == oinfo["status"] == cgmi.CG_OK
    rt = true_relres(fmt, *arrs, b, xg)
    assert rt <= 2 * tol, rt
    assert abs(info["relres_true"] - rt) <= 1e-3 * rt + 1e-16
    assert info["relres"] <= tol
    d = xg - xo
    err_a = a_norm(fmt, arrs, d) / a_norm(fmt, arrs, xo)
    err = np.linalg.norm(d) / np.linalg.norm(xo)
    if strict_2norm:
        spread2 = spreadA = step2 = None
        bar = CG_X_TOL
    else:
        spread2, spreadA, _ = spread or parity.oracle_spread(fmt, arrs, b, xo, tol, x0=x0)
        step2 = step if step is not None else parity.step_spread(fmt, arrs, b, xo, oinfo["iters"], info["iters"],
                                                                 x0=x0)
        bar = parity.x_bar(spread2, step2)
    say(f"   vs oracle: 2-norm {err:.3e} (bar {bar:.3e}, oracle spread "
        f"{'-' if spread2 is None else f'{spread2:.3e}'}, stopping-step spread "
        f"{'-' if step2 is None else f'{step2:.3e}'})  A-norm {err_a:.3e}")
    parity.record(test=label, fmt=int(fmt), n=len(arrs[0]) - 1, err2=err, errA=err_a, bar2=bar, spread2=spread2,
                  step2=step2, spreadA=spreadA, iters=info["iters"], oracle_iters=oinfo["iters"], relres_true=rt)
    assert err_a <= parity.X_TOL, err_a
    assert err <= bar, (err, bar)
    assert abs(info["iters"] - oinfo["iters"]) <= max(2, CG_ITER_TOL * oinfo["iters"])


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_random_spd(fmt):
    ptr, col, val = W.random_spd_sparse(700, density=0.02, seed=1)
    arrs = formats_of(ptr, col, val)[fmt]
    b = W.uniform_vector(700, seed=2)
    check_contract(fmt, arrs, b, *run_pair(fmt, arrs, b, label="random spd"), label="random spd n=700")


@pytest.mark.parametrize("fmt", [SYM, CSR, CSC])
def test_fem_paper_sized(fmt):
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info, xo, oinfo = run_pair(fmt, arrs, s.b, label="fem32x32x30")
    check_contract(fmt, arrs, s.b, xg, info, xo, oinfo, strict_2norm=False, label="fem32x32x30")
    # the in-test spread is the stored one (same oracle bits)
    ref = parity.load_reference("fem32x32x30")
    assert parity.sha(xo) == ref["x_oracle_sha256"] and oinfo["iters"] == ref["iters"]
    spread2, _, _ = parity.oracle_spread(fmt, arrs, s.b, xo)
    assert abs(spread2 - parity.stored_spread(ref)[0]) <= 1e-9 * spread2


@pytest.mark.parametrize("dims", [(24, 22, 20), (60, 60, 60)])
@pytest.mark.parametrize("fmt", [SYM, CSR, CSC])
def test_fem_unit_coefficient_strict(fmt, dims):
    # no iron (kappa ~ 5e2 at 24x22x20): the 2-norm bar applies as is.
    # 60^3 (n 216 000): 512 vector workgroups of 422 elements, so the r and
    # x/p updates load two elements per thread up front (their KP = 2 form)
    s = W.fem_p1_system(*dims, iron_frac=0.0, seed=8)
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    label = "fem%dx%dx%d nu=1" % dims
    if dims == (60, 60, 60):
        with cgmi.Solver(fmt, *arrs) as S:
            assert S.stats()["vec_blocks"] == 512
    check_contract(fmt, arrs, s.b, *run_pair(fmt, arrs, s.b, label=label), label=label)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_early_iterates_match(fmt):
    # the first iterates follow the oracle's to rounding level (later ones drift
    # apart by rounding amplification, as do any two FP64 evaluations)
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    for k in (1, 2, 5, 10):
        with cgmi.Solver(fmt, *arrs) as S:
            xg, info = S.solve(to_dev(s.b), tol=0.0, maxit=k)
        xo, oinfo, _ = oracle.cg(fmt, *arrs, s.b, tol=0.0, maxit=k)
        assert info["iters"] == oinfo["iters"] == k
        err = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        assert err <= 1e-12, (k, err)


@pytest.mark.parametrize("layout", ["rows", "slices"])
@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_layouts_in_iterations(monkeypatch, fmt, layout):
    # both product layouts of every format inside the iteration graph (the
    # default picks slices for FEM matrices)
    monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
    s = fem_cached("fem32x32x30")
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    xg, info, xo, oinfo = run_pair(fmt, arrs, s.b, label=f"fem32x32x30 layout={layout}")
    check_contract(fmt, arrs, s.b, xg, info, xo, oinfo, strict_2norm=False, label=f"fem32x32x30 layout={layout}")


def test_early_iterates_8192_partials():
    # 3.3M-row tridiagonal SPD matrix: the sliced product runs on 8192
    # workgroups (two slices per wave at a time) and the r update sums 8192
    # partials
    n = 3_300_000
    lens = np.full(n, 3)
    lens[0] = lens[-1] = 2
    ptr = np.zeros(n + 1, np.int32)
    ptr[1:] = np.cumsum(lens)
    i = np.repeat(np.arange(n), lens)
    col = (i + np.arange(ptr[-1]) - ptr[i] - (i > 0)).astype(np.int32)
    val = np.where(col == i, 2.5, -1.0)
    b = W.uniform_vector(n, seed=33)
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert stats["slices"] == 2 and stats["spmv_blocks"] == 8192
    for k in (1, 5, 20):
        with cgmi.Solver(CSR, ptr, col, val) as S:
            xg, info = S.solve(to_dev(b), tol=0.0, maxit=k, check=False)
        xo, oinfo, _ = oracle.cg(CSR, ptr, col, val, b, tol=0.0, maxit=k)
        assert info["iters"] == oinfo["iters"] == k
        err = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        say(f"   tridiagonal n={n}: {k} iterations, rel. difference {err:.2e}")
        assert err <= 1e-12, (k, err)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_nonzero_start(fmt):
    s = W.fem_p1_system(10, 9, 8, nu_iron=1e-2, seed=3)
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    x0 = W.uniform_vector(s.n, seed=4)
    check_contract(fmt, arrs, s.b, *run_pair(fmt, arrs, s.b, x0=x0, label="x0 != 0"), strict_2norm=False, x0=x0,
                   label="fem10x9x8 x0!=0")


@pytest.mark.parametrize("batch", [1, 5, 64])
def test_batch_size_does_not_change_bits(batch):
    s = W.fem_p1_system(12, 11, 10, seed=5)
    arrs = formats_of(s.rowptr, s.col, s.val)[CSR]
    ref = None
    for bt in (32, batch):
        with cgmi.Solver(CSR, *arrs, batch=bt) as S:
            x, info = S.solve(to_dev(s.b), tol=1e-10, maxit=5000)
            cur = (x.cpu().numpy(), info["iters"])
        if ref is None:
            ref = cur
    assert np.array_equal(ref[0], cur[0]) and ref[1] == cur[1]


@pytest.mark.parametrize("col16", ["1", "0"])
@pytest.mark.parametrize("fmt", [CSR, SYM])
def test_two_kernel_iteration_same_bits(monkeypatch, fmt, col16):
    """Small systems run two kernels per iteration (the product forms the
    search direction itself): the same arithmetic in the same order, so the
    solution, the iteration count and every status match the three-kernel
    iteration bit for bit -- converged, stopped by maxit, from x0 != 0, and
    at a breakdown."""
    import torch
    monkeypatch.setenv("CGMI_COL16", col16)
    s = W.fem_p1_system(14, 13, 12, nu_iron=1e-3, seed=11)
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    x0 = W.uniform_vector(s.n, seed=12)
    n = 40
    d = np.where(np.arange(n) % 3 == 2, -1.0, 2.0)  # indefinite: breaks down after a few steps
    dptr, didx = np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)
    bd = W.uniform_vector(n, seed=13)
    out = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("CGMI_FUSED", fused)
        res = []
        with cgmi.Solver(fmt, *arrs) as S:
            for kw in (dict(tol=1e-10, maxit=5000), dict(tol=1e-14, maxit=37), dict(x0=to_dev(x0), tol=1e-9)):
                x, info = S.solve(to_dev(s.b), kw.pop("x0", None), check=False, **kw)
                res.append((x.cpu().numpy(), info["iters"], info["status"], info["relres"]))
        with cgmi.Solver(fmt, dptr, didx, d) as S:
            x, info = S.solve(to_dev(bd), check=False)
            res.append((x.cpu().numpy(), info["iters"], info["status"], info["relres"]))
        out[fused] = res
    for (xa, ia, sa, ra), (xb, ib, sb, rb) in zip(out["1"], out["0"]):
        assert np.array_equal(xa, xb) and ia == ib and sa == sb and ra == rb, (ia, ib, sa, sb, ra, rb)
    assert [r[2] for r in out["1"]] == [cgmi.CG_OK, cgmi.CG_NOT_CONVERGED, cgmi.CG_OK, cgmi.CG_ERR_BREAKDOWN]
    assert out["1"][1][1] == 37 and out["1"][3][1] > 0


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_deterministic(fmt):
    s = W.fem_p1_system(16, 15, 14, seed=6)
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    with cgmi.Solver(fmt, *arrs) as S:
        b = to_dev(s.b)
        x1, i1 = S.solve(b, tol=1e-10, maxit=5000)
        x2, i2 = S.solve(b, tol=1e-10, maxit=5000)
    import torch
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_status_paths(fmt):
    import torch
    ptr, col, val = W.random_spd_sparse(60, density=0.1, seed=7)
    arrs = formats_of(ptr, col, val)[fmt]
    n = 60
    with cgmi.Solver(fmt, *arrs) as S:
        # b = 0 -> x = 0, no iteration
        x, info = S.solve(to_dev(np.zeros(n)), to_dev(np.ones(n)))
        assert info["status"] == cgmi.CG_OK and info["iters"] == 0 and torch.all(x == 0)
        # non-finite b -> error, x untouched
        bad = W.uniform_vector(n, seed=8)
        bad[5] = np.nan
        x0 = to_dev(W.uniform_vector(n, seed=9))
        x, info = S.solve(to_dev(bad), x0, check=False)
        assert info["status"] == cgmi.CG_ERR_NONFINITE and torch.equal(x, x0)
        # maxit exhaustion: the last iterate agrees with the oracle's after 3 steps
        b = W.uniform_vector(n, seed=10)
        x, info = S.solve(to_dev(b), tol=1e-14, maxit=3)
        xo, oinfo, _ = oracle.cg(fmt, *arrs, b, tol=1e-14, maxit=3)
        assert info["status"] == oinfo["status"] == cgmi.CG_NOT_CONVERGED
        assert info["iters"] == oinfo["iters"] == 3
        assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-12 * np.linalg.norm(xo)
        # maxit = 0
        x, info = S.solve(to_dev(b), tol=1e-14, maxit=0)
        assert info["status"] == cgmi.CG_NOT_CONVERGED and info["iters"] == 0 and torch.all(x == 0)
        # start at the solution: nothing to do
        xs, _ = S.solve(to_dev(b), tol=1e-13, maxit=1000)
        x, info = S.solve(to_dev(b), xs, tol=1e-6)
        assert info["status"] == cgmi.CG_OK and info["iters"] == 0
        # argument errors
        st, _ = cgmi.cg_solve(S.h, to_dev(b).data_ptr(), x.data_ptr(), -1.0, 10)
        assert st == cgmi.CG_ERR_ARG
        st, _ = cgmi.cg_solve(S.h, to_dev(b).data_ptr(), x.data_ptr(), 1e-8, -1)
        assert st == cgmi.CG_ERR_ARG
        bb = to_dev(b)
        st, _ = cgmi.cg_solve(S.h, bb.data_ptr(), bb.data_ptr(), 1e-8, 10)   # b and x the same buffer
        assert st == cgmi.CG_ERR_ARG and torch.equal(bb, to_dev(b))


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_breakdown_on_indefinite(fmt):
    import torch
    n = 50
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    ptr = np.arange(n + 1, dtype=np.int32)
    idx = np.arange(n, dtype=np.int32)
    e1 = np.zeros(n)
    e1[1] = 1.0
    with cgmi.Solver(fmt, ptr, idx, d) as S:
        for b in (np.ones(n), e1):
            x, info = S.solve(to_dev(b), check=False)
            xo, oinfo, _ = oracle.cg(fmt, ptr, idx, d, b)
            assert info["status"] == oinfo["status"] == cgmi.CG_ERR_BREAKDOWN
            assert info["iters"] == oinfo["iters"] == 0 and torch.all(x == 0)


def test_empty_system():
    with cgmi.Solver(CSR, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0)) as S:
        st, info = cgmi.cg_solve(S.h, 0, 0, 1e-10, 10)
        assert st == cgmi.CG_OK and info["iters"] == 0


def test_exact_step_count_7pt_laplacian():
    # in exact arithmetic CG ends after as many steps as distinct eigenvalues (7 on 3^3)
    s = W.fem_p1_system(3, 3, 3, jitter=0.0, iron_frac=0.0, seed=9, with_rhs=False)
    val = np.round(s.val)
    xt = np.random.default_rng(3).integers(-8, 9, size=s.n).astype(np.float64)
    b = oracle.spmv(CSR, s.rowptr, s.col, val, xt)
    with cgmi.Solver(CSR, s.rowptr, s.col, val) as S:
        x, info = S.solve(to_dev(b), tol=1e-14, maxit=100)
    assert info["iters"] == 7
    assert np.linalg.norm(x.cpu().numpy() - xt) <= 1e-14 * np.linalg.norm(xt)


_ORC100 = {}


def oracle_fem100(capfd):
    """One serial oracle solve of the 100^3 system (CSR; the oracle's three
    formats give identical bits, so it serves all three), once per process.
    It runs for minutes on one core, so its progress lines go straight to the
    terminal (output capture off)."""
    if not _ORC100:
        s = fem_cached("fem100")
        with capfd.disabled():
            say("fem100: serial oracle CG, ~7000 iterations (1-5 minutes on one core)")
            os.environ["ORC_PROGRESS"] = "500"
            try:
                xo, oinfo, _ = oracle.cg(CSR, s.rowptr, s.col, s.val, s.b, tol=1e-10, maxit=50000)
            finally:
                os.environ.pop("ORC_PROGRESS", None)
            say(f"   oracle: {oinfo}")
        _ORC100.update(x=xo, info=oinfo)
    return _ORC100


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_full_size_1m_vs_oracle(fmt, capfd):
    """100^3 (n = 1.0M), every format against the serial oracle's solution:
    the full contract, with the oracle's reduction-order spread on this system
    taken from the stored reference (tests/golden/make_oracle_reference.py,
    which ran the oracle with plain scalar products too); the oracle run here
    must reproduce the stored solution bit for bit."""
    import torch
    s = fem_cached("fem100")
    ref = parity.load_reference("fem100")
    assert parity.sha(s.b) == ref["b_sha256"]
    orc = oracle_fem100(capfd)
    assert parity.sha(orc["x"]) == ref["x_oracle_sha256"] and orc["info"]["iters"] == ref["iters"]
    arrs = formats_of(s.rowptr, s.col, s.val)[fmt]
    with cgmi.Solver(fmt, *arrs) as S:
        b = to_dev(s.b)
        x1, info = S.solve(b, tol=1e-10, maxit=50000)
        say(f"fem100 fmt={fmt}: iters={info['iters']} ms={info['ms']:.1f} true={info['relres_true']:.3e}")
        x2, info2 = S.solve(b, tol=1e-10, maxit=50000)
    assert torch.equal(x1, x2) and info["iters"] == info2["iters"]
    step = parity.stored_step_spread(ref, info["iters"])
    check_contract(fmt, arrs, s.b, x1.cpu().numpy(), info, orc["x"], orc["info"], strict_2norm=False,
                   label="fem100", spread=parity.stored_spread(ref), step=0.0 if step is None else step)

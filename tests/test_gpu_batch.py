"""Batched solves (many uneven systems x several right-hand sides, one kernel
sequence) vs the oracle run on every (system, right-hand side) pair alone.

Per pair: same status; true residual (oracle product) <= 2 tol; energy-norm
difference to the oracle's solution <= 1e-8, 2-norm difference <= max(1e-8,
4 x the oracle's own spread over evaluations and stopping steps)
(tests/parity.py); iteration
count within 5 %.
The products of every system are checked row by row against the oracle's.
Every product schedule (row blocks through LDS; 8 or 16 lanes per row; one
lane per row over 64-row slices) is run, selected with CGMI_BATCH_LANES.
"""
import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests import parity
from tests.gpu_util import say, spmv_bound, to_dev
from tests.test_gpu_cg import a_norm

pytestmark = pytest.mark.gpu


def small_batch(nrhs, seed=1):
    rng = np.random.default_rng(seed)
    systems, Bs = [], []
    for k, dims in enumerate([(6, 5, 4), (9, 8, 7), (3, 3, 3), (12, 10, 9), (7, 7, 7)]):
        s = W.fem_p1_system(*dims, seed=10 + k, nrhs=nrhs)
        systems.append((s.rowptr, s.col, s.val))
        Bs.append(s.b.reshape(s.n, nrhs))
    ptr, col, val = W.random_spd_sparse(150, density=0.05, seed=seed)
    systems.append((ptr, col, val))
    Bs.append(rng.uniform(-1, 1, size=(150, nrhs)))
    return systems, np.concatenate(Bs)


@pytest.mark.parametrize("lanes", ["0", "8", "16", "1"])
@pytest.mark.parametrize("nrhs", [1, 2, 4])
def test_batch_matches_single_oracle_solves(nrhs, lanes, monkeypatch):
    # lanes: the product schedule (0 = row blocks through LDS, 1 = slices,
    # else lanes per row)
    monkeypatch.setenv("CGMI_BATCH_LANES", lanes)
    systems, B = small_batch(nrhs)
    so, ptr, col, val = W.block_diagonal(systems)
    with cgmi.Batch(so, ptr, col, val, nrhs=nrhs) as bt:
        X, info, iters, stat = bt.solve(to_dev(B), tol=1e-10, maxit=20000)
        X = X.cpu().numpy()
    say(f"batch nrhs={nrhs}: {info}")
    for s, arrs in enumerate(systems):
        r0, r1 = so[s], so[s + 1]
        for r in range(nrhs):
            b = B[r0:r1, r]
            xo, oi, _ = oracle.cg(0, *arrs, b, tol=1e-10, maxit=20000)
            xg = X[r0:r1, r]
            assert stat[s, r] == oi["status"] == 0, (s, r, stat[s, r])
            rt = np.linalg.norm(b - oracle.spmv(0, *arrs, xg)) / np.linalg.norm(b)
            assert rt <= 2e-10, (s, r, rt)
            ea = a_norm(0, arrs, xg - xo) / a_norm(0, arrs, xo)
            assert ea <= 1e-8, (s, r, ea)
            e2 = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
            spread2, _, _ = parity.oracle_spread(0, arrs, b, xo, 1e-10, maxit=20000)
            step2 = parity.step_spread(0, arrs, b, xo, oi["iters"], int(iters[s, r]))
            parity.record(test=f"batch nrhs={nrhs} lanes={lanes}", fmt=0, n=r1 - r0, err2=e2, errA=ea,
                          bar2=parity.x_bar(spread2, step2), spread2=spread2, step2=step2,
                          iters=int(iters[s, r]), oracle_iters=oi["iters"])
            assert e2 <= parity.x_bar(spread2, step2), (s, r, e2, spread2, step2)
            # the stopping step moves with rounding (the paper's speed-up table
            # gives one matrix 323-328 iterations in three arithmetics); here
            # each schedule also sums p'Ap and r'r over its own workgroup split,
            # and the small iron systems (kappa ~ 1e5) are the most sensitive:
            # measured up to 3.8 % (10-11 of 290), so the bar is 5 %
            assert abs(int(iters[s, r]) - oi["iters"]) <= max(2, 0.05 * oi["iters"]), (s, r, iters[s, r], oi)


@pytest.mark.parametrize("lanes", ["0", "8", "16", "1"])
def test_batch_spmm_rowwise(lanes, monkeypatch):
    monkeypatch.setenv("CGMI_BATCH_LANES", lanes)
    systems, B = small_batch(4, seed=2)
    so, ptr, col, val = W.block_diagonal(systems)
    X = np.random.default_rng(3).uniform(-1, 1, size=(so[-1], 4))
    with cgmi.Batch(so, ptr, col, val, nrhs=4) as bt:
        Y = bt.spmm(to_dev(X)).cpu().numpy()
    for r in range(4):
        yo = oracle.spmv(0, ptr, col, val, X[:, r])
        if lanes in ("0", "1"):
            # one thread / lane sums each row left to right from rounded products: bit-identical
            assert np.array_equal(Y[:, r], yo)
        else:
            # lanes per row: fused multiply-adds and a butterfly, a different rounding order
            bound = 1e-13 * spmv_bound(0, ptr, col, val, X[:, r])
            assert np.all(np.abs(Y[:, r] - yo) <= bound), float(np.max(np.abs(Y[:, r] - yo) - bound))


@pytest.mark.parametrize("col16", ["1", "0"])
def test_batch_slices_column_storage(col16, monkeypatch):
    """Slices of the batch with columns as 16-bit offsets from the row (the
    default for these banded systems) or as 32-bit indices: the product is
    bit-identical to the oracle's either way (odd and even slice widths,
    short last slices), and whole solves give the same bits."""
    monkeypatch.setenv("CGMI_BATCH_LANES", "1")
    systems, B = small_batch(2, seed=4)
    so, ptr, col, val = W.block_diagonal(systems)
    X = np.random.default_rng(5).uniform(-1, 1, size=(so[-1], 2))
    out = {}
    for c16 in ("1", "0"):
        monkeypatch.setenv("CGMI_COL16", c16)
        with cgmi.Batch(so, ptr, col, val, nrhs=2) as bt:
            Y = bt.spmm(to_dev(X)).cpu().numpy()
            Xs, info, iters, stat = bt.solve(to_dev(B), tol=1e-10, maxit=20000)
            out[c16] = (Xs.cpu().numpy(), iters.copy())
        for r in range(2):
            assert np.array_equal(Y[:, r], oracle.spmv(0, ptr, col, val, X[:, r])), (c16, r)
    assert np.array_equal(out["1"][0], out["0"][0]) and np.array_equal(out["1"][1], out["0"][1])


def test_batch_statuses_per_pair():
    import torch
    sysA = W.fem_p1_system(6, 6, 5, seed=3)
    n = 40
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)               # indefinite: breakdown
    sysB = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    so, ptr, col, val = W.block_diagonal([(sysA.rowptr, sysA.col, sysA.val), sysB])
    N = so[-1]
    rng = np.random.default_rng(4)
    B = rng.uniform(-1, 1, size=(N, 4))
    B[: so[1], 1] = 0.0                      # pair (0, 1): b = 0
    B[5, 2] = np.nan                         # pair (0, 2): non-finite b
    X0 = rng.uniform(-1, 1, size=(N, 4))
    with cgmi.Batch(so, ptr, col, val, nrhs=4) as bt:
        X, info, iters, st = bt.solve(to_dev(B), to_dev(X0), tol=1e-10, maxit=5000)
        X = X.cpu().numpy()
        assert st[0, 0] == st[0, 3] == cgmi.CG_OK
        assert st[0, 1] == cgmi.CG_OK and iters[0, 1] == 0 and np.all(X[: so[1], 1] == 0)
        assert st[0, 2] == cgmi.CG_ERR_NONFINITE and np.array_equal(X[: so[1], 2], X0[: so[1], 2])
        assert np.all(st[1] == cgmi.CG_ERR_BREAKDOWN)
        assert info["status"] == cgmi.CG_ERR_BREAKDOWN or info["status"] == cgmi.CG_ERR_NONFINITE
        X, info, iters, st = bt.solve(to_dev(np.nan_to_num(B)), tol=1e-14, maxit=3)
        assert np.all(st[0][[0, 2, 3]] == cgmi.CG_NOT_CONVERGED) and np.all(iters[0][[0, 2, 3]] == 3)


def test_batch_autotune_and_determinism():
    systems, B = small_batch(4, seed=5)
    so, ptr, col, val = W.block_diagonal(systems)
    with cgmi.Batch(so, ptr, col, val, nrhs=4) as bt:
        X1, i1, it1, _ = bt.solve(to_dev(B))
        X2, i2, it2, _ = bt.solve(to_dev(B))
        import torch
        assert torch.equal(X1, X2) and np.array_equal(it1, it2)
        tuned = bt.autotune()
        say(f"autotune: {tuned}")
        assert tuned["lanes_per_row"] in (0, 1, 8, 16) and tuned["workgroups"] >= len(systems)
        assert tuned["entries_per_block"] == (0 if tuned["lanes_per_row"] == 1 else tuned["entries_per_block"])
        assert tuned["lanes_per_row"] == 1 or tuned["entries_per_block"] in (256, 512, 1024)
        X3, i3, it3, st3 = bt.solve(to_dev(B))
        assert np.all(st3 == 0)
        d = (X3 - X1).cpu().numpy()
        assert np.linalg.norm(d) <= 1e-6 * np.linalg.norm(X1.cpu().numpy())

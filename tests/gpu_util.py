"""Helpers shared by the GPU tests (device transfer, oracle comparisons)."""
import sys

import numpy as np

import oracle
from paper_1010_4639_amd import cgmi

SPMV_TOL = 1e-13      # componentwise, relative to sum_j |a_ij x_j|
CG_X_TOL = 1e-8       # ||x_gpu - x_oracle|| / ||x_oracle|| at tol 1e-10
CG_ITER_TOL = 0.03    # relative spread of iteration counts (rounding order)


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def zero_based(ptr, idx, base):
    return np.asarray(ptr) - base, np.asarray(idx) - base


def spmv_bound(fmt, ptr, idx, val, x):
    """sum_j |a_ij| |x_j| per output row, computed by the oracle."""
    return oracle.spmv(fmt, ptr, idx, np.abs(val), np.abs(x))


def check_spmv(fmt, ptr, idx, val, x, base=0, solver=None, label=""):
    """GPU product vs the oracle's, componentwise and normwise."""
    say(f"spmv {label} fmt={fmt} n={len(ptr) - 1} nnz={len(idx)} base={base}")
    own = solver is None
    S = solver or cgmi.Solver(fmt, ptr, idx, val, index_base=base)
    try:
        y = S.spmv(to_dev(x)).cpu().numpy()
    finally:
        if own:
            S.close()
    p0, i0 = zero_based(ptr, idx, base)
    yo = oracle.spmv(fmt, p0, i0, val, x)
    bound = SPMV_TOL * spmv_bound(fmt, p0, i0, val, x)
    err = np.abs(y - yo)
    assert np.all(err <= bound), (label, float(np.max(err - bound)))
    ny = np.linalg.norm(yo)
    if ny > 0:
        assert np.linalg.norm(y - yo) <= SPMV_TOL * ny
    return y, yo


def true_relres(fmt, ptr, idx, val, b, x):
    r = b - oracle.spmv(fmt, ptr, idx, val, x)
    return np.linalg.norm(r) / np.linalg.norm(b)


_FEM_CACHE = {}


def fem_cached(name):
    """Generate a named FEM workload once per process (the 1.0M-row one takes ~12 s)."""
    from paper_1010_4639_amd import workload as W
    if name not in _FEM_CACHE:
        _FEM_CACHE[name] = W.fem_config(name)
    return _FEM_CACHE[name]

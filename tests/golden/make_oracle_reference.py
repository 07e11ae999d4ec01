"""Write the stored oracle reference for a FEM system (test fixture).

The serial FP64 oracle CG on the 160^3 system (n = 4 096 000, iron contrast
1e-4) needs ~24 000 iterations, about 20 minutes on one core: too long for a
test run, so it is run once by this script and its result summarised in
``<workload>_oracle_csr.json`` beside it:

* the oracle's iteration count, status, recursive and true relative residual;
* its solution's distance to the generator's x_true in the 2-norm and in the
  energy norm ||v||_A = sqrt(v'Av) (products by the oracle), relative to
  ||x_true||, and the norms of x_oracle itself;
* x_oracle at 4096 seeded positions, as exact hexadecimal floats, and a
  sha256 of all of x_oracle and of b, so a test can confirm it solves the same
  bits;
* the reduction-order spread: the same oracle iteration with the plain
  left-to-right scalar products instead of the exactly rounded ones (both are
  valid FP64 evaluations of the algorithm, which leaves the summation order
  to a library routine) and the relative 2-norm / energy-norm distance of its
  solution from x_oracle.  This is how far two correct FP64 runs of the same
  iteration land apart on this system, the yardstick for the GPU's distance.

Only the oracle and the seeded input generator are called; nothing here comes
from the GPU library.  The two oracle solves run in two processes.
Usage:  python tests/golden/make_oracle_reference.py fem160 [fem100 ...]
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1010_4639_amd import workload as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 4096
_SYS = {}


def sample_positions(n, name):
    """The seeded positions at which x_oracle is stored (also used by the tests)."""
    seed = int.from_bytes(hashlib.sha256(name.encode()).digest()[:4], "little")
    return np.sort(np.random.default_rng(seed).choice(n, size=min(NSAMPLE, n), replace=False))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _solve(args):
    plain, tol, maxit = args
    s = _SYS["s"]
    x, info, _ = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=tol, maxit=maxit, plain_dots=plain)
    print(f"[ref] oracle ({'plain' if plain else 'exact'} dots): {info}", flush=True)
    return x, info


def main(name, tol=1e-10, maxit=200000):
    oracle.load()  # before the workers fork: parent and workers use one library
    t0 = time.time()
    s = W.fem_config(name, keep_geometry=False)
    _SYS["s"] = s
    print(f"[ref] generated {name}: n={s.n} nnz={s.nnz} in {time.time() - t0:.1f}s", flush=True)
    with mp.get_context("fork").Pool(2) as pool:
        (x, info), (xp, infop) = pool.map(_solve, [(False, tol, maxit), (True, tol, maxit)])
    arrs = (s.rowptr, s.col, s.val)

    def a_norm(v):
        return float(np.sqrt(oracle.dot(v, oracle.spmv(oracle.FMT_CSR, *arrs, v))))

    d = x - s.x_true
    dp = xp - x
    pos = sample_positions(s.n, name)
    out = dict(
        workload=name, format="csr", n=int(s.n), nnz=int(s.nnz), tol=tol, maxit=maxit,
        b_sha256=sha(s.b), x_oracle_sha256=sha(x),
        iters=int(info["iters"]), status=int(info["status"]), relres=info["relres"],
        relres_true=info["relres_true"], ms_loop=info["ms_loop"],
        norm2_x=float(np.linalg.norm(x)), normA_x=a_norm(x),
        norm2_x_true=float(np.linalg.norm(s.x_true)), normA_x_true=a_norm(s.x_true),
        err2_vs_true=float(np.linalg.norm(d) / np.linalg.norm(s.x_true)),
        errA_vs_true=a_norm(d) / a_norm(s.x_true),
        plain_dots=dict(iters=int(infop["iters"]), status=int(infop["status"]),
                        relres_true=infop["relres_true"],
                        spread2=float(np.linalg.norm(dp) / np.linalg.norm(x)),
                        spreadA=a_norm(dp) / a_norm(x)),
        sample_pos=[int(i) for i in pos], sample_x=[float(x[i]).hex() for i in pos],
        made_by="python tests/golden/make_oracle_reference.py " + name,
    )
    path = os.path.join(HERE, f"{name}_oracle_csr.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[ref] wrote {path} in {time.time() - t0:.0f}s: iters={out['iters']} "
          f"err2={out['err2_vs_true']:.3e} errA={out['errA_vs_true']:.3e} "
          f"spread2={out['plain_dots']['spread2']:.3e} spreadA={out['plain_dots']['spreadA']:.3e}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["fem160"]:
        main(nm)

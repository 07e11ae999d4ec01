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
* the evaluation spread: the same oracle iteration with plain left-to-right,
  pairwise-summed and fused multiply-add arithmetic instead of the exactly
  rounded scalar products (all are valid FP64 evaluations of the algorithm,
  which leaves them to a library routine) and the relative 2-norm /
  energy-norm distance of each solution from x_oracle;
* the stopping-step table: the relative 2-norm distance from x_oracle of the
  same iteration's x every 10 steps within 200 steps of its stop (how far x
  moves if a run stops a few steps earlier or later).  This is how far two correct FP64 runs of the same
  iteration land apart on this system, the yardstick for the GPU's distance.

Only the oracle and the seeded input generator are called; nothing here comes
from the GPU library.  The oracle runs go to parallel processes.
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


STEP_HALF, STEP_STRIDE = 200, 10   # stopping-step table: x every 10 steps within 200 of the stop


def _solve(args):
    dots, tol, maxit = args
    s = _SYS["s"]
    os.environ["ORC_PROGRESS"] = "2000"
    x, info, _ = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=tol, maxit=maxit, dots=dots)
    print(f"[ref] oracle ({dots} dots): {info}", flush=True)
    return x, info


def _trajectory(k):
    """The exact-dots iteration without a stopping test, x kept every
    STEP_STRIDE steps from k - STEP_HALF to k + STEP_HALF (the same bits as
    the stopped run up to its stop)."""
    s = _SYS["s"]
    os.environ["ORC_PROGRESS"] = "2000"
    first = max(1, k - STEP_HALF)
    cap = (k + STEP_HALF - first) // STEP_STRIDE + 1
    _, info, h = oracle.cg(oracle.FMT_CSR, s.rowptr, s.col, s.val, s.b, tol=0.0, maxit=first + (cap - 1) * STEP_STRIDE,
                           x_stride=STEP_STRIDE, x_cap=cap, x_first=first)
    print(f"[ref] trajectory to step {info['iters']}", flush=True)
    steps = [first + j * STEP_STRIDE for j in range(cap)]
    X = h["x"]
    xk = X[steps.index(k)]   # x after step k: the stopped run's solution, bit for bit
    nx = np.linalg.norm(xk)
    return steps, [float(np.linalg.norm(X[j] - xk) / nx) for j in range(cap)], sha(xk)


def _job(args):
    return _trajectory(args[1]) if args[0] == "trajectory" else _solve(args)


def main(name, tol=1e-10, maxit=200000):
    oracle.load()  # before the workers fork: parent and workers use one library
    t0 = time.time()
    s = W.fem_config(name, keep_geometry=False)
    _SYS["s"] = s
    print(f"[ref] generated {name}: n={s.n} nnz={s.nnz} in {time.time() - t0:.1f}s", flush=True)
    # the stop of the exact run is known when a reference of the same system
    # exists (then the trajectory runs beside the four solves), else found first
    path = os.path.join(HERE, f"{name}_oracle_csr.json")
    k_known = None
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("b_sha256") == sha(s.b) and old.get("tol") == tol:
            k_known = int(old["iters"])
    jobs = [("exact", tol, maxit), ("plain", tol, maxit), ("pairwise", tol, maxit), ("fused", tol, maxit)]
    if k_known is not None:
        jobs.append(("trajectory", k_known))
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(_job, jobs)
    (x, info), (xp, infop), (xw, infow), (xf, inff) = res[:4]
    if k_known is None or k_known != info["iters"]:
        steps, dist2, xk_sha = _trajectory(int(info["iters"]))
    else:
        steps, dist2, xk_sha = res[4]
    assert xk_sha == sha(x), "the trajectory run does not pass through the stopped run's solution"
    step_table = dict(iters=steps, dist2=dist2)
    arrs = (s.rowptr, s.col, s.val)

    def a_norm(v):
        return float(np.sqrt(oracle.dot(v, oracle.spmv(oracle.FMT_CSR, *arrs, v))))

    d = x - s.x_true

    def alt(xa, ia):
        da = xa - x
        return dict(iters=int(ia["iters"]), status=int(ia["status"]), relres_true=ia["relres_true"],
                    spread2=float(np.linalg.norm(da) / np.linalg.norm(x)), spreadA=a_norm(da) / a_norm(x))
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
        plain_dots=alt(xp, infop), pairwise_dots=alt(xw, infow), fused_dots=alt(xf, inff),
        step_table=step_table,
        sample_pos=[int(i) for i in pos], sample_x=[float(x[i]).hex() for i in pos],
        made_by="python tests/golden/make_oracle_reference.py " + name,
    )
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
    os.replace(tmp, path)
    print(f"[ref] wrote {path} in {time.time() - t0:.0f}s: iters={out['iters']} "
          f"err2={out['err2_vs_true']:.3e} errA={out['errA_vs_true']:.3e} "
          f"plain: spread2={out['plain_dots']['spread2']:.3e} spreadA={out['plain_dots']['spreadA']:.3e}; "
          f"pairwise: spread2={out['pairwise_dots']['spread2']:.3e} spreadA={out['pairwise_dots']['spreadA']:.3e}; "
          f"fused: spread2={out['fused_dots']['spread2']:.3e} spreadA={out['fused_dots']['spreadA']:.3e}; "
          f"steps {steps[0]}..{steps[-1]}: max dist2 {max(step_table['dist2']):.3e}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["fem160"]:
        main(nm)

"""Write the stored FP64 oracle gradient of the 100^3 adjoint case (test fixture).

The case: the 100^3 FEM mesh (6 181 806 tetrahedra), one reluctivity per
element nu_e = (its cell's coefficient) x U(0.8, 1.25) (seed 101), the loss
L = ||x - x_obs||^2 with the generator's x_obs, A(nu) x = b.  The oracle
(oracle/fem.py over the serial oracle CG at tol 1e-12) takes the forward
solve, the adjoint solve A lam = 2 (x - x_obs) and dL/dnu_e = -lam_e' K_e x_e;
two serial 1.0M-row solves of ~9000 iterations are too slow for a test run,
so this script runs them once and stores in ``fem100_adjoint_oracle.json``:

* L, the iteration counts, ||g||_2 of the full gradient, sum_e nu_e g_e and
  -2 (x - x_obs)' x (the homogeneity identity), sha256 of x and of g;
* g at 4096 seeded element positions, as exact hexadecimal floats.

Only the oracle and the seeded input generator are called.
Usage:  python tests/golden/make_adjoint_reference.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import fem as OF  # noqa: E402
from paper_1010_4639_amd import workload as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 4096
TOL = 1e-12


def sample_elements(m):
    """The seeded element positions at which g is stored (also used by the test)."""
    seed = int.from_bytes(hashlib.sha256(b"fem100-adjoint").digest()[:4], "little")
    return np.sort(np.random.default_rng(seed).choice(m, size=min(NSAMPLE, m), replace=False))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def element_matrices(coords, tets, chunk=1 << 20):
    out = np.empty((tets.shape[0], 4, 4))
    for i in range(0, tets.shape[0], chunk):
        out[i:i + chunk] = OF.element_matrices(coords, tets[i:i + chunk])
    return out


def main():
    t0 = time.time()
    s = W.fem_config("fem100")
    coords, tets, dof, nu_cell = W.fem_mesh(s)
    nu = nu_cell * np.random.default_rng(101).uniform(0.8, 1.25, size=nu_cell.size)
    xo = W.observation(s)
    K = element_matrices(coords, tets)
    print(f"[adj] mesh and element matrices in {time.time() - t0:.0f}s", flush=True)
    os.environ["ORC_PROGRESS"] = "2000"
    ref = OF.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, tol=TOL)
    g, x = ref["g_nu"], ref["x"]
    pos = sample_elements(g.size)
    out = dict(
        workload="fem100 adjoint: nu_e = cell coefficient x U(0.8, 1.25) (seed 101), L = ||x - x_obs||^2",
        tol=TOL, n=int(s.n), elements=int(g.size), L=ref["L"],
        iters_forward=int(ref["info"][0]["iters"]), iters_adjoint=int(ref["info"][1]["iters"]),
        relres_true_forward=ref["info"][0]["relres_true"], relres_true_adjoint=ref["info"][1]["relres_true"],
        norm2_g=float(np.linalg.norm(g)), identity_lhs=float(nu @ g), identity_rhs=float(-2.0 * ((x - xo) @ x)),
        x_sha256=sha(x), g_sha256=sha(g), b_sha256=sha(s.b),
        sample_elem=[int(i) for i in pos], sample_g=[float(g[i]).hex() for i in pos],
        made_by="python tests/golden/make_adjoint_reference.py",
    )
    path = os.path.join(HERE, "fem100_adjoint_oracle.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print(f"[adj] wrote {path} in {time.time() - t0:.0f}s: L={out['L']:.6e} iters {out['iters_forward']} / "
          f"{out['iters_adjoint']} ||g|| {out['norm2_g']:.6e}", flush=True)


if __name__ == "__main__":
    main()

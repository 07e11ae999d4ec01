"""Solution-parity yardstick for the CG tests, and the record of measured values.

CG on an ill-conditioned system stops ~kappa * tol away from the exact
solution, so where it stops depends on rounding: two valid FP64 evaluations
of the same iteration do not land on the same x.  The yardstick is the
oracle's own spread -- its iteration with exactly rounded scalar products
(the reference) against the same iteration with the plain left-to-right
products (the paper leaves the summation order to a library routine): both
are correct FP64 runs of the algorithm.  The GPU's solution must lie within

    ||x_gpu - x_oracle||_2 / ||x_oracle||_2  <=  max(1e-8, 10 * spread_2)

and, in the norm CG minimises, ||x_gpu - x_oracle||_A / ||x_oracle||_A <= 1e-8.
On well-conditioned systems the spread is far below 1e-8 and the bar is the
plain 1e-8.  Every measured value is printed and, when CGMI_PARITY_RECORD
names a file, appended to it as one JSON line.
"""
import hashlib
import json
import os

import numpy as np

import oracle

X_TOL = 1e-8          # relative solution difference at tol 1e-10 (2-norm floor, energy norm)
SPREAD_FACTOR = 10.0  # allowed multiple of the oracle's own reduction-order spread

_SPREAD = {}


def _key(b, n):
    return hashlib.sha1(np.ascontiguousarray(b).tobytes()).hexdigest() + f":{n}"


def a_norm(fmt, arrs, v):
    return float(np.sqrt(oracle.dot(v, oracle.spmv(fmt, *arrs, v))))


def oracle_spread(fmt, arrs, b, x_ref, tol=1e-10, x0=None, maxit=200000):
    """Relative 2-norm and energy-norm distance between the oracle's solution
    x_ref (exact scalar products) and the oracle run with plain products."""
    n = len(arrs[0]) - 1
    k = _key(b, n) + ("" if x0 is None else _key(x0, n)) + f":{tol}"
    if k not in _SPREAD:
        xp, info, _ = oracle.cg(fmt, *arrs, b, x0=x0, tol=tol, maxit=maxit, plain_dots=True)
        d = xp - x_ref
        _SPREAD[k] = (float(np.linalg.norm(d) / np.linalg.norm(x_ref)),
                      a_norm(fmt, arrs, d) / a_norm(fmt, arrs, x_ref), info["iters"])
    return _SPREAD[k]


def x_bar(spread2):
    return max(X_TOL, SPREAD_FACTOR * spread2)


def record(**kw):
    path = os.environ.get("CGMI_PARITY_RECORD")
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps({k: (float(v) if isinstance(v, np.floating) else v) for k, v in kw.items()}) + "\n")


def load_reference(name):
    """Stored oracle reference of a large system (tests/golden/make_oracle_reference.py)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_oracle_csr.json")
    with open(path) as f:
        ref = json.load(f)
    ref["sample_x"] = np.array([float.fromhex(h) for h in ref["sample_x"]])
    ref["sample_pos"] = np.array(ref["sample_pos"], dtype=np.int64)
    return ref


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()

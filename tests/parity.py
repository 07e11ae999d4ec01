"""Solution-parity yardstick for the CG tests, and the record of measured values.

CG on an ill-conditioned system stops ~kappa * tol away from the exact
solution, so where it stops depends on rounding: two valid FP64 evaluations
of the same iteration do not land on the same x.  The 2-norm yardstick is
the oracle's own spread, the larger of two distances:

* evaluation spread -- its iteration with exactly rounded scalar products
  (the reference) against the same iteration with plain left-to-right,
  pairwise-summed, or fused multiply-add arithmetic (the paper leaves the
  scalar products and vector updates to a library routine): all are
  correct FP64 runs of the algorithm;
* stopping-step spread -- the oracle's own iterate after as many iterations
  as the GPU needed, against its solution.  CG's residual is not monotone:
  near the tolerance it can dip below it, rise and fall again, while x keeps
  moving (its energy-norm error falls at every step).  On a 504-row FEM
  system the oracle stops at step 301; a run whose residual at step 301 is
  a little higher stops at 311, 3.9e-8 away in the 2-norm -- where an FP64
  run with a library's blocked scalar products lands too.

The GPU's solution must lie within

    ||x_gpu - x_oracle||_2 / ||x_oracle||_2  <=  max(1e-8, 4 * spread_2)

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

ALT_DOTS = ("plain", "pairwise", "fused")  # the alternative evaluations of the iteration
X_TOL = 1e-8          # relative solution difference at tol 1e-10 (2-norm floor, energy norm)
SPREAD_FACTOR = 4.0   # allowed multiple of the oracle's own reduction-order spread

_SPREAD = {}


def _key(b, n):
    return hashlib.sha1(np.ascontiguousarray(b).tobytes()).hexdigest() + f":{n}"


def a_norm(fmt, arrs, v):
    return float(np.sqrt(oracle.dot(v, oracle.spmv(fmt, *arrs, v))))


def oracle_spread(fmt, arrs, b, x_ref, tol=1e-10, x0=None, maxit=200000):
    """Largest relative 2-norm and energy-norm distance between the oracle's
    solution x_ref (exact scalar products) and the oracle runs with the
    alternative arithmetic of ALT_DOTS; and the iteration counts of those
    runs."""
    n = len(arrs[0]) - 1
    k = _key(b, n) + ("" if x0 is None else _key(x0, n)) + f":{tol}"
    if k not in _SPREAD:
        s2 = sA = 0.0
        its = []
        for mode in ALT_DOTS:
            xp, info, _ = oracle.cg(fmt, *arrs, b, x0=x0, tol=tol, maxit=maxit, dots=mode)
            d = xp - x_ref
            s2 = max(s2, float(np.linalg.norm(d) / np.linalg.norm(x_ref)))
            sA = max(sA, a_norm(fmt, arrs, d) / a_norm(fmt, arrs, x_ref))
            its.append(info["iters"])
        _SPREAD[k] = (s2, sA, its)
    return _SPREAD[k]


def step_spread(fmt, arrs, b, x_ref, k_ref, k_other, x0=None):
    """Relative 2-norm distance between the oracle's iterate after k_other
    iterations (no stopping test) and its solution x_ref after k_ref: the
    same bits up to step min(k_ref, k_other)."""
    if k_other == k_ref or k_other <= 0:
        return 0.0
    n = len(arrs[0]) - 1
    k = _key(b, n) + ("" if x0 is None else _key(x0, n)) + f":step{k_other}"
    if k not in _SPREAD:
        xk, _, _ = oracle.cg(fmt, *arrs, b, x0=x0, tol=0.0, maxit=k_other)
        _SPREAD[k] = float(np.linalg.norm(xk - x_ref) / np.linalg.norm(x_ref))
    return _SPREAD[k]


def stored_step_spread(ref, k_other):
    """Stopping-step spread from a stored reference's table of
    ||x_oracle(j) - x_oracle|| / ||x_oracle|| (every `step_stride` iterations
    around its stop): the larger of the two tabulated steps around k_other;
    None if k_other lies outside the table."""
    tab = ref.get("step_table")
    if not tab:
        return None
    js = np.array(tab["iters"])
    ds = np.array(tab["dist2"])
    if k_other == ref["iters"]:
        return 0.0
    if k_other < js[0] or k_other > js[-1]:
        return None
    lo = np.searchsorted(js, k_other, side="right") - 1
    hi = min(lo + 1, js.size - 1)
    return float(max(ds[lo], ds[hi]))


def stored_spread(ref):
    """The spread of a stored reference (tests/golden/make_oracle_reference.py):
    the larger distance over its alternative evaluations."""
    alts = [ref[k] for k in ("plain_dots", "pairwise_dots", "fused_dots") if k in ref]
    return (max(a["spread2"] for a in alts), max(a["spreadA"] for a in alts), [a["iters"] for a in alts])


def x_bar(spread2, step2=0.0):
    return max(X_TOL, SPREAD_FACTOR * max(spread2, step2))


def record(**kw):
    path = os.environ.get("CGMI_PARITY_RECORD")
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps({k: (v.item() if isinstance(v, np.generic) else v) for k, v in kw.items()}) + "\n")


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


FMT_NAMES = {0: "CSR", 1: "symmetric CSR", 2: "CSC"}


def records_markdown(path):
    """The parity records of one GPU test run (CGMI_PARITY_RECORD) as
    markdown tables: FP64 CG against the oracle, the full-size solves against
    the stored oracle run, mixed precision, and a summary of the batched
    pairs."""
    rows = [json.loads(line) for line in open(path)]
    fmt = lambda v: "–" if v is None else (f"{v:.3g}" if isinstance(v, float) else str(v))
    out = ["| case | format | iters GPU / oracle | 2-norm diff | bar | energy-norm diff | true relres |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        if "err2" in r and "bar2" in r and not r["test"].startswith(("batch", "mixed")):
            out.append(f"| {r['test']} | {FMT_NAMES.get(r['fmt'], r['fmt'])} | {r.get('iters')} / "
                       f"{r.get('oracle_iters')} | {fmt(r['err2'])} | {fmt(r['bar2'])} | {fmt(r.get('errA'))} | "
                       f"{fmt(r.get('relres_true'))} |")
    out += ["", "Full-size solves against the stored serial oracle run (4096 sampled entries; errors against "
            "x_true over all entries):", "",
            "| case | sampled 2-norm diff | bar | energy-norm error vs x_true (oracle) | 2-norm error vs x_true "
            "(oracle) | iters GPU / oracle |", "|---|---|---|---|---|---|"]
    for r in rows:
        if "err2_sampled" in r:
            bar = "not asserted (mixed)" if "mixed" in r["test"] else fmt(r["bar2"])
            out.append(f"| {r['test']} | {fmt(r['err2_sampled'])} | {bar} | {fmt(r['errA_vs_true'])} "
                       f"({fmt(r['oracle_errA_vs_true'])}) | {fmt(r['err2_vs_true'])} ({fmt(r['oracle_err2_vs_true'])}) "
                       f"| {fmt(r.get('iters'))} / {fmt(r.get('oracle_iters'))} |")
    out += ["", "Mixed precision (refinement stops on the true residual; energy-norm difference to the FP64 "
            "oracle, 2-norm errors against x_true):", "",
            "| case | format | energy-norm diff | 2-norm diff | 2-norm error vs x_true (oracle's) | inner / outer |",
            "|---|---|---|---|---|---|"]
    for r in rows:
        if r["test"].startswith("mixed") and "errA" in r:
            out.append(f"| {r['test']} | {FMT_NAMES.get(r['fmt'], r['fmt'])} | {fmt(r['errA'])} | {fmt(r['err2'])} | "
                       f"{fmt(r['err2_vs_true'])} ({fmt(r['oracle_err2_vs_true'])}) | {r.get('inner_iters')} / "
                       f"{r.get('outer')} |")
    batch = [r for r in rows if r["test"].startswith("batch")]
    if batch:
        worst = max(batch, key=lambda r: r.get("err2", 0.0) / max(r.get("bar2", 1.0), 1e-300))
        out += ["", f"Batched: {len(batch)} (system, right-hand side) pairs against single oracle solves; worst "
                f"2-norm diff / bar: {fmt(worst.get('err2'))} / {fmt(worst.get('bar2'))} ({worst['test']}); "
                f"largest energy-norm diff {fmt(max(r.get('errA', 0.0) for r in batch))}."]
    return "\n".join(out)


if __name__ == "__main__":
    import sys
    print(records_markdown(sys.argv[1]))

"""Solve a system stored in files, as the paper's program does (section III:
the matrix in full or symmetric CSR form, with b and x).

    python -m paper_1010_4639_amd.solve_file A.mtx [--rhs b.mtx] [--x0 x0.mtx]
        [--storage csr|symcsr|csc|paper] [--tol 1e-10] [--maxit N] [--out x.mtx]

A.mtx: Matrix Market coordinate file (a "symmetric" file stores one triangle,
1-based, like the paper's arrays).  --storage chooses what is handed to the
GPU library: the full matrix by rows or by columns, the upper triangle, or
the paper's own layout (lower triangle L + D by rows, 1-based, read through
CG_LOWER).  Without --rhs, b = A * ones (formed on the GPU by the library's
own product).  Prints one JSON line: iterations, status, true residual, time.
"""
import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("matrix")
    ap.add_argument("--rhs")
    ap.add_argument("--x0")
    ap.add_argument("--storage", default="paper", choices=["csr", "symcsr", "csc", "paper"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=None)
    ap.add_argument("--out")
    a = ap.parse_args(argv)
    import numpy as np
    import torch

    from paper_1010_4639_amd import cgmi, mmio

    M = mmio.read_matrix(a.matrix)
    if a.storage == "paper":
        ptr, idx, val = M.lower_one_based()
        S = cgmi.Solver("symcsr", ptr, idx, val, index_base=1, flags=cgmi.CG_LOWER)
    elif a.storage == "symcsr":
        S = cgmi.Solver("symcsr", *M.upper())
    else:
        S = cgmi.Solver(a.storage, *(M.csc() if a.storage == "csc" else M.csr()))
    dev = torch.device("cuda:0")
    with S:
        if a.rhs:
            b = torch.from_numpy(np.ascontiguousarray(mmio.read_vector(a.rhs), dtype=np.float64)).to(dev)
        else:
            b = S.spmv(torch.ones(M.n, dtype=torch.float64, device=dev))
        x0 = torch.from_numpy(mmio.read_vector(a.x0)).to(dev) if a.x0 else None
        x, info = S.solve(b, x0, tol=a.tol, maxit=a.maxit if a.maxit is not None else max(10 * M.n, 1))
    out = dict(matrix=a.matrix, n=M.n, stored_entries=int(M.vals.size), symmetric_file=M.symmetric,
               storage=a.storage, **{k: info[k] for k in ("iters", "status", "relres", "relres_true", "ms")},
               status_text=cgmi.cg_status_string(info["status"]))
    if a.out:
        mmio.write_vector(a.out, x.cpu().numpy())
    print(json.dumps(out), flush=True)
    return 0 if info["status"] == cgmi.CG_OK else 1


if __name__ == "__main__":
    sys.exit(main())

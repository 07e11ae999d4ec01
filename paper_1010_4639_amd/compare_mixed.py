"""Time-to-tolerance of FP64 CG vs mixed-precision refinement on one system.

    python -m paper_1010_4639_amd.compare_mixed [--workload fem160] [--formats csr]
        [--tol 1e-10] [--inner-tol 1e-2] [--reps 2]

For each format: the FP64 solve (cg_solve) and the mixed solve
(cg_solve_mixed: FP32 product and search directions inside FP64 iterative
refinement), both from x0 = 0 to ||b - A x|| <= tol ||b||, timed on the
device with the host blocking on the result (median of `reps` after one
warm-up).  The mixed solve works on D^-1/2 A D^-1/2; a third arm, "fp64_scaled",
runs the FP64 cg_solve on that same scaled system (scaled on the host as
input data, x = D^-1/2 y) so that the gain of the scaling and the gain of FP32
storage are reported apart.  Prints one JSON line with the times, iteration
counts, true residuals and the relative 2-norm differences of the solutions.
"""
import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="fem160")
    ap.add_argument("--formats", default="csr")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=1e-2)
    ap.add_argument("--maxit", type=int, default=200000)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cpu-iters", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args(argv)
    import statistics
    import time

    import numpy as np
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W

    dev = torch.device("cuda:0")
    t0 = time.time()
    s = W.fem_config(a.workload, keep_geometry=False)
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    arrs = {"csr": (s.rowptr, s.col, s.val), "symcsr": (up, uc, uv), "csc": (s.rowptr, s.col, s.val)}
    print(f"[mixed] generated {a.workload} n={s.n} nnz={s.nnz} in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    b = torch.from_numpy(s.b).to(dev)
    out = {"workload": a.workload, "n": s.n, "nnz": s.nnz, "tol": a.tol, "inner_tol": a.inner_tol}
    for name in a.formats.split(","):
        with cgmi.Solver(name, *arrs[name], mixed=True) as S:
            res = {}
            for mode in ("fp64", "mixed"):
                times, info, x = [], None, None
                for r in range(a.reps + 1):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    if mode == "fp64":
                        x, info = S.solve(b, tol=a.tol, maxit=a.maxit)
                    else:
                        x, info = S.solve_mixed(b, tol=a.tol, maxit=a.maxit, inner_tol=a.inner_tol,
                                                max_outer=100)
                    torch.cuda.synchronize()
                    if r > 0:
                        times.append((time.perf_counter() - t1) * 1e3)
                    print(f"[mixed] {name} {mode} rep {r}: {info}", file=sys.stderr, flush=True)
                res[mode] = dict(ms=round(statistics.median(times), 3), iters=info["iters"],
                                 outer=info.get("outer", 0), status=info["status"],
                                 relres_true=info["relres_true"], x=x)
            # FP64 CG on the Jacobi-scaled system (same scaling as the mixed inner solve)
            p_, i_, v_ = arrs[name]
            line = np.repeat(np.arange(s.n), np.diff(p_))
            dg = np.zeros(s.n)
            dpos = line == i_
            dg[line[dpos]] = v_[dpos]
            sc = 1.0 / np.sqrt(dg)
            sct = torch.from_numpy(sc).to(dev)
            with cgmi.Solver(name, p_, i_, v_ * sc[line] * sc[i_]) as S2:
                bs = sct * b
                times = []
                for r in range(a.reps + 1):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    y, info = S2.solve(bs, tol=a.tol, maxit=a.maxit)
                    torch.cuda.synchronize()
                    if r > 0:
                        times.append((time.perf_counter() - t1) * 1e3)
                xs_ = sct * y
                # true residual of the unscaled system, through the FP64 product of S
                rt = float(torch.linalg.norm(b - S.spmv(xs_)) / torch.linalg.norm(b))
                res["fp64_scaled"] = dict(ms=round(statistics.median(times), 3), iters=info["iters"],
                                          status=info["status"], relres_true=rt, x=xs_)
            xd, xm = res["fp64"].pop("x"), res["mixed"].pop("x")
            xsc = res["fp64_scaled"].pop("x")
            res["rel_diff_2norm"] = float(torch.linalg.norm(xd - xm) / torch.linalg.norm(xd))
            xt = torch.from_numpy(s.x_true).to(dev)
            res["fp64"]["err_vs_x_true"] = float(torch.linalg.norm(xd - xt) / torch.linalg.norm(xt))
            res["mixed"]["err_vs_x_true"] = float(torch.linalg.norm(xm - xt) / torch.linalg.norm(xt))
            res["fp64_scaled"]["err_vs_x_true"] = float(torch.linalg.norm(xsc - xt) / torch.linalg.norm(xt))
            res["speedup"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
            res["speedup_vs_scaled_fp64"] = round(res["fp64_scaled"]["ms"] / res["mixed"]["ms"], 3)
            out[name] = res
    if not a.no_cpu:
        # the oracle beside it: serial C CG per iteration on the same system
        # (a bounded sample), scaled by the FP64 iteration count
        import oracle
        name = a.formats.split(",")[0]
        _, oi, _ = oracle.cg(cgmi.FORMATS[name], *arrs[name], s.b, tol=0.0, maxit=a.cpu_iters)
        ms_it = oi["ms_loop"] / max(oi["iters"], 1)
        out["cpu_baseline"] = dict(kind="oracle", cores=1, unit="ms",
                                   value=round(ms_it * out[name]["fp64"]["iters"], 1),
                                   sample=f"{oi['iters']} oracle CG iterations in {name} at {ms_it:.2f} ms each, "
                                          f"scaled by the FP64 GPU iteration count")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

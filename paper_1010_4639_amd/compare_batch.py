"""Batched solve vs a loop of single solves on the same systems.

    python -m paper_1010_4639_amd.compare_batch [--nsys 256] [--nrhs 4]
        [--lo 20] [--hi 60] [--workers 16] [--loop-systems 32]

Builds `nsys` FEM systems with interior grid edges drawn per axis from
U{lo..hi} (seed 4), each with `nrhs` right-hand sides, and times:
  * one cg_batch_solve over all (system, right-hand side) pairs, after the
    project's autotuner has chosen row-block size and workgroup budget;
  * cg_solve for each pair in turn (one handle per system).  With
    --loop-systems k < nsys only the first k systems are looped and the time
    is scaled by (total nnz) / (looped nnz), as stated in the output.
Both to ||r|| <= 1e-10 ||b|| from x0 = 0.  Prints one JSON line.
"""
import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsys", type=int, default=256)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--lo", type=int, default=20)
    ap.add_argument("--hi", type=int, default=60)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--loop-systems", type=int, default=32)
    ap.add_argument("--cpu-systems", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args(argv)
    import numpy as np
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W

    dev = torch.device("cuda:0")
    t0 = time.time()
    systems, B, _ = W.fem_batch(a.nsys, lo=a.lo, hi=a.hi, nrhs=a.nrhs, workers=a.workers)
    so, ptr, col, val = W.block_diagonal(systems)
    print(f"[batch] {a.nsys} systems, N={so[-1]}, nnz={ptr[-1]} generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    Bd = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    out = {"nsys": a.nsys, "nrhs": a.nrhs, "N": int(so[-1]), "nnz": int(ptr[-1]), "tol": a.tol}
    with cgmi.Batch(so, ptr, col, val, nrhs=a.nrhs) as bt:
        tuned = bt.autotune()
        print(f"[batch] autotune: {tuned}", file=sys.stderr, flush=True)
        bt.solve(Bd, tol=a.tol)                               # warm-up (graph build)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, info, iters, st = bt.solve(Bd, tol=a.tol)
        torch.cuda.synchronize()
        out["batched_ms"] = round((time.perf_counter() - t1) * 1e3, 3)
        out["batched_status_ok"] = int((st == 0).sum())
        out["batched_max_iters"] = int(iters.max())
        out["autotune"] = tuned
    k = min(a.loop_systems, a.nsys)
    loop_ms, loop_nnz = 0.0, 0
    for s in range(k):
        rp, c, v = systems[s]
        with cgmi.Solver("csr", rp, c, v) as S:
            r0, r1 = so[s], so[s + 1]
            for r in range(a.nrhs):
                b = Bd[r0:r1, r].contiguous()
                if s == 0 and r == 0:
                    S.solve(b, tol=a.tol)                      # warm-up (graph build)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                S.solve(b, tol=a.tol)
                torch.cuda.synchronize()
                loop_ms += (time.perf_counter() - t1) * 1e3
        loop_nnz += int(rp[-1])
    out["loop_systems_timed"] = k
    out["loop_ms_timed"] = round(loop_ms, 3)
    out["loop_ms_scaled"] = round(loop_ms * int(ptr[-1]) / loop_nnz, 3)
    out["speedup_vs_loop"] = round(out["loop_ms_scaled"] / out["batched_ms"], 3)
    if not a.no_cpu:
        # the oracle beside it: serial C CG on the first looped systems (every
        # right-hand side, to the same tolerance), scaled by nnz like the loop
        import oracle
        t_ms, o_nnz = 0.0, 0
        for s in range(min(a.cpu_systems, a.nsys)):
            rp, c, v = systems[s]
            r0, r1 = so[s], so[s + 1]
            for r in range(a.nrhs):
                _, oi, _ = oracle.cg(0, rp, c, v, np.ascontiguousarray(B[r0:r1, r]), tol=a.tol, maxit=50000)
                t_ms += oi["ms_loop"]
            o_nnz += int(rp[-1])
        out["cpu_baseline"] = dict(kind="oracle", cores=1, unit="ms", value=round(t_ms * int(ptr[-1]) / o_nnz, 1),
                                   sample=f"oracle CG on {min(a.cpu_systems, a.nsys)} systems x {a.nrhs} right-hand "
                                          f"sides ({t_ms:.0f} ms), scaled by total nnz / sampled nnz")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

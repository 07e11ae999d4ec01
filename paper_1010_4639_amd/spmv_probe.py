"""SpMV micro-benchmark: y = A x through the C-ABI for each storage format.

    python -m paper_1010_4639_amd.spmv_probe [--workload fem100] [--reps 20]
        [--formats csr,symcsr,csc] [--copy-gib 1]

Runs `reps` back-to-back products per format (timed with HIP events on the
launch stream) and one plain device-to-device copy of `copy-gib` GiB (the
known-size transfer used to calibrate hardware byte counters).  Short enough
to run under a counter-collecting profiler.
"""
import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="fem100")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--formats", default="csr,symcsr,csc")
    ap.add_argument("--copy-gib", type=float, default=1.0)
    a = ap.parse_args(argv)
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W

    dev = torch.device("cuda:0")
    s = W.fem_config(a.workload, with_rhs=False, keep_geometry=False)
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    arrs = {"csr": ((s.rowptr, s.col, s.val), s.nnz), "symcsr": ((up, uc, uv), len(uc)),
            "csc": ((s.rowptr, s.col, s.val), s.nnz)}
    x = torch.from_numpy(W.uniform_vector(s.n, seed=5)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    out = {"workload": a.workload, "n": s.n}
    for name in a.formats.split(","):
        (ptr, idx, val), nnz = arrs[name]
        with cgmi.Solver(name, ptr, idx, val) as S:
            S.spmv(x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(a.reps):
                S.spmv(x, y)
            e1.record(stream)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / a.reps
            byts = 12 * nnz + 4 * (s.n + 1) + 16 * s.n
            out[name] = dict(us=round(us, 3), bytes=byts, GBps=round(byts / us / 1e3, 1), stats=S.stats())
            print(f"[probe] {name}: {us:.1f} us, {byts / us / 1e3:.0f} GB/s", file=sys.stderr, flush=True)
    if a.copy_gib > 0:
        nel = int(a.copy_gib * (1 << 30)) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_bytes_each_way"] = nel * 8
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

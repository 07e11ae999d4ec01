#!/usr/bin/env python3
"""Benchmark: CG time-to-1e-10 residual and SpMV bandwidth on one MI355X.

Workload (default fem100): the synthetic P1 / Kuhn-tet stiffness matrix of a
100^3 interior grid (n = 1 000 000, nnz = 14 761 198, iron contrast 1e-3),
b = A x_true, x0 = 0, tol 1e-10 relative to ||b||.  One step solves that
system three times, with A stored as full CSR, as symmetric CSR (upper
triangle) and as CSC, i.e. one pass of every product variant and of the
fused CG vector kernels.  Inputs are resident in HBM before timing starts.

Printed: one JSON line (metric = time-to-solution of the step, lower is
better) with the per-format breakdown, a roofline entry for the dominant
kernel (algorithmic bytes / average launch time, timed live with HIP events
on the launch stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, AMD public figure
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fem100.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1010_4639_amd", "csrc", "kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fem100")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=50000)
    ap.add_argument("--batch", type=int, default=None, help="CG iterations per graph launch")
    ap.add_argument("--spmv-reps", type=int, default=100)
    ap.add_argument("--cpu-iters", type=int, default=120, help="oracle CG iterations per format (cpu_baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def spmv_bytes(fmt, n, nnz_stored):
    """Algorithmic bytes of one product: idx + val per stored entry, ptr, x and y."""
    return 12 * nnz_stored + 4 * (n + 1) + 16 * n


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(kind):
    """HBM bytes per launch from the committed counter runs, or None if the
    kernels changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != kernel_source_sha():
        return None
    return t.get("per_launch_bytes", {}).get(kind)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cgmi.load()
    dev = torch.device("cuda:0")
    t0 = time.time()
    s = W.fem_config(args.workload)
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    log(f"[bench] generated {args.workload}: n={s.n} nnz={s.nnz} nnz_upper={len(uc)} in {time.time() - t0:.1f}s")
    formats = {
        "csr": (cgmi.CG_FMT_CSR, (s.rowptr, s.col, s.val), s.nnz),
        "symcsr": (cgmi.CG_FMT_SYM_CSR, (up, uc, uv), len(uc)),
        "csc": (cgmi.CG_FMT_CSC, (s.rowptr, s.col, s.val), s.nnz),
    }
    solvers = {}
    for name, (fmt, arrs, _) in formats.items():
        t1 = time.time()
        solvers[name] = cgmi.Solver(fmt, *arrs, batch=args.batch)
        log(f"[bench] created {name} handle in {time.time() - t1:.1f}s: {solvers[name].stats()}")
    b = torch.from_numpy(s.b).to(dev)
    x0 = torch.zeros_like(b)

    def step():
        out = {}
        for name, S in solvers.items():
            x, info = S.solve(b, x0, tol=args.tol, maxit=args.maxit)
            if info["status"] != cgmi.CG_OK:
                raise RuntimeError(f"{name}: solve failed {info}")
            out[name] = info
        return out

    for w in range(args.warmup):
        info = step()
        log(f"[bench] warmup {w}: " + ", ".join(f"{k} {v['iters']} it {v['ms']:.1f} ms" for k, v in info.items()))
    torch.cuda.synchronize()
    per = {k: [] for k in solvers}
    t_start = time.perf_counter()
    for k in range(args.steps):
        info = step()
        for name, v in info.items():
            per[name].append(v)
        log(f"[bench] step {k}: " + ", ".join(f"{n} {v['iters']} it {v['ms']:.1f} ms" for n, v in info.items()))
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1e3 / args.steps

    # SpMV: average launch duration with HIP events on the launch stream
    stream = torch.cuda.current_stream()
    xs = torch.from_numpy(W.uniform_vector(s.n, seed=99)).to(dev)
    ys = torch.empty_like(xs)
    spmv = {}
    for name, S in solvers.items():
        for _ in range(10):
            S.spmv(xs, ys)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.spmv_reps):
            S.spmv(xs, ys)
        e1.record(stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / args.spmv_reps
        byts = spmv_bytes(name, s.n, formats[name][2])
        spmv[name] = dict(us=us, bytes=byts, GBps=byts / us / 1e3, colors=S.stats()["colors"])
        log(f"[bench] spmv {name}: {us:.1f} us/launch, {byts / 1e6:.1f} MB algorithmic, "
            f"{byts / us / 1e3:.0f} GB/s")
    # cold products: a 1 GiB read evicts the matrix from the caches (L2, and
    # the 256 MB Infinity Cache) before each single timed launch, leaving
    # clean lines behind (a write would leave dirty ones to be written back
    # during the timed launch); median of 5
    scratch = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    flushed = torch.empty(1, dtype=torch.float64, device=dev)
    torch.sum(scratch, dim=0, keepdim=True, out=flushed)
    for name, S in solvers.items():
        cold = []
        for i in range(5):
            torch.sum(scratch, dim=0, keepdim=True, out=flushed)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            S.spmv(xs, ys)
            e1.record(stream)
            e1.synchronize()
            cold.append(e0.elapsed_time(e1) * 1e3)
        spmv[name]["cold_us"] = float(np.median(cold))
        log(f"[bench] spmv {name} cold: {spmv[name]['cold_us']:.1f} us/launch, "
            f"{spmv[name]['bytes'] / spmv[name]['cold_us'] / 1e3:.0f} GB/s")
    del scratch, flushed
    # plain device copy of 1 GiB for the practical bandwidth ceiling
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        c.copy_(a)
    e1.record(stream)
    e1.synchronize()
    copy_gbps = 2 * a.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, c

    per_format = {}
    for name in solvers:
        its = [v["iters"] for v in per[name]]
        ms = float(np.mean([v["ms"] for v in per[name]]))
        per_format[name] = dict(time_to_tol_ms=round(ms, 3), iters=its[-1], us_per_iter=round(1e3 * ms / its[-1], 3),
                                relres_true=per[name][-1]["relres_true"],
                                spmv_us=round(spmv[name]["us"], 3), spmv_GBps=round(spmv[name]["GBps"], 1),
                                spmv_cold_us=round(spmv[name]["cold_us"], 3),
                                spmv_cold_GBps=round(spmv[name]["bytes"] / spmv[name]["cold_us"] / 1e3, 1),
                                spmv_colors=spmv[name]["colors"],
                                sliced=solvers[name].stats()["slices"] == 1,
                                matrix_cache_resident=solvers[name].stats()["cached_loads"] == 1)
    # dominant product kernel: largest share of the step's time
    dom = max(solvers, key=lambda k: spmv[k]["us"] * per_format[k]["iters"])
    sliced = solvers[dom].stats()["slices"] == 1
    kernel_name = {"csr": "k_spmv_slices (CSR product, 64-row slices)" if sliced else
                          "k_spmv_csr_rows (CSR product, row blocks)",
                   "symcsr": ("k_scatter_slices" if sliced else "k_scatter_sums") +
                             " + k_scatter_gather (symmetric-CSR product)",
                   "csc": ("k_spmv_slices" if sliced else "k_panel_rows") +
                          " + k_panel_gather (CSC product on column panels)"}[dom]
    traffic = load_traffic(dom)
    roofline = dict(bound="hbm", achieved=round(spmv[dom]["GBps"], 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(spmv[dom]["GBps"] / HBM_PEAK_GBPS, 4), traffic=traffic, kernel=kernel_name,
                    bytes_per_launch=spmv[dom]["bytes"], avg_us=round(spmv[dom]["us"], 3))

    cpu = None
    if not args.no_cpu:
        import oracle
        cpu_ms = 0.0
        sample = []
        for name, (fmt, arrs, _) in formats.items():
            _, oinfo, _ = oracle.cg(fmt, *arrs, s.b, tol=0.0, maxit=args.cpu_iters)
            ms_it = oinfo["ms_loop"] / max(oinfo["iters"], 1)
            cpu_ms += ms_it * per_format[name]["iters"]
            sample.append(f"{name}: {oinfo['iters']} it at {ms_it:.2f} ms/it")
            log(f"[bench] oracle {name}: {ms_it:.2f} ms/iteration")
        cpu = dict(value=round(cpu_ms, 1), unit="ms", cores=1, kind="oracle",
                   sample=f"{args.cpu_iters} oracle CG iterations per format on the same system (serial C, "
                          f"-O2), scaled by the GPU's iteration counts; " + "; ".join(sample))

    res = {
        "metric": "CG time-to-1e-10 residual (CSR + symmetric-CSR + CSC solves of one system)",
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: 3D P1 Kuhn-tet FEM stiffness, {s.nx}x{s.ny}x{s.nz} interior grid, "
                        f"n={s.n}, nnz={s.nnz} (upper {len(uc)}), iron box {s.iron_fraction:.3f} of cells, "
                        f"x0=0, tol={args.tol:g}, formats csr+symcsr+csc",
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_format": per_format,
        "stream_copy_GBps": round(copy_gbps, 1),
    }
    for S in solvers.values():
        S.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

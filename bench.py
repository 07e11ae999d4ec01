#!/usr/bin/env python3
"""Benchmark: CG time-to-1e-10 residual and product bandwidth on one MI355X.

Step (the timed unit): one FP64 conjugate-gradient solve, from x0 = 0 to
||b - A x|| <= 1e-10 ||b||, of the synthetic P1 / Kuhn-tet stiffness system of
a 160^3 interior grid (n = 4 096 000, nnz = 60 827 518, iron contrast 1e-4)
stored as full CSR.  The iteration is the paper's unpreconditioned CG (one
product Ap, two scalar products and three vector updates per iteration, all
on the device).  Inputs are resident in HBM before timing starts.

Printed: ONE JSON line.  Besides the step time it carries
  * roofline: the dominant kernel (the CSR product, ~75 % of the step) as
    algorithmic bytes / average launch time over back-to-back launches timed
    with HIP events on the launch stream, against the 8 TB/s HBM peak, and
    the HBM bytes one launch moves according to the committed counter runs
    (profiles/traffic_<workload>.json), while the kernel source is unchanged;
  * cpu_baseline: the CPU oracle's CSR iteration timed on every host core
    (its OpenMP timing mode; a bounded sample of iterations, median of 3,
    scaled by the GPU's iteration count) and, beside it, on one core;
  * extras, each timed on its own (--extras): the symmetric-CSR and CSC
    solves and products of the same system; mixed precision (FP32 product
    inside FP64 refinement) against plain FP64 CG and against FP64 CG on the
    same Jacobi-scaled system, in CSR and symmetric CSR; the paper-sized
    32x32x30 system in all formats; the batch of 256 uneven systems x 4
    right-hand sides solved together against a fully measured loop of the
    1024 single solves; the adjoint (gradient) solve on the 100^3 system.

Other modes (--mode): `counters` runs only the product of one format
back-to-back plus a 1 GiB device copy, for hardware-counter runs under
rocprofv3 --pmc; `parse-counters` turns two such runs (FETCH_SIZE, then
WRITE_SIZE) into profiles/traffic_<workload>.json.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, AMD public figure
KERNEL_SRC = os.path.join(ROOT, "paper_1010_4639_amd", "csrc", "kernels.hip")
# kernels of one product of each format (name prefixes as the profiler prints
# them; CSR and CSC slices differ in their first template argument)
PRODUCT_KERNELS = {"csr": ("k_spmv_slices<false", "k_spmv_csr"),
                   "symcsr": ("k_scatter_",),
                   "csc": ("k_spmv_slices<true", "k_panel_")}
EXTRAS = ("formats", "mixed", "small", "batch", "adjoint", "cpu")
T_START = time.time()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="bench", choices=("bench", "counters", "parse-counters", "summarize-trace"))
    ap.add_argument("--workload", default="fem160")
    ap.add_argument("--format", default="csr", choices=("csr", "symcsr", "csc"))
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=200000)
    ap.add_argument("--spmv-reps", type=int, default=100)
    ap.add_argument("--extras", default="all", help="comma list of " + ",".join(EXTRAS) + ", or all / none")
    ap.add_argument("--budget-s", type=float, default=300.0,
                    help="skip the remaining extras once this much wall time has passed")
    ap.add_argument("--inner-tol", type=float, default=1e-2)
    ap.add_argument("--loop-systems", type=int, default=256, help="batch extra: systems in the loop of single solves")
    ap.add_argument("--formats", default="csr,symcsr,csc", help="counters mode: formats to run")
    ap.add_argument("--counter-dirs", default="", help="parse-counters: FETCH_SIZE run dir,WRITE_SIZE run dir")
    ap.add_argument("--trace-dir", default="", help="summarize-trace: a rocprofv3 --kernel-trace --stats output dir")
    ap.add_argument("--windows", default="", help="summarize-trace: first,last kernel name prefixes of the solve "
                    "windows whose idle time to report (e.g. k_binit_vec,k_bfinish)")
    a = ap.parse_args()
    a.extras = set(EXTRAS) if a.extras == "all" else set() if a.extras == "none" else set(a.extras.split(","))
    return a


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n, nnz_stored, value_bytes=8):
    """Algorithmic bytes of one product: index + value per stored entry, the
    line pointers, x read and y written once."""
    return (4 + value_bytes) * nnz_stored + 4 * (n + 1) + (value_bytes + 8) * n


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def load_traffic(workload, fmt):
    """HBM bytes per launch from the committed counter runs, or None if the
    kernels changed since they were taken."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != kernel_source_sha():
        return None
    return t.get("per_launch_bytes", {}).get(fmt)


def host_cpu():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


class Timer:
    """HIP events on the current torch stream (the stream the library's work
    is launched on: the Solver binds its handle to it)."""

    def __init__(self, torch):
        self.torch = torch
        self.stream = torch.cuda.current_stream()

    def per_call_us(self, fn, reps, warm=5):
        for _ in range(warm):
            fn()
        e0 = self.torch.cuda.Event(enable_timing=True)
        e1 = self.torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(reps):
            fn()
        e1.record(self.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps


def timed_solve(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, out


def product_figures(torch, timer, S, xs, ys, nbytes, reps, flush):
    """Back-to-back average and cold (after evicting the caches) product time."""
    us = timer.per_call_us(lambda: S.spmv(xs, ys), reps)
    cold = []
    for _ in range(5):
        flush()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(timer.stream)
        S.spmv(xs, ys)
        e1.record(timer.stream)
        e1.synchronize()
        cold.append(e0.elapsed_time(e1) * 1e3)
    cus = statistics.median(cold)
    st = S.stats()
    out = dict(us=round(us, 3), GBps=round(nbytes / us / 1e3, 1), cold_us=round(cus, 3),
               cold_GBps=round(nbytes / cus / 1e3, 1), bytes=nbytes, colors=st["colors"],
               sliced=st["slices"] >= 1, col16=st["slices"] == 2, matrix_cache_resident=st["cached_loads"] == 1,
               plan_bytes=st["plan_bytes"], device_bytes=st["device_bytes"])
    if st["format"] == 1:
        out.update(compact_blocks=st["compact"] == 1, parked_per_row=round(st["parked"] / max(st["n"], 1), 3))
    return out


def energy_err(torch, S, x, x_true):
    """||x - x_true||_A / ||x_true||_A through the handle's FP64 product."""
    e = x - x_true
    return float(torch.sqrt((e @ S.spmv(e)) / (x_true @ S.spmv(x_true))))


# ---------------------------------------------------------------- extras
def extra_formats(torch, cgmi, W, s, a, b, timer, xs, ys, flush, res):
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    arrs = {"csr": (s.rowptr, s.col, s.val), "symcsr": (up, uc, uv), "csc": (s.rowptr, s.col, s.val)}
    out = {}
    for name in ("symcsr", "csc"):
        if name == a.format:
            continue
        t0 = time.perf_counter()
        with cgmi.Solver(name, *arrs[name]) as S:
            plan_ms = (time.perf_counter() - t0) * 1e3
            S.solve(b, tol=a.tol, maxit=a.maxit)   # graph build
            ms, (x, info) = timed_solve(torch, lambda: S.solve(b, tol=a.tol, maxit=a.maxit))
            nb = spmv_bytes(s.n, len(arrs[name][1]))
            out[name] = dict(time_to_tol_ms=round(ms, 3), iters=info["iters"],
                             us_per_iter=round(1e3 * ms / max(info["iters"], 1), 3),
                             relres_true=info["relres_true"], create_ms=round(plan_ms, 1),
                             spmv=product_figures(torch, timer, S, xs, ys, nb, a.spmv_reps, flush))
        log(f"{name}: {out[name]['iters']} it, {out[name]['time_to_tol_ms']:.1f} ms, product "
            f"{out[name]['spmv']['us']:.1f} us")
    res["formats"] = out
    return arrs


def extra_mixed(torch, cgmi, W, s, a, b, arrs, res):
    import numpy as np
    dev = b.device
    xt = torch.from_numpy(s.x_true).to(dev)
    out = {}
    for name in ("csr", "symcsr"):
        p_, i_, v_ = arrs[name]
        with cgmi.Solver(name, p_, i_, v_, mixed=True) as S:
            S.solve_mixed(b, tol=a.tol, maxit=a.maxit, inner_tol=a.inner_tol, max_outer=100)
            times, x, info = [], None, None
            for _ in range(3):
                ms, (x, info) = timed_solve(torch, lambda: S.solve_mixed(b, tol=a.tol, maxit=a.maxit,
                                                                         inner_tol=a.inner_tol, max_outer=100))
                times.append(ms)
            mixed = dict(ms=round(statistics.median(times), 3), inner_iters=info["iters"], outer=info["outer"],
                         relres_true=info["relres_true"], errA_vs_x_true=energy_err(torch, S, x, xt))
            # FP64 CG on D^-1/2 A D^-1/2 (the scaling of the mixed inner solve), x = D^-1/2 y
            line = np.repeat(np.arange(s.n), np.diff(p_))
            dg = np.zeros(s.n)
            dpos = line == i_
            dg[line[dpos]] = v_[dpos]
            sc = 1.0 / np.sqrt(dg)
            sct = torch.from_numpy(sc).to(dev)
            with cgmi.Solver(name, p_, i_, v_ * sc[line] * sc[i_]) as S2:
                bs = sct * b
                S2.solve(bs, tol=a.tol, maxit=a.maxit)
                times = []
                for _ in range(3):
                    ms, (y, info2) = timed_solve(torch, lambda: S2.solve(bs, tol=a.tol, maxit=a.maxit))
                    times.append(ms)
                xs_ = sct * y
                rt = float(torch.linalg.norm(b - S.spmv(xs_)) / torch.linalg.norm(b))
                scaled = dict(ms=round(statistics.median(times), 3), iters=info2["iters"], relres_true=rt,
                              errA_vs_x_true=energy_err(torch, S, xs_, xt))
        fp64 = (res["step"] if name == a.format else res.get("formats", {}).get(name))
        entry = dict(mixed=mixed, fp64_scaled=scaled, inner_tol=a.inner_tol,
                     speedup_vs_scaled_fp64=round(scaled["ms"] / mixed["ms"], 3))
        if fp64:
            entry["fp64_ms"] = fp64["time_to_tol_ms"]
            entry["speedup_vs_fp64"] = round(fp64["time_to_tol_ms"] / mixed["ms"], 2)
        out[name] = entry
        log(f"mixed {name}: {mixed['ms']:.1f} ms ({mixed['inner_iters']} inner, {mixed['outer']} outer), "
            f"scaled FP64 {scaled['ms']:.1f} ms ({scaled['iters']} it)")
    res["mixed"] = out


def extra_small(torch, cgmi, W, a, res):
    s = W.fem_config("fem32x32x30")
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    arrs = {"symcsr": (up, uc, uv), "csr": (s.rowptr, s.col, s.val), "csc": (s.rowptr, s.col, s.val)}
    b = torch.from_numpy(s.b).to(torch.device("cuda:0"))
    out = {"workload": "fem32x32x30: n=30720, nnz=437622 (upper 234171), iron contrast 1e-3"}
    for name, arr in arrs.items():
        with cgmi.Solver(name, *arr) as S:
            S.solve(b, tol=a.tol, maxit=a.maxit)
            times = []
            for _ in range(5):
                ms, (x, info) = timed_solve(torch, lambda: S.solve(b, tol=a.tol, maxit=a.maxit))
                times.append(ms)
            ms = statistics.median(times)
            out[name] = dict(time_to_tol_ms=round(ms, 3), iters=info["iters"],
                             us_per_iter=round(1e3 * ms / max(info["iters"], 1), 3), relres_true=info["relres_true"])
        log(f"small {name}: {out[name]['iters']} it, {ms:.2f} ms, {out[name]['us_per_iter']:.2f} us/it")
    res["small"] = out


def extra_batch(torch, cgmi, W, a, res):
    import numpy as np
    dev = torch.device("cuda:0")
    t0 = time.time()
    systems, B, _ = W.fem_batch(256, lo=20, hi=60, nrhs=4, workers=8)
    so, ptr, col, val = W.block_diagonal(systems)
    log(f"batch: 256 systems, N={so[-1]}, nnz={ptr[-1]} generated in {time.time() - t0:.1f}s")
    Bd = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    out = dict(workload="256 FEM systems, interior grid edges U{20..60} per axis (seed 4), 4 right-hand sides each",
               N=int(so[-1]), nnz=int(ptr[-1]))
    with cgmi.Batch(so, ptr, col, val, nrhs=4) as bt:
        out["autotune"] = bt.autotune()
        bt.solve(Bd, tol=a.tol)
        ms, (X, info, iters, st) = timed_solve(torch, lambda: bt.solve(Bd, tol=a.tol))
        out["batched_ms"] = round(ms, 3)
        out["batched_ok"] = int((st == 0).sum())
        out["batched_max_iters"] = int(iters.max())
    log(f"batch: one batched solve {ms:.0f} ms, autotune {out['autotune']}")
    k = min(a.loop_systems, 256)
    loop_ms, pairs, ok = 0.0, 0, 0
    for si in range(k):
        rp, c, v = systems[si]
        with cgmi.Solver("csr", rp, c, v) as S:
            r0, r1 = so[si], so[si + 1]
            for r in range(4):
                bb = Bd[r0:r1, r].contiguous()
                if si == 0 and r == 0:
                    S.solve(bb, tol=a.tol)
                ms1, (_, inf1) = timed_solve(torch, lambda: S.solve(bb, tol=a.tol))
                loop_ms += ms1
                pairs += 1
                ok += inf1["status"] == 0
    out["loop_pairs_timed"] = pairs
    out["loop_ok"] = ok
    out["loop_ms"] = round(loop_ms, 3)
    if k == 256:
        out["speedup_vs_loop"] = round(loop_ms / out["batched_ms"], 3)
    log(f"batch: loop of {pairs} single solves {loop_ms:.0f} ms")
    res["batch"] = out


def extra_adjoint(torch, cgmi, W, a, res):
    import numpy as np

    from paper_1010_4639_amd import adjoint
    dev = torch.device("cuda:0")
    t0 = time.time()
    s = W.fem_config("fem100")
    coords, tets, dof, nu_cell = W.fem_mesh(s)
    nu = nu_cell * np.random.default_rng(101).uniform(0.8, 1.25, size=nu_cell.size)
    xo = torch.from_numpy(W.observation(s)).to(dev)
    b = torch.from_numpy(s.b).to(dev)
    log(f"adjoint: fem100 mesh, {nu.size} elements, generated in {time.time() - t0:.1f}s")
    FS = adjoint.FemSolve(coords, tets, dof, s.n)
    fwd, bwd = [], []
    g = x = None
    for r in range(3):
        nu_t = torch.from_numpy(nu).to(dev).requires_grad_(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x = FS(nu_t, b, tol=a.tol)
        L = ((x - xo) ** 2).sum()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if r > 0:
            fwd.append((t2 - t1) * 1e3)
            bwd.append((t3 - t2) * 1e3)
        g = nu_t.grad
    xs = x.detach()
    lhs, rhs = float(torch.from_numpy(nu).to(dev) @ g), -2.0 * float((xs - xo) @ xs)
    res["adjoint"] = dict(workload=f"fem100: n={s.n}, {nu.size} per-element nu, L=||x-x_obs||^2, tol {a.tol:g}",
                          forward_ms=round(statistics.median(fwd), 3), backward_ms=round(statistics.median(bwd), 3),
                          identity_rel_diff=abs(lhs - rhs) / abs(rhs))
    FS.close()
    log(f"adjoint: forward {res['adjoint']['forward_ms']:.1f} ms, backward {res['adjoint']['backward_ms']:.1f} ms")


def cpu_baseline(s, fmt, gpu_iters, target_ms=6000.0):
    """The oracle's CSR iteration on every host core (OpenMP timing mode) and
    on one core, each on a bounded sample of iterations, scaled by the GPU's
    iteration count (the time to tolerance the oracle would need)."""
    import oracle
    model, ncpu, usable = host_cpu()
    arrs = (s.rowptr, s.col, s.val)
    _, probe = oracle.cg_csr_omp(*arrs, s.b, tol=0.0, maxit=10)
    per = probe["ms_loop"] / max(probe["iters"], 1)
    m = int(max(20, min(2000, target_ms / max(per, 1e-3))))
    runs = []
    for _ in range(3):
        _, oi = oracle.cg_csr_omp(*arrs, s.b, tol=0.0, maxit=m)
        runs.append(oi["ms_loop"] / max(oi["iters"], 1))
    ms_it = statistics.median(runs)
    _, ser, _ = oracle.cg(oracle.FMT_CSR, *arrs, s.b, tol=0.0, maxit=20)
    ser_it = ser["ms_loop"] / max(ser["iters"], 1)
    log(f"cpu: oracle {ms_it:.2f} ms/iteration on {probe['threads']} threads, {ser_it:.2f} on one core")
    return dict(value=round(ms_it * gpu_iters, 1), unit="ms", cores=probe["threads"], kind="oracle",
                sample=(f"oracle CSR CG, OpenMP timing mode (static loops, exactly rounded dots), {m} iterations x 3 "
                        f"runs on {probe['threads']} threads, median {ms_it:.3f} ms/iteration, scaled by the GPU's "
                        f"{gpu_iters} iterations; host: {model}, nproc {ncpu}, usable {usable}"),
                one_core=dict(value=round(ser_it * gpu_iters, 1), ms_per_iter=round(ser_it, 3),
                              sample=f"serial oracle orc_cg (the correctness reference), 20 iterations"),
                format=fmt)


# ----------------------------------------------------------------- modes
def counters_mode(a):
    """Products only, for hardware-counter runs: `reps` back-to-back launches
    of each format, then one 1 GiB device-to-device copy (calibration)."""
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W
    dev = torch.device("cuda:0")
    s = W.fem_config(a.workload, with_rhs=False, keep_geometry=False)
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    arrs = {"csr": (s.rowptr, s.col, s.val), "symcsr": (up, uc, uv), "csc": (s.rowptr, s.col, s.val)}
    x = torch.from_numpy(W.uniform_vector(s.n, seed=5)).to(dev)
    y = torch.empty_like(x)
    out = {"workload": a.workload, "n": s.n, "reps": a.spmv_reps, "order": []}
    for name in a.formats.split(","):
        with cgmi.Solver(name, *arrs[name]) as S:
            S.spmv(x, y)
            torch.cuda.synchronize()
            log(f"counters: {name} x {a.spmv_reps}")
            for _ in range(a.spmv_reps):
                S.spmv(x, y)
            torch.cuda.synchronize()
            out["order"].append(name)
    nel = (1 << 30) // 8
    src = torch.ones(nel, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_bytes_each_way"] = nel * 8
    print(json.dumps(out), flush=True)


def short_kernel_name(k):
    """A profiler kernel name without namespaces and argument list."""
    k = k.replace("void ", "").replace("cgmi::", "").replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            k = k[:i]
            break
    return k if len(k) <= 90 else k[:87] + "..."


def window_idle(trace_csv, first, last):
    """Per window from a launch of `first` to the next launch of `last`: wall
    time, time with at least one kernel running, and the rest (launch gaps)."""
    ev = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_kernel_name(r["Kernel_Name"])))
    ev.sort()
    out = ["## Solve windows (" + first + " ... " + last + ")", "",
           "| window | launches | wall ms | kernel-busy ms | idle % | largest gap us |", "|---|---|---|---|---|---|"]
    i, w = 0, 0
    while i < len(ev):
        if not ev[i][2].startswith(first):
            i += 1
            continue
        j = i
        while j < len(ev) and not ev[j][2].startswith(last):
            j += 1
        if j == len(ev):
            break
        seg = ev[i:j + 1]
        busy, end, gap = 0, seg[0][0], 0
        for s0, e0, _ in seg:
            if s0 > end:
                gap = max(gap, s0 - end)
            busy += max(0, e0 - max(s0, end))
            end = max(end, e0)
        wall = end - seg[0][0]
        w += 1
        out.append(f"| {w} | {len(seg)} | {wall / 1e6:.2f} | {busy / 1e6:.2f} | {100 * (wall - busy) / wall:.3f} | "
                   f"{gap / 1e3:.1f} |")
        i = j + 1
    return out + [""]


def summarize_trace(a):
    """Markdown tables from a rocprofv3 run: its --stats summary per kernel,
    and per kernel and grid size the launches and median / mean duration
    from the kernel trace (raw trace files are not kept)."""
    stats = glob.glob(os.path.join(a.trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    trace = glob.glob(os.path.join(a.trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    lines = []
    for f in stats:
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        lines += ["## rocprofv3 --stats (kernel_stats.csv)", "",
                  "| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
        for r in rows[:25]:
            lines.append(f"| `{short_kernel_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f} |")
        lines.append("")
    for f in trace:
        per = {}
        with open(f) as fh:
            for r in csv.DictReader(fh):
                key = (short_kernel_name(r["Kernel_Name"]), int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0))
                per.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        if a.windows:
            lines += window_idle(f, *a.windows.split(","))
        lines += ["## Per kernel and grid size (work-items), from the kernel trace", "",
                  "| kernel | grid | launches | median us | mean us | total ms |", "|---|---|---|---|---|---|"]
        for (k, g), v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:25]:
            lines.append(f"| `{k}` | {g} | {len(v)} | {statistics.median(v):.2f} | {statistics.mean(v):.2f} | "
                         f"{sum(v) / 1e3:.1f} |")
        lines.append("")
    print("\n".join(lines))


def parse_counters(a):
    """Per-launch HBM bytes of each format's product from a FETCH_SIZE run and
    a WRITE_SIZE run of `--mode counters` (rocprofv3 counter_collection.csv),
    each scaled by what the counter reads for the 1 GiB copy of the same run."""
    dirs = a.counter_dirs.split(",")
    per = {}
    calib = {}
    for d, ctr in zip(dirs, ("FETCH_SIZE", "WRITE_SIZE")):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        rows = []
        for f in files:
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r.get("Counter_Name") == ctr]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        copy = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()
                or "elementwise" in r["Kernel_Name"].lower()]
        calib[ctr] = dict(copy_kib=copy[-1] if copy else None)
        byk = {}
        for r in rows:
            byk.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        calib[ctr]["kernels"] = {k: dict(launches=len(v), mean_kib=statistics.mean(v)) for k, v in byk.items()}
    nb = (1 << 30)
    f_scale = nb / (calib["FETCH_SIZE"]["copy_kib"] * 1024)
    w_scale = nb / (calib["WRITE_SIZE"]["copy_kib"] * 1024)
    for fmt in ("csr", "symcsr", "csc"):
        ks = PRODUCT_KERNELS[fmt]
        per[fmt] = dict(fetch_bytes=0, write_bytes=0, kernels={})
        for k in calib["FETCH_SIZE"]["kernels"]:
            if not any(x in k for x in ks):
                continue
            fk = round(calib["FETCH_SIZE"]["kernels"][k]["mean_kib"] * 1024 * f_scale)
            wk = round(calib["WRITE_SIZE"]["kernels"].get(k, {"mean_kib": 0.0})["mean_kib"] * 1024 * w_scale)
            per[fmt]["kernels"][short_kernel_name(k)] = dict(fetch_bytes=fk, write_bytes=wk)
            per[fmt]["fetch_bytes"] += fk
            per[fmt]["write_bytes"] += wk
        per[fmt]["total"] = per[fmt]["fetch_bytes"] + per[fmt]["write_bytes"]
    # the commands that made these numbers, with the run directories given
    show = [os.path.abspath(d).replace(ROOT, "$REPO", 1) for d in dirs]
    run = ("cd /tmp && export TMPDIR=/tmp PYTHONPATH=$REPO && rocprofv3 --pmc {c} -d {d} -o c --output-format csv "
           "-- python3 $REPO/bench.py --mode counters --workload {w} --spmv-reps {r}")
    out = dict(kernel_src_sha=kernel_source_sha(), workload=a.workload,
               calibration=dict(copy_bytes_each_way=nb, fetch_scale=f_scale, write_scale=w_scale),
               per_launch_bytes={k: v["total"] for k, v in per.items()}, detail=per,
               command="; ".join([run.format(c=c, d=d, w=a.workload, r=a.spmv_reps)
                                  for c, d in zip(("FETCH_SIZE", "WRITE_SIZE"), show)]
                                 + [f"python3 $REPO/bench.py --mode parse-counters --workload {a.workload} "
                                    f"--spmv-reps {a.spmv_reps} --counter-dirs {show[0]},{show[1]}"]),
               note="HBM bytes per product launch (mean over its launches), each counter scaled by what it reads "
                    "for a 1 GiB device copy in the same run (FETCH_SIZE counts 64-byte requests, hence the factor "
                    "~2); symcsr and csc include their row-pass kernel (k_scatter_gather / k_panel_gather) of the "
                    "lone product, which inside CG is folded into the r update; detail.<format>.kernels splits the "
                    "bytes by kernel")
    with open(traffic_file(a.workload), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): this build has no multi-GPU path; "
              f"the value for one GPU is what it measures", file=sys.stderr)
        sys.exit(2)
    if a.mode == "parse-counters":
        return parse_counters(a)
    if a.mode == "summarize-trace":
        return summarize_trace(a)
    if a.mode == "counters":
        return counters_mode(a)
    import numpy as np
    import torch

    from paper_1010_4639_amd import cgmi
    from paper_1010_4639_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cgmi.load()
    dev = torch.device("cuda:0")
    t0 = time.time()
    s = W.fem_config(a.workload, keep_geometry=False)
    log(f"generated {a.workload}: n={s.n} nnz={s.nnz} in {time.time() - t0:.1f}s")
    if a.format == "symcsr":
        arrs = W.upper_triangle(s.rowptr, s.col, s.val)
    else:
        arrs = (s.rowptr, s.col, s.val)
    t1 = time.perf_counter()
    S = cgmi.Solver(a.format, *arrs)
    create_ms = (time.perf_counter() - t1) * 1e3
    log(f"created {a.format} handle in {create_ms:.0f} ms: {S.stats()}")
    b = torch.from_numpy(s.b).to(dev)
    x0 = torch.zeros_like(b)

    def step():
        x, info = S.solve(b, x0, tol=a.tol, maxit=a.maxit)
        if info["status"] != cgmi.CG_OK:
            raise RuntimeError(f"solve failed: {info}")
        return info

    for w in range(a.warmup):
        info = step()
        log(f"warmup {w}: {info['iters']} it, {info['ms']:.1f} ms")
    torch.cuda.synchronize()
    infos = []
    t_start = time.perf_counter()
    for k in range(a.steps):
        infos.append(step())
        log(f"step {k}: {infos[-1]['iters']} it, {infos[-1]['ms']:.1f} ms")
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1e3 / a.steps
    iters = infos[-1]["iters"]
    res = {"step": dict(time_to_tol_ms=round(ms_per_step, 3), iters=iters,
                        us_per_iter=round(1e3 * ms_per_step / iters, 3), relres_true=infos[-1]["relres_true"],
                        create_ms=round(create_ms, 1), device_bytes=S.stats()["device_bytes"])}

    # the dominant kernel: the product, back to back and cold
    timer = Timer(torch)
    xs = torch.from_numpy(W.uniform_vector(s.n, seed=99)).to(dev)
    ys = torch.empty_like(xs)
    scratch = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    flushed = torch.empty(1, dtype=torch.float64, device=dev)

    def flush():
        # a 1 GiB read evicts L2 and the 256 MB Infinity Cache, leaving clean lines
        torch.sum(scratch, dim=0, keepdim=True, out=flushed)

    nbytes = spmv_bytes(s.n, len(arrs[1]))
    prod = product_figures(torch, timer, S, xs, ys, nbytes, a.spmv_reps, flush)
    res["spmv"] = prod
    log(f"product {a.format}: {prod['us']:.1f} us back to back ({prod['GBps']:.0f} GB/s), cold {prod['cold_us']:.1f} us")
    # plain device copy of 1 GiB: the practical bandwidth ceiling
    c = torch.empty_like(scratch)
    copy_us = timer.per_call_us(lambda: c.copy_(scratch), 10, warm=2)
    copy_gbps = 2 * scratch.numel() * 8 / copy_us / 1e3
    del c
    kernel = {"csr": "k_spmv_slices (CSR product, 64-row slices)" if prod["sliced"] else "k_spmv_csr_rows",
              "symcsr": "symmetric-CSR product (scatter kernel + row pass)",
              "csc": "CSC product on column panels (slot kernel + row pass)"}[a.format]
    # a matrix that stays in the Infinity Cache between products is priced
    # against HBM on its cold launches (after the 1 GiB read); its warm rate
    # is an effective cache rate, reported beside it
    resident = prod["matrix_cache_resident"]
    use_us, use_gbps = (prod["cold_us"], prod["cold_GBps"]) if resident else (prod["us"], prod["GBps"])
    roofline = dict(bound="hbm", achieved=use_gbps, peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(use_gbps / HBM_PEAK_GBPS, 4), traffic=load_traffic(a.workload, a.format),
                    kernel=kernel, bytes_per_launch=nbytes, avg_us=use_us,
                    timing="cold launches (matrix cache-resident when warm)" if resident else "back to back",
                    cold_frac=round(prod["cold_GBps"] / HBM_PEAK_GBPS, 4),
                    matrix_cache_resident=resident,
                    frac_of_copy=round(use_gbps / copy_gbps, 4))
    if resident:
        roofline["warm_cache_GBps"] = prod["GBps"]

    def room(name):
        if name not in a.extras:
            return False
        if time.time() - T_START > a.budget_s:
            res.setdefault("skipped", []).append(name)
            log(f"skipping {name}: {time.time() - T_START:.0f} s spent")
            return False
        return True

    cpu = None
    all_arrs = None
    if room("formats"):
        all_arrs = extra_formats(torch, cgmi, W, s, a, b, timer, xs, ys, flush, res)
    del scratch, flushed
    S.close()
    if room("mixed"):
        if all_arrs is None:
            up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
            all_arrs = {"csr": (s.rowptr, s.col, s.val), "symcsr": (up, uc, uv)}
        extra_mixed(torch, cgmi, W, s, a, b, all_arrs, res)
    if room("cpu"):
        cpu = cpu_baseline(s, a.format, iters)
    del all_arrs
    if room("small"):
        extra_small(torch, cgmi, W, a, res)
    if room("adjoint"):
        extra_adjoint(torch, cgmi, W, a, res)
    if room("batch"):
        extra_batch(torch, cgmi, W, a, res)

    out = {
        "metric": "CG time-to-1e-10 residual",
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload}: 3D P1 Kuhn-tet FEM stiffness, {s.nx}x{s.ny}x{s.nz} interior grid, "
                        f"n={s.n}, nnz={s.nnz}, iron box {s.iron_fraction:.3f} of cells, one FP64 CG solve "
                        f"stored as {a.format}, x0=0, tol={a.tol:g}",
            "format": a.format,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stream_copy_GBps": round(copy_gbps, 1),
        **res,
        "elapsed_s": round(time.time() - T_START, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

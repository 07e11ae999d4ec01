"""Timing of the differentiable solve on the 100^3 system with per-element nu.

    python -m paper_1010_4639_amd.bench_adjoint [--workload fem100] [--reps 3]

Loss L = ||x - x_obs||^2, x = A(nu)^-1 b, nu = the generator's cell values
times U(0.8, 1.25) per element (seeded), x0 = 0, tol 1e-10.  Reports, as one
JSON line: the forward pass (assembly + CG) and the backward pass (assembly
again + adjoint CG + dL/dnu), both wall-clock with the host blocking on the
result; the plain FP64 solve of the same system for comparison; and the two
operator kernels (assembly, dL/dnu) as average launch time over 20 launches
(HIP events on the launch stream) with their algorithmic bytes:
  assembly  4(nnz+1) + 8 nnz + 4 C + 8 C + 8 C   (C = element contributions:
            list entry, nu_e and K_e[p] read once per contribution)
  dL/dnu    (16 + 80 + 8) nelem + 16 n           (dofs, K_e, gradient; lam, x)
"""
import argparse
import json
import statistics
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="fem100")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-iters", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args(argv)
    import numpy as np
    import torch

    from paper_1010_4639_amd import adjoint, cgmi
    from paper_1010_4639_amd import workload as W

    dev = torch.device("cuda:0")
    t0 = time.time()
    s = W.fem_config(a.workload)
    coords, tets, dof, nu_cell = W.fem_mesh(s)
    nu = nu_cell * np.random.default_rng(101).uniform(0.8, 1.25, size=nu_cell.size)
    xo = torch.from_numpy(W.observation(s)).to(dev)
    b = torch.from_numpy(s.b).to(dev)
    print(f"[adjoint] {a.workload}: n={s.n} nnz={s.nnz} nelem={nu.size} generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    t1 = time.time()
    FS = adjoint.FemSolve(coords, tets, dof, s.n)
    print(f"[adjoint] operator + solver planned in {time.time() - t1:.1f}s", file=sys.stderr, flush=True)
    fwd, bwd, plain = [], [], []
    g = None
    for r in range(a.reps + 1):
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
        print(f"[adjoint] rep {r}: forward {1e3 * (t2 - t1):.1f} ms, backward {1e3 * (t3 - t2):.1f} ms",
              file=sys.stderr, flush=True)
    xs = x.detach()
    ident = (float(torch.from_numpy(nu).to(dev) @ g), -2.0 * float((xs - xo) @ xs))
    # the plain FP64 solve on the same matrix (values as in the last forward)
    for r in range(a.reps + 1):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = FS.solver.solve(b, tol=a.tol)
        torch.cuda.synchronize()
        if r > 0:
            plain.append((time.perf_counter() - t1) * 1e3)
    # operator kernels
    stream = torch.cuda.current_stream()
    nu_d = torch.from_numpy(nu).to(dev)
    vals = FS.fem.assemble(nu_d)
    lam = torch.from_numpy(W.uniform_vector(s.n, seed=41)).to(dev)
    gout = torch.empty(nu.size, dtype=torch.float64, device=dev)

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    us_asm = timed(lambda: FS.fem.assemble(nu_d, out=vals))
    FS_vals = vals.cpu().numpy()
    FS_rp, FS_col = FS.fem.pattern()
    us_grad = timed(lambda: FS.fem.nu_grad(lam, xs, out=gout))
    nnz, nelem = FS.nnz, FS.nelem
    ncontrib = int(np.sum(np.count_nonzero(dof[tets] >= 0, axis=1) ** 2))
    by_asm = 4 * (nnz + 1) + 8 * nnz + 20 * ncontrib
    by_grad = 104 * nelem + 16 * s.n
    out = {
        "workload": f"{a.workload}: n={s.n}, nnz={s.nnz}, nelem={nelem}, per-element nu, L=||x-x_obs||^2",
        "tol": a.tol,
        "forward_ms": round(statistics.median(fwd), 3),
        "backward_ms": round(statistics.median(bwd), 3),
        "plain_fp64_solve_ms": round(statistics.median(plain), 3),
        "iters_plain": info["iters"],
        "identity_sum_nu_grad": ident[0], "identity_rhs": ident[1],
        "identity_rel_diff": abs(ident[0] - ident[1]) / abs(ident[1]),
        "assemble_us": round(us_asm, 3), "assemble_bytes": by_asm, "assemble_GBps": round(by_asm / us_asm / 1e3, 1),
        "nu_grad_us": round(us_grad, 3), "nu_grad_bytes": by_grad, "nu_grad_GBps": round(by_grad / us_grad / 1e3, 1),
        "contributions": ncontrib,
    }
    FS.close()
    if not a.no_cpu:
        # the oracle beside it (test infrastructure, timed on a bounded sample):
        # its CG per iteration on the same matrix, scaled by the GPU's forward +
        # adjoint iteration counts, plus its element gradient over every element
        import oracle
        from oracle import fem as OF
        vals = FS_vals
        t1 = time.perf_counter()
        _, oi, _ = oracle.cg(oracle.FMT_CSR, FS_rp, FS_col, vals, s.b, tol=0.0, maxit=a.cpu_iters)
        ms_it = oi["ms_loop"] / max(oi["iters"], 1)
        t2 = time.perf_counter()
        K = np.empty((nelem, 4, 4))
        for i in range(0, nelem, 1 << 20):
            K[i:i + (1 << 20)] = OF.element_matrices(coords, tets[i:i + (1 << 20)])
        lam_h = W.uniform_vector(s.n, seed=41)
        t3 = time.perf_counter()
        OF.nu_grad(K, tets, dof, lam_h, xs.cpu().numpy())
        t4 = time.perf_counter()
        out["cpu_baseline"] = dict(kind="oracle", cores=1, unit="ms",
                                   value=round(ms_it * 2 * info["iters"] + (t4 - t3) * 1e3, 1),
                                   sample=f"{oi['iters']} oracle CG iterations ({ms_it:.2f} ms each) scaled by "
                                          f"2 x {info['iters']} (forward + adjoint); element gradient "
                                          f"{(t4 - t3) * 1e3:.0f} ms (numpy, after {(t3 - t2):.1f} s of element "
                                          f"matrices)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

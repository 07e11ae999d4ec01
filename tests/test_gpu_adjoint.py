"""Differentiable solve on the GPU against the adjoint oracle.

Kernel parity (seeded inputs, never GPU outputs, fed to both sides):
  * the operator's pattern equals the generator's (integer structure, exact);
  * assembly A(nu) per entry within 1e-13 of sum_e |nu_e| sqrt(K_aa K_bb)
    (the size of each element term before cancellation);
  * dL/dnu_e = -lam_e' K_e x_e per element within 1e-13 of
    sum_ab sqrt(K_aa K_bb) |lam_a| |x_b|;
  * dL/d(stored value) bit-exact in every storage form (one or two rounded
    products and one rounded sum, the same on both sides);
  * new values through cg_set_values give the same bits as a fresh handle.
End to end (torch.autograd): gradients against the oracle's dense or CG
adjoint, central finite differences of the oracle's dense forward on 32
random nu entries, and, on the 100^3 system (6 181 806 elements), the
homogeneity identity sum_e nu_e dL/dnu_e = -2 (x - x_obs)' x and central
differences of the GPU forward on 32 random elements against a bound built
from the measured residuals; and against the FP64 oracle gradient of the same
case, stored by tests/golden/make_adjoint_reference.py (loss, gradient norm,
4096 sampled elements).
"""
import hashlib
import os

import numpy as np
import pytest

from oracle import fem as OF
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

_MESH = {}


def mesh(name):
    """(system, coords, tets, dof, nu_cell) for a named case, cached per process."""
    if name not in _MESH:
        if name == "fem12":
            s = W.fem_p1_system(12, 11, 10, nu_iron=1e-2, seed=7)
        elif name == "fem40":
            s = W.fem_p1_system(40, 40, 40, nu_iron=1e-3, seed=5)
        else:
            s = W.fem_config("fem100")
        _MESH[name] = (s,) + W.fem_mesh(s)
    return _MESH[name]


def oracle_K(coords, tets, chunk=1 << 20):
    out = np.empty((tets.shape[0], 4, 4))
    for i in range(0, tets.shape[0], chunk):
        out[i:i + chunk] = OF.element_matrices(coords, tets[i:i + chunk])
    return out


@pytest.mark.parametrize("name", ["fem12", "fem40", "fem100"])
def test_fem_pattern_and_generator_values(name):
    s, coords, tets, dof, nu = mesh(name)
    say(f"fem pattern {name}: n={s.n} nelem={tets.shape[0]}")
    with cgmi.FemOperator(coords, tets, dof, s.n) as F:
        rp, col = F.pattern()
        assert np.array_equal(rp, s.rowptr) and np.array_equal(col, s.col)
        v = F.assemble(to_dev(nu)).cpu().numpy()
    # the generator assembles the same operator by another route (upper keys, bincount)
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    dpos = np.nonzero(rows == s.col)[0]
    dval = np.zeros(s.n)
    dval[rows[dpos]] = np.abs(s.val[dpos])
    err = np.abs(v - s.val)
    assert np.all(err <= 1e-12 * dval[rows]), float(np.max(err / dval[rows]))


@pytest.mark.parametrize("name", ["fem12", "fem40"])
def test_fem_assemble_parity(name):
    s, coords, tets, dof, _ = mesh(name)
    rng = np.random.default_rng(31)
    nu = rng.uniform(0.2, 2.0, size=tets.shape[0])
    K = oracle_K(coords, tets)
    ref = OF.assemble(nu, K, tets, dof, s.rowptr, s.col)
    scale = OF.assemble(np.abs(nu), OF.cauchy_schwarz_scale(K), tets, dof, s.rowptr, s.col)
    say(f"fem assemble {name}: nnz={s.col.size}")
    with cgmi.FemOperator(coords, tets, dof, s.n) as F:
        v = F.assemble(to_dev(nu)).cpu().numpy()
        v2 = F.assemble(to_dev(nu)).cpu().numpy()
    assert np.array_equal(v, v2)                      # fixed summation order
    assert np.all(np.abs(v - ref) <= 1e-13 * scale), float(np.max(np.abs(v - ref) / scale))


@pytest.mark.parametrize("name", ["fem12", "fem40", "fem100"])
def test_fem_nu_grad_parity(name):
    s, coords, tets, dof, _ = mesh(name)
    lam = W.uniform_vector(s.n, seed=41)
    x = W.uniform_vector(s.n, seed=42)
    say(f"fem nu_grad {name}: nelem={tets.shape[0]}")
    with cgmi.FemOperator(coords, tets, dof, s.n) as F:
        g = F.nu_grad(to_dev(lam), to_dev(x)).cpu().numpy()
    chunk = 1 << 20
    for i in range(0, tets.shape[0], chunk):
        t = tets[i:i + chunk]
        K = OF.element_matrices(coords, t)
        ref = OF.nu_grad(K, t, dof, lam, x)
        scale = -OF.nu_grad(OF.cauchy_schwarz_scale(K), t, dof, np.abs(lam), np.abs(x))
        err = np.abs(g[i:i + chunk] - ref)
        assert np.all(err <= 1e-13 * scale + 1e-300), (i, float(np.max(err - 1e-13 * scale)))


def _formats(s):
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    lp, lc, lv = W.transpose_csr(s.n, s.n, up, uc, uv)          # lower triangle by rows
    return [("csr", s.rowptr, s.col, s.val, 0, 0), ("csc", s.rowptr, s.col, s.val, 0, 0),
            ("symcsr", up, uc, uv, 0, 0), ("symcsr", lp, lc, lv, 0, cgmi.CG_LOWER),
            ("csr", s.rowptr + 1, s.col + 1, s.val, 1, 0)]


def _oracle_pattern_grad(fmt, ptr, idx, flags, lam, x):
    f = cgmi.FORMATS[fmt]
    if flags & cgmi.CG_LOWER:
        # a stored lower entry l_ij stands for A_ij and A_ji: the symmetric rule
        return OF.pattern_grad(1, ptr, idx, lam, x)
    return OF.pattern_grad(f, ptr, idx, lam, x)


def test_pattern_grad_bit_exact():
    s = mesh("fem12")[0]
    lam = W.uniform_vector(s.n, seed=51)
    x = W.uniform_vector(s.n, seed=52)
    for fmt, ptr, idx, val, base, flags in _formats(s):
        say(f"pattern_grad {fmt} base={base} flags={flags}")
        with cgmi.Solver(fmt, ptr, idx, val, index_base=base, flags=flags) as S:
            g = S.pattern_grad(to_dev(lam), to_dev(x)).cpu().numpy()
        ref = _oracle_pattern_grad(fmt, np.asarray(ptr) - base, np.asarray(idx) - base, flags, lam, x)
        assert np.array_equal(g, ref), (fmt, flags, float(np.max(np.abs(g - ref))))


def test_set_values_matches_fresh_handle():
    s = mesh("fem12")[0]
    rng = np.random.default_rng(61)
    xv = to_dev(W.uniform_vector(s.n, seed=62))
    for fmt, ptr, idx, val, base, flags in _formats(s):
        val2 = val * rng.uniform(0.5, 1.5, size=val.size)
        say(f"set_values {fmt} base={base} flags={flags}")
        with cgmi.Solver(fmt, ptr, idx, val, index_base=base, flags=flags) as S, \
                cgmi.Solver(fmt, ptr, idx, val2, index_base=base, flags=flags) as T:
            S.set_values(to_dev(val2))
            assert np.array_equal(S.spmv(xv).cpu().numpy(), T.spmv(xv).cpu().numpy())


def test_set_values_mixed():
    s = mesh("fem12")[0]
    b = to_dev(s.b)
    # a symmetric rescaling keeps A SPD: D A D with D > 0
    d = np.random.default_rng(71).uniform(0.5, 2.0, size=s.n)
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    val2 = s.val * d[rows] * d[s.col]
    with cgmi.Solver("csr", s.rowptr, s.col, s.val, mixed=True) as S, \
            cgmi.Solver("csr", s.rowptr, s.col, val2, mixed=True) as T:
        S.set_values(to_dev(val2))
        xs, i1 = S.solve_mixed(b, tol=1e-12)
        xt, i2 = T.solve_mixed(b, tol=1e-12)
        assert i1["status"] == 0 and i1["iters"] == i2["iters"]
        assert np.array_equal(xs.cpu().numpy(), xt.cpu().numpy())
        bad = val2.copy()
        bad[np.nonzero(rows == s.col)[0][3]] = -1.0
        with pytest.raises(cgmi.CgError):
            S.set_values(to_dev(bad))


def test_set_values_errors():
    s = mesh("fem12")[0]
    with cgmi.Solver("csr", s.rowptr, s.col, s.val) as S:
        with pytest.raises(TypeError):
            S.set_values(to_dev(s.val[:-1]))
        assert cgmi.cg_set_values(S.h, 0) == cgmi.CG_ERR_ARG
        assert cgmi.cg_pattern_grad(S.h, 0, 0, 0) == cgmi.CG_ERR_ARG


def test_fem_create_errors():
    s, coords, tets, dof, _ = mesh("fem12")
    bad_t = tets.copy()
    bad_t[5, 2] = coords.shape[0]
    st, h = cgmi.cg_fem_create(coords, bad_t, dof, s.n)
    assert st == cgmi.CG_ERR_ARG and "tets" in cgmi.cg_fem_last_error(None)
    bad_d = dof.copy()
    bad_d[0] = s.n
    assert cgmi.cg_fem_create(coords, tets, bad_d, s.n)[0] == cgmi.CG_ERR_ARG
    bad_c = coords.copy()
    bad_c[3, 1] = np.nan
    assert cgmi.cg_fem_create(bad_c, tets, dof, s.n)[0] == cgmi.CG_ERR_NONFINITE
    flat = tets.copy()
    flat[7, 3] = flat[7, 2]                          # repeated vertex: zero volume
    assert cgmi.cg_fem_create(coords, flat, dof, s.n)[0] == cgmi.CG_ERR_ARG
    # an empty operator is valid
    with cgmi.FemOperator(np.zeros((0, 3)), np.zeros((0, 4), np.int32), np.zeros(0, np.int32), 0) as F:
        assert F.nnz == 0


# ------------------------------------------------------------- end to end
def _loss_grads(name, tol=1e-12):
    import torch
    from paper_1010_4639_amd import adjoint
    s, coords, tets, dof, _ = mesh(name)
    rng = np.random.default_rng(81)
    nu = rng.uniform(0.2, 2.0, size=tets.shape[0])
    xo = W.observation(s)
    with adjoint.FemSolve(coords, tets, dof, s.n) as FS:
        nu_t = to_dev(nu).requires_grad_(True)
        b_t = to_dev(s.b).requires_grad_(True)
        x = FS(nu_t, b_t, tol=tol)
        L = ((x - to_dev(xo)) ** 2).sum()
        L.backward()
        out = dict(x=x.detach().cpu().numpy(), L=float(L.detach()), g_nu=nu_t.grad.cpu().numpy(),
                   g_b=b_t.grad.cpu().numpy())
        # the same through the pattern-valued solve
        vals = FS.fem.assemble(to_dev(nu)).requires_grad_(True)
        b2 = to_dev(s.b)
        x2 = adjoint.sparse_solve(vals, b2, FS.solver, tol=tol)
        ((x2 - to_dev(xo)) ** 2).sum().backward()
        out["g_vals"] = vals.grad.cpu().numpy()
        out["x2"] = x2.detach().cpu().numpy()
    return s, coords, tets, dof, nu, xo, out


def test_autograd_vs_dense_oracle_and_fd():
    s, coords, tets, dof, nu, xo, g = _loss_grads("fem12")
    K = OF.element_matrices(coords, tets)
    ref = OF.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)
    for k_gpu, k_orc in (("x", "x"), ("g_nu", "g_nu"), ("g_b", "g_b"), ("g_vals", "g_vals")):
        err = np.linalg.norm(g[k_gpu] - ref[k_orc]) / np.linalg.norm(ref[k_orc])
        say(f"fem12 {k_gpu}: rel err {err:.2e}")
        assert err <= 1e-7, (k_gpu, err)
    assert np.array_equal(g["x"], g["x2"])
    # central differences of the oracle's dense forward on 32 random elements
    rng = np.random.default_rng(91)
    touch = np.nonzero((dof[tets] >= 0).any(axis=1))[0]
    for e in rng.choice(touch, size=32, replace=False):
        h = 1e-5 * nu[e]
        nup, num = nu.copy(), nu.copy()
        nup[e] += h
        num[e] -= h
        Lp = OF.solve_grad(nup, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)["L"]
        Lm = OF.solve_grad(num, s.b, xo, K, tets, dof, s.rowptr, s.col, dense_solve=True)["L"]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g["g_nu"][e]) <= 1e-5 * abs(fd) + 1e-7 * np.abs(g["g_nu"]).max(), (e, fd, g["g_nu"][e])


def test_autograd_vs_cg_oracle_fem40():
    s, coords, tets, dof, nu, xo, g = _loss_grads("fem40")
    K = oracle_K(coords, tets)
    ref = OF.solve_grad(nu, s.b, xo, K, tets, dof, s.rowptr, s.col, tol=1e-12)
    for k in ("x", "g_nu", "g_b", "g_vals"):
        err = np.linalg.norm(g[k] - ref[k]) / np.linalg.norm(ref[k])
        say(f"fem40 {k}: rel err {err:.2e}")
        assert err <= 1e-6, (k, err)


def test_fem100_adjoint_identity_and_fd():
    """The 100^3 adjoint (6 181 806 per-element coefficients)."""
    import torch
    from paper_1010_4639_amd import adjoint
    s, coords, tets, dof, nu_cell = mesh("fem100")
    rng = np.random.default_rng(101)
    nu = nu_cell * rng.uniform(0.8, 1.25, size=nu_cell.size)
    xo = W.observation(s)
    tol = 1e-12
    say(f"fem100 adjoint: n={s.n} nelem={nu.size}")
    with adjoint.FemSolve(coords, tets, dof, s.n) as FS:
        nu_t = to_dev(nu).requires_grad_(True)
        b_t = to_dev(s.b)
        x = FS(nu_t, b_t, tol=tol)
        L = ((x - to_dev(xo)) ** 2).sum()
        L.backward()
        g = nu_t.grad.cpu().numpy()
        xn = x.detach().cpu().numpy()
        # identity: sum_e nu_e dL/dnu_e = -lam' A x = -lam' b = -2 (x - x_obs)' x
        lhs = float(nu @ g)
        rhs = -2.0 * float((xn - xo) @ xn)
        say(f"fem100 identity: {lhs:.12e} vs {rhs:.12e}")
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs)
        # central differences of the GPU forward, warm-started, on 32 elements;
        # first-order bound of the solve error in L: |lam' r| <= ||lam|| ||r||
        lam = (torch.linalg.norm(FS.solver.solve(2.0 * (x.detach() - to_dev(xo)), tol=tol)[0])).item()
        nb = float(np.linalg.norm(s.b))
        touch = np.nonzero((dof[tets] >= 0).all(axis=1))[0]
        worst = 0.0
        for e in rng.choice(touch, size=32, replace=False):
            h = 1e-3 * nu[e]
            Ls, rr = [], []
            for sgn in (1.0, -1.0):
                nup = nu_t.detach().clone()
                nup[int(e)] += sgn * h
                FS.solver.set_values(FS.fem.assemble(nup))
                xp, info = FS.solver.solve(b_t, x0=x.detach(), tol=1e-13)
                Ls.append(float(((xp - to_dev(xo)) ** 2).sum()))
                rr.append(info["relres_true"] * nb)
            fd = (Ls[0] - Ls[1]) / (2 * h)
            bound = lam * (rr[0] + rr[1]) / (2 * h) + 1e-5 * abs(g[e]) + 1e-13 * abs(float(L)) / h
            worst = max(worst, abs(fd - g[e]) / bound)
            assert abs(fd - g[e]) <= bound, (int(e), fd, g[e], bound)
        say(f"fem100 fd: worst |fd - g| / bound = {worst:.3f}")


def test_fem100_adjoint_vs_stored_oracle_gradient():
    """The 100^3 gradient against the FP64 oracle's (two serial oracle CG
    solves at tol 1e-12 over oracle/fem.py, stored by
    tests/golden/make_adjoint_reference.py): the loss, the homogeneity
    identity and dL/dnu at 4096 seeded elements.  The two gradients come
    from different FP64 evaluations of the same two solves, so they agree to
    the solves' accuracy, not bit for bit: bar 1e-6 relative (2-norm over the
    sample, and per element against the sample's largest entry)."""
    import json
    from paper_1010_4639_amd import adjoint
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fem100_adjoint_oracle.json")
    with open(path) as f:
        ref = json.load(f)
    s, coords, tets, dof, nu_cell = mesh("fem100")
    nu = nu_cell * np.random.default_rng(101).uniform(0.8, 1.25, size=nu_cell.size)
    xo = W.observation(s)
    assert hashlib.sha256(np.ascontiguousarray(s.b).tobytes()).hexdigest() == ref["b_sha256"]
    pos = np.array(ref["sample_elem"], dtype=np.int64)
    g_ref = np.array([float.fromhex(h) for h in ref["sample_g"]])
    with adjoint.FemSolve(coords, tets, dof, s.n) as FS:
        nu_t = to_dev(nu).requires_grad_(True)
        x = FS(nu_t, to_dev(s.b), tol=ref["tol"])
        L = ((x - to_dev(xo)) ** 2).sum()
        L.backward()
        g = nu_t.grad.cpu().numpy()
    Lg = float(L.detach())
    err = np.linalg.norm(g[pos] - g_ref) / np.linalg.norm(g_ref)
    worst = float(np.max(np.abs(g[pos] - g_ref)) / np.max(np.abs(g_ref)))
    say(f"fem100 adjoint vs stored oracle: L {Lg:.12e} / {ref['L']:.12e}, sampled g rel 2-norm {err:.2e}, "
        f"max {worst:.2e}, ||g|| {np.linalg.norm(g):.6e} / {ref['norm2_g']:.6e}")
    assert abs(Lg - ref["L"]) <= 1e-8 * ref["L"]
    assert abs(np.linalg.norm(g) - ref["norm2_g"]) <= 1e-6 * ref["norm2_g"]
    assert err <= 1e-6 and worst <= 1e-6, (err, worst)

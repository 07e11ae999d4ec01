"""Seeded synthetic inputs for the CG / SpMV path.

This module only MAKES inputs: a finite-element stiffness matrix of the kind
the paper solves (symmetric positive definite, about 15 nonzeros per row, from
a 3D electrical-machine style model with a high-permeability "iron" region),
its right-hand side, and small test matrices.  It holds none of the solver's
arithmetic (no CSR/CSC product, no CG step); both the GPU library's tests and
the CPU oracle's tests draw their inputs from here.

FEM workload (stand-in for the paper's 30 880 x 30 880 machine matrix,
section III; the paper's files are not available):

* lattice of nodes h*(i, j, k), h = 1, i in [0, nx+1] etc.; interior nodes
  1..nx x 1..ny x 1..nz are the unknowns, numbered x-fastest
  (id = (i-1) + nx*((j-1) + ny*(k-1))); the lattice boundary is Dirichlet 0,
  so those rows/columns are simply absent;
* every interior node is moved by U(-jitter, jitter)*h per coordinate,
  boundary nodes stay put (the domain remains a box);
* every lattice cube is split into the 6 Kuhn tetrahedra
  (for each axis permutation s, lexicographic order: v0 = c, v1 = v0 + e_s0,
  v2 = v1 + e_s1, v3 = c + (1,1,1)); all edges then point along one of the 7
  positive directions {0,1}^3 \\ {0}, which gives the 15-point stencil;
* linear (P1) element stiffness K_e = nu_e |T_e| G^T G, G = gradients of the
  4 barycentric basis functions;
* reluctivity nu = 1 ("air") except in a box of cells with side
  round(frac^(1/3) * cells) per axis at a seeded integer origin ("iron"),
  where nu = nu_iron;
* assembly keeps only the upper key (lower node, direction), accumulated in a
  fixed order (axis permutation outer, then vertex pair, then cell x-fastest),
  and mirrors it, so the matrix is exactly (bitwise) symmetric; the pattern
  comes from the mesh graph, not from the values (a stored entry may be 0);
* b = A x_true, formed element by element (sum over elements of K_e x_e),
  x_true ~ U(-1, 1).

Seeds: numpy SeedSequence(seed).spawn(4) gives the PCG64 streams
[jitter, iron, x_true, x_obs]; jitter is drawn as an array of shape
(nz, ny, nx, 3) in C order, the iron origin as three integers (x, y, z).
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

# direction code d = dx + 2*dy + 4*dz, d = 1..7; code 0 is the diagonal
DIRS = np.array([[(d >> 0) & 1, (d >> 1) & 1, (d >> 2) & 1] for d in range(8)], dtype=np.int64)
PERMS = list(itertools.permutations((0, 1, 2)))          # lexicographic order
PERM_SIGN = [1, -1, -1, 1, 1, -1]                         # sign of each permutation above


@dataclasses.dataclass
class FemSystem:
    """A generated FEM system, full CSR (0-based, int32 indices, float64 values)."""
    nx: int
    ny: int
    nz: int
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    x_true: np.ndarray
    b: np.ndarray
    coords: np.ndarray        # (nz+2, ny+2, nx+2, 3) node positions incl. boundary
    nu_cell: np.ndarray       # (nz+1, ny+1, nx+1) reluctivity per cube
    iron_box: tuple           # ((ox, oy, oz), (Lx, Ly, Lz)) in cell indices
    iron_fraction: float
    min_orient_det: float     # min over tets of sign(perm)*det(J)
    seed: int = 0

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def iron_box(cells, frac, rng):
    """Box of cells with side round(frac^(1/3) * C_d) on each axis, origin uniform
    over the integers [0, C_d - L_d] (drawn x, y, z)."""
    side = [int(np.floor(frac ** (1.0 / 3.0) * c + 0.5)) for c in cells]
    org = [int(rng.integers(0, c - s + 1)) for c, s in zip(cells, side)]
    return tuple(org), tuple(side)


def _lattice(nx, ny, nz, jitter, rng):
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    P = np.stack([i, j, k], axis=-1).astype(np.float64)
    d = rng.uniform(-jitter, jitter, size=(nz, ny, nx, 3))
    P[1:-1, 1:-1, 1:-1, :] += d
    return P


def _node_ids(nx, ny, nz):
    """Lattice (k, j, i) -> interior id, -1 on the boundary."""
    ids = -np.ones((nz + 2, ny + 2, nx + 2), dtype=np.int64)
    ids[1:-1, 1:-1, 1:-1] = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    return ids


def direction_offsets(nx, ny):
    return DIRS[:, 0] + nx * DIRS[:, 1] + nx * ny * DIRS[:, 2]


def fem_p1_system(nx, ny, nz, *, nu_iron=1e-3, iron_frac=0.4, jitter=0.2, seed=1,
                  with_rhs=True, keep_geometry=True, nrhs=1) -> FemSystem:
    """Assemble the P1 / Kuhn-tet stiffness matrix on an nx*ny*nz interior grid.
    nrhs > 1: x_true and b get shape (n, nrhs) (columns drawn in order from the
    x_true stream; the first column equals the nrhs = 1 draw)."""
    rng_jit, rng_iron, rng_x, _ = _streams(seed)
    n = nx * ny * nz
    P = _lattice(nx, ny, nz, jitter, rng_jit)
    ids = _node_ids(nx, ny, nz)
    cells = (nx + 1, ny + 1, nz + 1)
    nu_cell = np.ones((nz + 1, ny + 1, nx + 1))
    if iron_frac > 0:
        (ox, oy, oz), (lx, ly, lz) = iron_box(cells, iron_frac, rng_iron)
        nu_cell[oz:oz + lz, oy:oy + ly, ox:ox + lx] = nu_iron
        box = ((ox, oy, oz), (lx, ly, lz))
    else:
        box = ((0, 0, 0), (0, 0, 0))
    iron_fraction = float(np.mean(nu_cell != 1.0))
    xcols = [rng_x.uniform(-1.0, 1.0, size=n) for _ in range(nrhs)] if with_rhs else []
    xls = []
    for xc in xcols:
        xl = np.zeros((nz + 2, ny + 2, nx + 2))
        xl[1:-1, 1:-1, 1:-1] = xc.reshape(nz, ny, nx)
        xls.append(xl.ravel())

    U8 = np.zeros(n * 8)                 # upper key (node, direction code)
    bcols = [np.zeros(n) for _ in xcols]
    cz, cy, cx = cells[2], cells[1], cells[0]
    nu_flat = nu_cell.ravel()
    min_orient = np.inf
    lat_shape = (nz + 2, ny + 2, nx + 2)
    ids_flat = ids.ravel()
    P_flat = P.reshape(-1, 3)
    # lattice linear index of every cell corner c, x-fastest over cells
    base = (np.arange(cz)[:, None, None] * (ny + 2) + np.arange(cy)[None, :, None]) * (nx + 2) \
        + np.arange(cx)[None, None, :]
    base = base.ravel()
    lat_stride = np.array([1, nx + 2, (nx + 2) * (ny + 2)], dtype=np.int64)
    for s_idx, perm in enumerate(PERMS):
        offs = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] += 1
            offs.append(cur)
        # offs = [0, e_s0, e_s0+e_s1, (1,1,1)]
        lin = [base + int(o @ lat_stride) for o in offs]
        V = [P_flat[l] for l in lin]
        J = np.stack([V[1] - V[0], V[2] - V[0], V[3] - V[0]], axis=-1)   # columns
        det = np.linalg.det(J)
        orient = PERM_SIGN[s_idx] * det
        min_orient = min(min_orient, float(orient.min()))
        if not np.all(orient > 0):
            raise ValueError("inverted tetrahedron: jitter too large for the Kuhn split")
        Jinv = np.linalg.inv(J)                          # rows = grad phi_1..3
        g = np.empty((base.size, 4, 3))
        g[:, 1:, :] = Jinv
        g[:, 0, :] = -Jinv.sum(axis=1)
        w = nu_flat * np.abs(det) / 6.0
        node = [ids_flat[l] for l in lin]
        keys_l, vals_l = [], []
        for a in range(4):
            for bb in range(a, 4):
                kab = w * np.einsum("ij,ij->i", g[:, a, :], g[:, bb, :])
                d = offs[bb] - offs[a]
                code = int(d[0] + 2 * d[1] + 4 * d[2])
                m = (node[a] >= 0) & (node[bb] >= 0)
                keys_l.append(node[a][m] * 8 + code)
                vals_l.append(kab[m])
        U8 += np.bincount(np.concatenate(keys_l), weights=np.concatenate(vals_l), minlength=n * 8)
        for xl, bc in zip(xls, bcols):
            for a in range(4):
                acc = np.zeros(base.size)
                for bb in range(4):
                    kab = w * np.einsum("ij,ij->i", g[:, a, :], g[:, bb, :])
                    acc += kab * xl[lin[bb]]
                m = node[a] >= 0
                bc += np.bincount(node[a][m], weights=acc[m], minlength=n)
        del J, Jinv, g, V
    rowptr, col, val = _upper_keys_to_csr(U8, nx, ny, nz)
    if not with_rhs:
        x_true = b = None
    elif nrhs == 1:
        x_true, b = xcols[0], bcols[0]
    else:
        x_true, b = np.stack(xcols, axis=1), np.stack(bcols, axis=1)
    return FemSystem(nx=nx, ny=ny, nz=nz, n=n, rowptr=rowptr, col=col, val=val,
                     x_true=x_true, b=b, coords=P if keep_geometry else None,
                     nu_cell=nu_cell, iron_box=box, iron_fraction=iron_fraction,
                     min_orient_det=min_orient, seed=seed)


def fem_mesh(s: FemSystem):
    """The tetrahedral mesh behind a generated system (needs keep_geometry).

    Returns (coords f64[npts, 3], tets int32[nelem, 4], dof int32[npts],
    nu_elem f64[nelem]): lattice points numbered x-fastest over the full
    (nx+2) x (ny+2) x (nz+2) lattice, boundary points included; dof = the
    unknown's id or -1 on the Dirichlet boundary; elements ordered as the
    generator visits them (axis permutation outer, then cells x-fastest),
    vertices (c, c + e_s0, c + e_s0 + e_s1, c + (1,1,1)); nu_elem = the
    reluctivity of each element's cell.  nelem = 6 (nx+1)(ny+1)(nz+1)."""
    if s.coords is None:
        raise ValueError("system was generated without keep_geometry")
    nx, ny, nz = s.nx, s.ny, s.nz
    coords = s.coords.reshape(-1, 3).copy()
    dof = _node_ids(nx, ny, nz).ravel().astype(np.int32)
    cz, cy, cx = nz + 1, ny + 1, nx + 1
    base = ((np.arange(cz)[:, None, None] * (ny + 2) + np.arange(cy)[None, :, None]) * (nx + 2)
            + np.arange(cx)[None, None, :]).ravel()
    stride = np.array([1, nx + 2, (nx + 2) * (ny + 2)], dtype=np.int64)
    tets = np.empty((6, base.size, 4), dtype=np.int64)
    for s_idx, perm in enumerate(PERMS):
        cur = np.zeros(3, dtype=np.int64)
        tets[s_idx, :, 0] = base
        for v, ax in enumerate(perm):
            cur[ax] += 1
            tets[s_idx, :, v + 1] = base + int(cur @ stride)
    nu_elem = np.tile(s.nu_cell.ravel(), 6)
    return coords, tets.reshape(-1, 4).astype(np.int32), dof, nu_elem


def observation(s: FemSystem):
    """x_obs ~ U(-1, 1), n values, from the fourth stream of the system's seed."""
    return _streams(s.seed)[3].uniform(-1.0, 1.0, size=s.n)


def _key_valid(nx, ny, nz):
    """valid[i, d]: node i has a neighbour at +DIRS[d] inside the interior."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    v = np.empty((i.size, 8), dtype=bool)
    for d in range(8):
        dx, dy, dz = DIRS[d]
        v[:, d] = (i + dx < nx) & (j + dy < ny) & (k + dz < nz)
    return v


def _upper_keys_to_csr(U8, nx, ny, nz):
    """Mirror the upper keys into a full, column-sorted CSR."""
    n = nx * ny * nz
    off = direction_offsets(nx, ny)
    valid = _key_valid(nx, ny, nz)
    U = U8.reshape(n, 8)
    # 15 candidate slots per row: lower (i - off_d), diagonal, upper (i + off_d)
    slot_off = np.concatenate([-off[1:], [0], off[1:]])
    order = np.argsort(slot_off, kind="stable")
    rows = np.arange(n, dtype=np.int64)
    cols = np.empty((n, 15), dtype=np.int64)
    vals = np.zeros((n, 15))
    mask = np.zeros((n, 15), dtype=bool)
    for s in range(15):
        if s < 7:                      # lower neighbour through direction d
            d = s + 1
            nb = rows - off[d]
            ok = nb >= 0
            okv = np.zeros(n, dtype=bool)
            okv[ok] = valid[nb[ok], d]
            mask[:, s] = okv
            cols[:, s] = nb
            vals[okv, s] = U[nb[okv], d]
        elif s == 7:
            mask[:, s] = True
            cols[:, s] = rows
            vals[:, s] = U[:, 0]
        else:
            d = s - 7
            mask[:, s] = valid[:, d]
            cols[:, s] = rows + off[d]
            vals[mask[:, s], s] = U[mask[:, s], d]
    cols, vals, mask = cols[:, order], vals[:, order], mask[:, order]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask]
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    return rowptr.astype(np.int32), col, val


# --------------------------------------------------------------------------
# named workloads: the synthetic configurations the path is measured on
# --------------------------------------------------------------------------
FEM_CONFIGS = {
    # paper-sized system, stored as Symmetric CSR in its measurement
    "fem32x32x30": dict(nx=32, ny=32, nz=30, nu_iron=1e-3, seed=1),
    # 1.0M unknowns, compared across CSR / Symmetric CSR / CSC
    "fem100": dict(nx=100, ny=100, nz=100, nu_iron=1e-3, seed=2),
    # 4.1M unknowns, iron contrast 1e-4
    "fem160": dict(nx=160, ny=160, nz=160, nu_iron=1e-4, seed=3),
}


def fem_config(name: str, **kw) -> FemSystem:
    args = dict(FEM_CONFIGS[name])
    args.update(kw)
    return fem_p1_system(**args)


# --------------------------------------------------------------------------
# format helpers that only move integers / copy values (no arithmetic)
# --------------------------------------------------------------------------
def upper_triangle(rowptr, col, val):
    """Entries with col >= row of a full CSR (row order kept)."""
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    keep = col >= rows
    cnt = np.bincount(rows[keep], minlength=n)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=rp[1:])
    return rp.astype(np.int32), col[keep].astype(np.int32), val[keep].copy()


def transpose_csr(n_rows, n_cols, rowptr, col, val):
    """Stable transpose (CSR of A -> CSR of A^T, i.e. CSC of A)."""
    rows = np.repeat(np.arange(n_rows), np.diff(rowptr))
    order = np.lexsort((rows, col))
    cnt = np.bincount(col, minlength=n_cols)
    cp = np.zeros(n_cols + 1, dtype=np.int64)
    np.cumsum(cnt, out=cp[1:])
    return cp.astype(np.int32), rows[order].astype(np.int32), val[order].copy()


# --------------------------------------------------------------------------
# small generic test matrices
# --------------------------------------------------------------------------
def random_sparse(n, *, density=0.05, seed=0, empty_rows=0, long_rows=0, long_len=None,
                  n_cols=None, allow_empty_cols=True):
    """Random non-symmetric sparse matrix in sorted CSR, ragged rows.

    empty_rows: number of rows with no entries; long_rows: rows with long_len
    entries (exercises the multi-pass row loop)."""
    rng = np.random.default_rng(seed)
    m = n if n_cols is None else n_cols
    lens = rng.binomial(m, density, size=n)
    if empty_rows:
        lens[rng.choice(n, size=min(empty_rows, n), replace=False)] = 0
    if long_rows:
        ll = long_len if long_len is not None else m
        lens[rng.choice(n, size=min(long_rows, n), replace=False)] = min(ll, m)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = np.empty(rowptr[-1], dtype=np.int32)
    for i in range(n):
        col[rowptr[i]:rowptr[i + 1]] = np.sort(rng.choice(m, size=lens[i], replace=False))
    val = rng.uniform(-1.0, 1.0, size=rowptr[-1])
    return rowptr.astype(np.int32), col, val


def banded_sparse(n, bw, *, density=0.01, seed=0, empty=0):
    """Random non-symmetric sparse matrix with every entry within bw of the
    diagonal (|i - j| <= bw), sorted CSR arrays (read them as CSC just as
    well); `empty` lines carry no entry.  Values ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    dead = set(rng.choice(n, size=empty, replace=False).tolist()) if empty else set()
    lines = []
    for j in range(n):
        lo, hi = max(0, j - bw), min(n, j + bw + 1)
        k = 0 if j in dead else rng.binomial(hi - lo, density)
        lines.append(np.sort(rng.choice(np.arange(lo, hi), size=k, replace=False)))
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in lines])
    idx = np.concatenate(lines).astype(np.int32)
    return ptr.astype(np.int32), idx, rng.uniform(-1.0, 1.0, size=idx.size)


def random_spd_dense(n, *, seed=0):
    """Dense SPD matrix M = B^T B + n I with B ~ U(-1,1), as full CSR."""
    rng = np.random.default_rng(seed)
    B = rng.uniform(-1.0, 1.0, size=(n, n))
    M = B.T @ B + n * np.eye(n)
    M = 0.5 * (M + M.T)                 # exact symmetry
    rowptr = (np.arange(n + 1) * n).astype(np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    return rowptr, col, M.ravel().copy(), M


def random_spd_sparse(n, *, density=0.05, seed=0):
    """Sparse SPD matrix: symmetric random pattern with values in (-1, 1) and a
    diagonal that strictly dominates each row (diag = 1 + sum |offdiag|)."""
    rng = np.random.default_rng(seed)
    k = max(1, int(density * n * n / 2))
    i = rng.integers(0, n, size=k)
    j = rng.integers(0, n, size=k)
    keep = i < j
    i, j = i[keep], j[keep]
    key = np.unique(i * n + j)
    i, j = key // n, key % n
    v = rng.uniform(-1.0, 1.0, size=i.size)
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    dvals = np.zeros(n)
    np.add.at(dvals, i, np.abs(v))
    np.add.at(dvals, j, np.abs(v))
    vals = np.concatenate([v, v, 1.0 + dvals])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals


def uniform_vector(n, *, seed=0, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def block_diagonal(systems):
    """Concatenate CSR systems [(rowptr, col, val), ...] into one block-diagonal
    CSR with global indices; returns (sys_off int64[nsys+1], rowptr, col, val).
    (Index bookkeeping only.)"""
    offs = [0]
    ptrs, cols, vals = [np.zeros(1, np.int64)], [], []
    nnz = 0
    for (rp, c, v) in systems:
        n = len(rp) - 1
        ptrs.append(np.asarray(rp[1:], dtype=np.int64) + nnz)
        cols.append(np.asarray(c, dtype=np.int64) + offs[-1])
        vals.append(np.asarray(v, dtype=np.float64))
        nnz += int(rp[-1])
        offs.append(offs[-1] + n)
    rowptr = np.concatenate(ptrs)
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    return (np.array(offs, dtype=np.int64), rowptr.astype(np.int32), np.concatenate(cols).astype(np.int32),
            np.concatenate(vals))


def fem_batch(nsys, *, lo=20, hi=60, nu_iron=1e-3, seed=4, nrhs=4, workers=1):
    """The batch workload: nsys systems of the FEM generator with interior grid
    edges drawn independently per axis, integer U{lo..hi}; system s uses the
    s-th child of SeedSequence(seed) for its own streams.  Right-hand sides
    b = A x_true for nrhs seeded x_true ~ U(-1, 1) per system (formed element
    by element).  Returns (list of FemSystem, B (N, nrhs), Xtrue (N, nrhs))."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(nsys + 1)
    dims = np.random.Generator(np.random.PCG64(kids[0])).integers(lo, hi + 1, size=(nsys, 3))
    args = [(int(d[0]), int(d[1]), int(d[2]), nu_iron, int(kids[s + 1].generate_state(1)[0]), nrhs)
            for s, d in enumerate(dims)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            out = pool.map(_batch_member, args)
    else:
        out = [_batch_member(a) for a in args]
    systems = [o[0] for o in out]
    B = np.concatenate([o[1] for o in out])
    X = np.concatenate([o[2] for o in out])
    return systems, B, X


def _batch_member(a):
    nx, ny, nz, nu, sd, nrhs = a
    s = fem_p1_system(nx, ny, nz, nu_iron=nu, seed=sd, with_rhs=True, keep_geometry=False, nrhs=nrhs)
    b = s.b.reshape(s.n, nrhs)
    x = s.x_true.reshape(s.n, nrhs)
    return (s.rowptr, s.col, s.val), b, x

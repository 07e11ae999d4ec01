"""Reading and writing sparse systems as text files (host side).

The paper's systems came as files holding the matrix in full or symmetric
(triangle) CSR form together with the vectors b and x (section III); their
exact layout is not given.  This module reads the public Matrix Market
exchange format, whose "symmetric" matrices store one triangle (L + D) with
1-based indices -- the paper's storage -- and returns the arrays cg_create
takes.  Vectors are Matrix Market "array" files (one column per right-hand
side).  Pure parsing and index bookkeeping: no solver arithmetic.

    read_matrix(path)          -> MatrixFile(n, rows, cols, vals, symmetric)
    MatrixFile.csr()           -> (rowptr, col, val)      full matrix, 0-based
    MatrixFile.csc()           -> (colptr, row, val)      full matrix by columns
    MatrixFile.upper()         -> (rowptr, col, val)      D + U by rows (CG_FMT_SYM_CSR)
    MatrixFile.lower_one_based() -> (rowptr, col, val)    L + D by rows, 1-based (CG_LOWER)
    read_vector(path)          -> ndarray (n,) or (n, k)
    write_matrix / write_vector
"""
from __future__ import annotations

import dataclasses

import numpy as np


class MatrixFileError(ValueError):
    pass


@dataclasses.dataclass
class MatrixFile:
    n: int
    rows: np.ndarray          # 0-based, as stored in the file (one triangle if symmetric)
    cols: np.ndarray
    vals: np.ndarray
    symmetric: bool

    def _csr(self, r, c, v):
        order = np.lexsort((c, r))
        r, c, v = r[order], c[order], v[order]
        if r.size > 1:
            dup = (r[1:] == r[:-1]) & (c[1:] == c[:-1])
            if np.any(dup):
                k = int(np.nonzero(dup)[0][0])
                raise MatrixFileError(f"entry ({r[k] + 1}, {c[k] + 1}) appears twice")
        ptr = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(np.bincount(r, minlength=self.n), out=ptr[1:])
        if ptr[-1] >= 2 ** 31:
            raise MatrixFileError("more than 2^31 - 1 stored entries")
        return ptr.astype(np.int32), c.astype(np.int32), v.astype(np.float64)

    def csr(self):
        """The full matrix by rows (a symmetric file is mirrored)."""
        r, c, v = self.rows, self.cols, self.vals
        if self.symmetric:
            off = r != c
            r, c, v = np.concatenate([r, c[off]]), np.concatenate([c, r[off]]), np.concatenate([v, v[off]])
        return self._csr(r, c, v)

    def csc(self):
        """The full matrix by columns (column pointers, row indices), 0-based."""
        r, c, v = self.rows, self.cols, self.vals
        if self.symmetric:
            off = r != c
            r, c, v = np.concatenate([r, c[off]]), np.concatenate([c, r[off]]), np.concatenate([v, v[off]])
        return self._csr(c, r, v)

    def _triangle(self, upper):
        r, c, v = self.rows, self.cols, self.vals
        if self.symmetric:
            # the file holds one triangle; put every entry on the requested side
            lo = np.minimum(r, c)
            hi = np.maximum(r, c)
            r, c = (lo, hi) if upper else (hi, lo)
        else:
            keep = (c >= r) if upper else (c <= r)
            r, c, v = r[keep], c[keep], v[keep]
        return self._csr(r, c, v)

    def upper(self):
        """D + U by rows, 0-based: the layout of CG_FMT_SYM_CSR."""
        return self._triangle(True)

    def lower_one_based(self):
        """L + D by rows, 1-based: the paper's symmetric storage (CG_LOWER, index_base 1)."""
        p, c, v = self._triangle(False)
        return p + 1, c + 1, v


def _header(line):
    parts = line.strip().split()
    if len(parts) < 5 or parts[0].lower() != "%%matrixmarket":
        raise MatrixFileError("not a Matrix Market file (first line must start with %%MatrixMarket)")
    return [p.lower() for p in parts[1:5]]


def _data_lines(f):
    for line in f:
        s = line.strip()
        if s and not s.startswith("%"):
            yield s


def read_matrix(path) -> MatrixFile:
    """A square real sparse matrix, `coordinate real|integer general|symmetric`."""
    with open(path) as f:
        obj, fmt, field, sym = _header(f.readline())
        if obj != "matrix" or fmt != "coordinate":
            raise MatrixFileError(f"expected a coordinate matrix, found {obj} {fmt}")
        if field not in ("real", "integer", "double"):
            raise MatrixFileError(f"unsupported field '{field}' (real or integer)")
        if sym not in ("general", "symmetric"):
            raise MatrixFileError(f"unsupported symmetry '{sym}' (general or symmetric)")
        lines = _data_lines(f)
        try:
            m, n, nnz = (int(t) for t in next(lines).split()[:3])
        except (StopIteration, ValueError):
            raise MatrixFileError("missing or malformed size line") from None
        if m != n:
            raise MatrixFileError(f"matrix is {m} x {n}, not square")
        data = np.loadtxt(lines, dtype=np.float64, ndmin=2) if nnz else np.zeros((0, 3))
    if data.shape[0] != nnz or (nnz and data.shape[1] < 3):
        raise MatrixFileError(f"expected {nnz} entries, found {data.shape[0]}")
    r = data[:, 0].astype(np.int64) - 1
    c = data[:, 1].astype(np.int64) - 1
    if nnz and (r.min() < 0 or c.min() < 0 or r.max() >= n or c.max() >= n):
        raise MatrixFileError("an index is outside 1..n")
    if nnz and (np.any(data[:, 0] != np.floor(data[:, 0])) or np.any(data[:, 1] != np.floor(data[:, 1]))):
        raise MatrixFileError("a non-integer index")
    symmetric = sym == "symmetric"
    if symmetric and nnz and not (np.all(r >= c) or np.all(r <= c)):
        raise MatrixFileError("a symmetric file must store one triangle")
    return MatrixFile(n=n, rows=r, cols=c, vals=data[:, 2].copy(), symmetric=symmetric)


def read_vector(path):
    """A dense `array real general` file: (n,) for one column, else (n, k)."""
    with open(path) as f:
        obj, fmt, field, sym = _header(f.readline())
        if obj != "matrix" or fmt != "array" or field not in ("real", "integer", "double"):
            raise MatrixFileError("expected 'matrix array real general'")
        lines = _data_lines(f)
        try:
            m, k = (int(t) for t in next(lines).split()[:2])
        except (StopIteration, ValueError):
            raise MatrixFileError("missing or malformed size line") from None
        vals = np.array([float(t) for s in lines for t in s.split()])
    if vals.size != m * k:
        raise MatrixFileError(f"expected {m * k} values, found {vals.size}")
    out = vals.reshape(k, m).T           # column-major in the file
    return out[:, 0].copy() if k == 1 else np.ascontiguousarray(out)


def write_matrix(path, n, rows, cols, vals, symmetric=False, comment=None):
    """Coordinate file from 0-based triplets (one triangle if symmetric)."""
    rows, cols, vals = np.asarray(rows), np.asarray(cols), np.asarray(vals, dtype=np.float64)
    with open(path, "w") as f:
        f.write(f"%%MatrixMarket matrix coordinate real {'symmetric' if symmetric else 'general'}\n")
        if comment:
            f.write(f"% {comment}\n")
        f.write(f"{n} {n} {rows.size}\n")
        for r, c, v in zip(rows.tolist(), cols.tolist(), vals.tolist()):
            f.write(f"{r + 1} {c + 1} {v!r}\n")


def write_vector(path, v):
    v = np.asarray(v, dtype=np.float64)
    cols = v.reshape(v.shape[0], -1)
    with open(path, "w") as f:
        f.write("%%MatrixMarket matrix array real general\n")
        f.write(f"{cols.shape[0]} {cols.shape[1]}\n")
        for j in range(cols.shape[1]):
            for x in cols[:, j].tolist():
                f.write(f"{x!r}\n")

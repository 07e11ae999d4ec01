"""GPU sparse products (CSR, symmetric CSR, CSC) through the C-ABI vs the oracle.

Bar: |y_gpu,i - y_oracle,i| <= 1e-13 * sum_j |a_ij x_j| for every row, and
||y_gpu - y_oracle|| <= 1e-13 ||y_oracle||.  (The rigorous bound for two
different summation orders of m <= 15 terms is 2 gamma_15 ~ 3.3e-15, so the
bar has a wide margin while still catching any dropped or duplicated term.)
"""
import numpy as np
import pytest

from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import check_spmv, fem_cached, say, to_dev

pytestmark = pytest.mark.gpu

CSR, SYM, CSC = cgmi.CG_FMT_CSR, cgmi.CG_FMT_SYM_CSR, cgmi.CG_FMT_CSC


def three_formats(s):
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    return {CSR: (s.rowptr, s.col, s.val), SYM: (up, uc, uv), CSC: (s.rowptr, s.col, s.val)}


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_fem_small(fmt):
    s = W.fem_p1_system(6, 5, 4, seed=11)
    x = W.uniform_vector(s.n, seed=1)
    check_spmv(fmt, *three_formats(s)[fmt], x, label="fem6x5x4")


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_fem_paper_sized(fmt):
    s = fem_cached("fem32x32x30")
    x = W.uniform_vector(s.n, seed=2)
    check_spmv(fmt, *three_formats(s)[fmt], x, label="fem32x32x30")


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_fem_full_size_1m(fmt):
    s = fem_cached("fem100")
    x = W.uniform_vector(s.n, seed=3)
    check_spmv(fmt, *three_formats(s)[fmt], x, label="fem100 (1.0M rows)")


@pytest.mark.parametrize("layout", ["rows", "slices"])
@pytest.mark.parametrize("fmt", [CSR, CSC])
def test_ragged_nonsymmetric(monkeypatch, fmt, layout):
    monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
    # empty rows/columns, lines far longer than a scatter block and than 64 lanes
    ptr, col, val = W.random_sparse(3000, density=0.004, seed=4, empty_rows=60, long_rows=3, long_len=2900)
    x = W.uniform_vector(3000, seed=5)
    check_spmv(fmt, ptr, col, val, x, label="ragged")


def test_csc_is_a_true_scatter():
    # non-symmetric arrays read as CSC must give A x with A the column reading,
    # which differs from the row reading of the same arrays
    ptr, col, val = W.random_sparse(500, density=0.02, seed=6)
    x = W.uniform_vector(500, seed=7)
    y_csc, _ = check_spmv(CSC, ptr, col, val, x, label="csc")
    y_csr, _ = check_spmv(CSR, ptr, col, val, x, label="csr")
    assert np.linalg.norm(y_csc - y_csr) > 1e-3 * np.linalg.norm(y_csr)


def test_sym_random_spd():
    ptr, col, val = W.random_spd_sparse(2000, density=0.01, seed=8)
    up, uc, uv = W.upper_triangle(ptr, col, val)
    x = W.uniform_vector(2000, seed=9)
    check_spmv(SYM, up, uc, uv, x, label="random spd")


@pytest.mark.parametrize("layout", ["rows", "slices"])
@pytest.mark.parametrize("case", ["fem_two_colours", "banded_empty_lines", "dense_row"])
def test_csc_panels(monkeypatch, case, layout):
    """CSC column panels: several panels in two colours, empty rows and
    columns, and a slot longer than a chunk (one row dense across a panel);
    slots summed by panel chunks or by slices."""
    monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
    if case == "fem_two_colours":
        s = W.fem_p1_system(30, 28, 26, seed=9)
        ptr, idx, val = s.rowptr, s.col, s.val
    elif case == "banded_empty_lines":
        ptr, idx, val = W.banded_sparse(10000, 1500, density=0.004, seed=11, empty=300)
    else:
        n = 9000
        lines = [np.array(sorted({j, 7, (j * 31) % n})) for j in range(n)]
        ptr = np.zeros(n + 1, np.int32)
        ptr[1:] = np.cumsum([c.size for c in lines])
        idx = np.concatenate(lines).astype(np.int32)
        val = W.uniform_vector(idx.size, seed=15)
    n = len(ptr) - 1
    st, P = cgmi.cg_analyze_panels(n, ptr, idx)
    assert bool(P["stats"]["slices"]) == (layout == "slices")
    say(f"panels {case}: width={P['width']} colours={P['stats']['colors']} chunks={P['stats']['scatter_blocks']}")
    check_spmv(CSC, ptr, idx, val, W.uniform_vector(n, seed=16), label=case)


@pytest.mark.parametrize("entries", ["32", "200", "2048", "9000"])
@pytest.mark.parametrize("fmt", [SYM])
def test_scatter_block_sizes(monkeypatch, fmt, entries):
    monkeypatch.setenv("CGMI_SCATTER_ENTRIES", entries)
    s = W.fem_p1_system(14, 13, 12, seed=10)
    x = W.uniform_vector(s.n, seed=11)
    check_spmv(fmt, *three_formats(s)[fmt], x, label=f"entries={entries}")


@pytest.mark.parametrize("entries", [None, "32", "200"])
def test_sym_sliced_blocks_same_bits(monkeypatch, entries):
    # the coloured plan of line ranges: its sliced blocks keep the blocks,
    # slots and summation order of the plain symmetric kernel -- identical
    # bits, and the oracle's bar (compact blocks are a different plan)
    monkeypatch.setenv("CGMI_SYM_PLAN", "colour")
    if entries:
        monkeypatch.setenv("CGMI_SCATTER_ENTRIES", entries)
    s = W.fem_p1_system(20, 18, 16, seed=25)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    x = W.uniform_vector(s.n, seed=26)
    ys = {}
    for layout in ("rows", "slices"):
        monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
        st, stats = cgmi.cg_analyze(SYM, s.n, *up)
        assert stats["slices"] == (layout == "slices")
        ys[layout], _ = check_spmv(SYM, *up, x, label=f"symcsr {layout} entries={entries}")
    assert np.array_equal(ys["rows"], ys["slices"])


@pytest.mark.parametrize("dims", [(20, 18, 16), (7, 5, 3), (1, 1, 1), (33, 2, 2)])
def test_sym_compact_vs_colour_plan(monkeypatch, dims):
    # compact blocks (the default for short lines) and coloured line ranges:
    # both within the oracle's bar, and run to run identical
    s = W.fem_p1_system(*dims, seed=29, with_rhs=False)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    x = W.uniform_vector(s.n, seed=30)
    st, stats = cgmi.cg_analyze(SYM, s.n, *up)
    assert stats["compact"] == 1
    yc, _ = check_spmv(SYM, *up, x, label=f"symcsr compact {dims}")
    yc2, _ = check_spmv(SYM, *up, x, label=f"symcsr compact {dims} again")
    assert np.array_equal(yc, yc2)
    monkeypatch.setenv("CGMI_SYM_PLAN", "colour")
    st, stats = cgmi.cg_analyze(SYM, s.n, *up)
    assert stats["compact"] == 0
    yk, yo = check_spmv(SYM, *up, x, label=f"symcsr colour {dims}")
    assert np.linalg.norm(yc - yk) <= 1e-13 * np.linalg.norm(yo)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_matrix_loads_same_bits(monkeypatch, fmt):
    # ordinary or non-temporal matrix loads: the same instructions otherwise,
    # so the same bits, for the product and for a whole solve
    s = W.fem_p1_system(20, 18, 16, seed=27)
    arrs = three_formats(s)[fmt]
    x = to_dev(W.uniform_vector(s.n, seed=28))
    b = to_dev(s.b)
    out = {}
    for mode in ("cached", "stream"):
        monkeypatch.setenv("CGMI_MATRIX_LOADS", mode)
        with cgmi.Solver(fmt, *arrs) as S:
            assert S.stats()["cached_loads"] == (mode == "cached")
            xs, info = S.solve(b, tol=1e-10, maxit=5000)
            out[mode] = (S.spmv(x).cpu().numpy(), xs.cpu().numpy(), info["iters"])
    assert np.array_equal(out["cached"][0], out["stream"][0])
    assert np.array_equal(out["cached"][1], out["stream"][1]) and out["cached"][2] == out["stream"][2]
    check_spmv(fmt, *arrs, x.cpu().numpy(), label="loads")


def test_split_long_row_symcsr(monkeypatch):
    monkeypatch.setenv("CGMI_SCATTER_ENTRIES", "32")
    n = 300
    rows = [np.arange(n)] + [np.array([i, i + 1]) if i + 1 < n else np.array([i]) for i in range(1, n)]
    ptr = np.zeros(n + 1, np.int32)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate(rows).astype(np.int32)
    val = W.uniform_vector(len(idx), seed=12) + 3.0
    check_spmv(SYM, ptr, idx, val, W.uniform_vector(n, seed=13), label="arrow")


@pytest.mark.parametrize("layout", ["rows", "slices"])
@pytest.mark.parametrize("mean_len", [2, 6, 30, 120])
def test_lane_widths(monkeypatch, mean_len, layout):
    monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
    n = 1500
    ptr, col, val = W.random_sparse(n, density=mean_len / n, seed=mean_len)
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert bool(stats["slices"]) == (layout == "slices")
    say(f"lanes={stats['lanes_per_line']} slices={stats['slices']}")
    y, yo = check_spmv(CSR, ptr, col, val, W.uniform_vector(n, seed=14), label=f"mean_len={mean_len}")
    if layout == "slices":   # every row summed left to right by one lane
        assert np.array_equal(y, yo)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_one_based(fmt):
    s = W.fem_p1_system(7, 6, 5, seed=15)
    ptr, idx, val = three_formats(s)[fmt]
    check_spmv(fmt, ptr + 1, idx + 1, val, W.uniform_vector(s.n, seed=16), base=1, label="1-based")


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_tiny_and_empty(fmt):
    check_spmv(fmt, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]), np.array([-3.0]),
               label="1x1")
    with cgmi.Solver(fmt, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0)) as S:
        assert S.n == 0
        assert S.stats()["n"] == 0
    if fmt != SYM:   # no entries at all: y = 0
        n = 70
        ptr = np.zeros(n + 1, np.int32)
        y, _ = check_spmv(fmt, ptr, np.zeros(0, np.int32), np.zeros(0), W.uniform_vector(n, seed=17),
                          label="all empty")
        assert np.all(y == 0)


@pytest.mark.parametrize("fmt", [CSR, SYM, CSC])
def test_deterministic_and_stream_ordered(fmt):
    import torch
    s = W.fem_p1_system(20, 18, 16, seed=18)
    arrs = three_formats(s)[fmt]
    x = to_dev(W.uniform_vector(s.n, seed=19))
    with cgmi.Solver(fmt, *arrs) as S:
        y1 = S.spmv(x).clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            y2 = S.spmv(x)
            y3 = y2 * 1.0              # consumes y2 on the same stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2) and torch.equal(y1, y3)


def test_errors_without_fallback():
    import torch
    s = W.fem_p1_system(4, 4, 4, seed=20)
    with cgmi.Solver(CSR, s.rowptr, s.col, s.val) as S:
        with pytest.raises(TypeError):
            S.spmv(torch.zeros(s.n, dtype=torch.float64))            # host tensor
        with pytest.raises(TypeError):
            S.spmv(torch.zeros(s.n, dtype=torch.float32, device="cuda"))
        x = to_dev(np.ones(s.n))
        assert cgmi.cg_spmv(S.h, x.data_ptr(), x.data_ptr()) == cgmi.CG_ERR_ARG   # aliased
    for bad in [(CSR, s.rowptr, s.col[::-1].copy(), s.val), (SYM, s.rowptr, s.col, s.val)]:
        st, h = cgmi.cg_create(bad[0], s.n, *bad[1:])
        assert st == cgmi.CG_ERR_STRUCTURE and h is None
    st, h = cgmi.cg_create(CSR, s.n, s.rowptr, s.col, np.full(s.nnz, np.inf))
    assert st == cgmi.CG_ERR_NONFINITE and h is None


@pytest.mark.parametrize("layout", ["auto", "rows", "slices"])
@pytest.mark.parametrize("case", ["fem32x32x30", "fem100", "ragged"])
def test_csr_bit_identical_to_oracle(monkeypatch, case, layout):
    # rows of <= 2048 entries with a mean of <= 32: the row-block kernel sums
    # each row left to right from rounded products, exactly like the oracle;
    # the sliced layout does the same in registers (any row length)
    if layout != "auto":
        monkeypatch.setenv("CGMI_ROW_LAYOUT", layout)
    if case == "ragged":
        ptr, col, val = W.random_sparse(5000, density=0.003, seed=21, empty_rows=40, long_rows=2, long_len=1500)
    else:
        s = fem_cached(case)
        ptr, col, val = s.rowptr, s.col, s.val
    st, stats = cgmi.cg_analyze(CSR, len(ptr) - 1, ptr, col, val)
    assert st == 0
    say(f"layout={layout} slices={stats['slices']} workgroups={stats['spmv_blocks']}")
    y, yo = check_spmv(CSR, ptr, col, val, W.uniform_vector(len(ptr) - 1, seed=22), label=f"bitwise {case}")
    assert np.array_equal(y, yo)


@pytest.mark.parametrize("col16", ["1", "0"])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 4097])
def test_csr_slices_ragged_shapes(monkeypatch, n, col16):
    # partial last slice, empty rows, one row far longer than the rest; the
    # columns as 16-bit offsets from the row (every column is within 32767
    # here) or as 32-bit indices
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "slices")
    monkeypatch.setenv("CGMI_COL16", col16)
    ptr, col, val = W.random_sparse(n, density=min(1.0, 9.0 / n), seed=n, empty_rows=n // 7,
                                    long_rows=1 if n > 1 else 0, long_len=min(n, 700))
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert st == 0 and stats["slices"] == (2 if col16 == "1" else 1)
    y, yo = check_spmv(CSR, ptr, col, val, W.uniform_vector(n, seed=n + 1), label=f"slices n={n}")
    assert np.array_equal(y, yo)


@pytest.mark.parametrize("fmt", ["csr", "csc"])
def test_col16_same_bits_and_fallback(monkeypatch, fmt):
    """CSR slices / CSC panel-slot slices with 16-bit column offsets against
    32-bit columns: the same products and CG iterates bit for bit (only the
    storage of the columns differs), and a matrix with a column farther than
    32767 from its row keeps 32-bit columns."""
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "slices")
    f = cgmi.FORMATS[fmt]
    s = W.fem_p1_system(20, 18, 16, seed=27)
    x = W.uniform_vector(s.n, seed=28)
    ys, xs = {}, {}
    for col16 in ("1", "0"):
        monkeypatch.setenv("CGMI_COL16", col16)
        st, stats = cgmi.cg_analyze(f, s.n, s.rowptr, s.col, s.val)
        assert st == 0 and stats["slices"] == (2 if col16 == "1" else 1)
        ys[col16], _ = check_spmv(f, s.rowptr, s.col, s.val, x, label=f"fem {fmt} col16={col16}")
        with cgmi.Solver(fmt, s.rowptr, s.col, s.val) as S:
            xg, info = S.solve(to_dev(s.b), tol=1e-10, maxit=5000)
            xs[col16] = (xg.cpu().numpy(), info["iters"])
    assert np.array_equal(ys["1"], ys["0"])
    assert np.array_equal(xs["1"][0], xs["0"][0]) and xs["1"][1] == xs["0"][1]
    monkeypatch.delenv("CGMI_COL16")
    if fmt == "csc":
        return
    n = 40000
    ptr, col, val = W.random_sparse(n, density=9.0 / n, seed=29)
    assert np.max(np.abs(col - np.repeat(np.arange(n), np.diff(ptr)))) > 32767
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert st == 0 and stats["slices"] == 1
    y, yo = check_spmv(CSR, ptr, col, val, W.uniform_vector(n, seed=30), label="wide band, 32-bit columns")
    assert np.array_equal(y, yo)


def test_csr_slices_several_per_wave():
    # 51 563 slices on 8192 workgroups: waves take two slices at a time, and
    # the product leaves 8192 dot partials
    n = 3_300_000
    ptr = np.zeros(n + 1, np.int32)
    lens = np.full(n, 3)
    lens[0] = lens[-1] = 2
    ptr[1:] = np.cumsum(lens)
    i = np.repeat(np.arange(n), lens)
    off = np.arange(ptr[-1]) - ptr[i] - (i > 0)
    col = (i + off).astype(np.int32)
    val = np.where(col == i, 2.0, -1.0) + 1e-3 * W.uniform_vector(ptr[-1], seed=30)
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert st == 0 and stats["slices"] == 2 and stats["spmv_blocks"] == 8192
    y, yo = check_spmv(CSR, ptr, col, val, W.uniform_vector(n, seed=31), label="3.3M rows, 3 per row")
    assert np.array_equal(y, yo)


def test_lower_triangle_input_matches_full_product():
    import scipy.sparse as sp
    s = W.fem_p1_system(9, 8, 7, seed=23)
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    L = sp.tril(A, format="csr")
    L.sort_indices()
    x = W.uniform_vector(s.n, seed=24)
    with cgmi.Solver(SYM, L.indptr.astype(np.int32) + 1, L.indices.astype(np.int32) + 1, L.data, index_base=1,
                     flags=cgmi.CG_LOWER) as S:
        y = S.spmv(to_dev(x)).cpu().numpy()
    import oracle
    yo = oracle.spmv(CSR, s.rowptr, s.col, s.val, x)
    assert np.all(np.abs(y - yo) <= 1e-13 * oracle.spmv(CSR, s.rowptr, s.col, np.abs(s.val), np.abs(x)))

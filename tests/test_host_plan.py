"""Host logic of the HIP library, checked on the CPU (no GPU calls).

* the shared library loads and exports every function include/cgmi.h declares;
* cg_analyze validates exactly as the oracle does (same status per case);
* the scatter plan (blocks, write slots, colours, first/last flags,
  contribution counts) is re-derived here from the matrix and compared.
"""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "cgmi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = cgmi.load()
    declared = header_functions()
    assert set(declared) == set(cgmi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    for st in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert cgmi.cg_status_string(st) != "unknown status"
    assert cgmi.cg_status_string(99) == "unknown status"


@pytest.mark.parametrize("case", pins.malformed_cases(), ids=lambda c: c[0])
def test_validation_matches_oracle(case):
    name, fmt, p, i, v, base, flags, want = case
    st, _ = cgmi.cg_analyze(fmt, len(p) - 1, p, i, v, base, flags)
    assert st == want == oracle.validate(fmt, p, i, v, base=base, flags=flags), (name, st)
    if st != 0:
        assert cgmi.cg_last_error(None) != ""


def test_null_and_empty_arguments():
    st, s = cgmi.cg_analyze(0, 0, None, None, None)
    assert st == 0 and s["n"] == 0
    st, _ = cgmi.cg_analyze(0, 3, None, None, None)
    assert st == cgmi.CG_ERR_ARG
    st, _ = cgmi.cg_analyze(0, -1, None, None, None)
    assert st == cgmi.CG_ERR_ARG
    st, _ = cgmi.cg_analyze(0, 2, np.array([0, 1, 2]), None, None)
    assert st == cgmi.CG_ERR_ARG


def test_csr_plan_shape():
    s = W.fem_config("fem32x32x30")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSR, s.n, s.rowptr, s.col, s.val)
    assert st == 0
    assert stats["lanes_per_line"] == 16          # ~14.25 entries per row
    assert stats["colors"] == 0 and stats["slots"] == 0
    assert 1 <= stats["spmv_blocks"] <= 8192 and 1 <= stats["vec_blocks"] <= 1024


def _slice_positions(ptr):
    # positions of the sliced layout: every 64-row slice padded to its longest row
    lens = np.diff(np.asarray(ptr, dtype=np.int64))
    ns = (lens.size + 63) // 64
    full = np.zeros(ns * 64, dtype=np.int64)
    full[:lens.size] = lens
    return int(full.reshape(ns, 64).max(axis=1).sum()) * 64, ns


def test_csr_layout_choice(monkeypatch):
    CSR = cgmi.CG_FMT_CSR
    # FEM rows differ little in length: sliced layout, padding within 12.5 %
    # (columns within 32767 of their rows: 16-bit offsets, 14 bytes a position
    # with the entry source and the value; else 32-bit columns, 16 bytes)
    s = W.fem_config("fem32x32x30")
    st, stats = cgmi.cg_analyze(CSR, s.n, s.rowptr, s.col, s.val)
    pos, ns = _slice_positions(s.rowptr)
    assert st == 0 and stats["slices"] == 2
    assert s.nnz <= pos <= 1.125 * s.nnz
    assert stats["plan_bytes"] == 4 * (ns + 1) + 14 * pos
    assert stats["spmv_blocks"] == min((ns + 3) // 4, 8192)
    monkeypatch.setenv("CGMI_COL16", "0")
    st, stats = cgmi.cg_analyze(CSR, s.n, s.rowptr, s.col, s.val)
    assert st == 0 and stats["slices"] == 1 and stats["plan_bytes"] == 4 * (ns + 1) + 16 * pos
    monkeypatch.delenv("CGMI_COL16")
    # one column 32768 away from its row: 32-bit columns
    n = 40000
    ptr = np.arange(n + 1, dtype=np.int32)
    ptr[-1] = n + 1  # the last row holds two entries: columns n - 32769 and n - 1
    col = np.insert(np.arange(n, dtype=np.int32), n - 1, n - 1 - 32768).astype(np.int32)
    val = np.ones(n + 1)
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert st == 0 and stats["slices"] == 1
    col[n - 1] = n - 1 - 32767  # 32767 away: still 16-bit
    st, stats = cgmi.cg_analyze(CSR, n, ptr, col, val)
    assert st == 0 and stats["slices"] == 2
    # two 1500-entry rows among ~15-entry rows: padding too large, row blocks
    ptr, col, val = W.random_sparse(5000, density=0.003, seed=21, empty_rows=40, long_rows=2, long_len=1500)
    st, stats = cgmi.cg_analyze(CSR, 5000, ptr, col, val)
    assert st == 0 and stats["slices"] == 0 and stats["plan_bytes"] < 5000
    # the knob forces either layout
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "slices")
    st, stats = cgmi.cg_analyze(CSR, 5000, ptr, col, val)
    pos, ns = _slice_positions(ptr)
    assert st == 0 and stats["slices"] == 2 and stats["plan_bytes"] == 4 * (ns + 1) + 14 * pos
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "rows")
    st, stats = cgmi.cg_analyze(CSR, s.n, s.rowptr, s.col, s.val)
    assert st == 0 and stats["slices"] == 0
    # CSC: slices over the panel slots (their segments are the lines)
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSC, s.n, s.rowptr, s.col, s.val)
    assert st == 0 and stats["slices"] == 0
    monkeypatch.delenv("CGMI_ROW_LAYOUT")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSC, s.n, s.rowptr, s.col, s.val)
    st2, P = cgmi.cg_analyze_panels(s.n, s.rowptr, s.col)
    pos, ns = _slice_positions(P["slot_ptr"])
    assert st == 0 and stats["slices"] == 2 and stats["spmv_blocks"] == min((ns + 3) // 4, 8192)
    assert s.nnz <= pos <= 1.125 * s.nnz
    # symmetric CSR: sliced blocks when no stored line has more than 8
    # entries (FEM upper triangle: the diagonal and 7 neighbours at most)
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    assert np.diff(up[0]).max() <= 8
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, *up)
    assert st == 0 and stats["slices"] == 1
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "rows")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, *up)
    assert st == 0 and stats["slices"] == 0
    monkeypatch.delenv("CGMI_ROW_LAYOUT")
    ptr, col, val = W.random_spd_sparse(2000, density=0.01, seed=8)
    up = W.upper_triangle(ptr, col, val)
    assert np.diff(up[0]).max() > 8
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, 2000, *up)
    assert st == 0 and stats["slices"] == 0


def test_matrix_loads_choice(monkeypatch):
    # ordinary (Infinity-Cache-resident) matrix loads while one iteration's
    # bytes stay below 336 MiB, non-temporal above; the knob forces either
    s = W.fem_config("fem32x32x30")
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    for fmt, arrs in ((cgmi.CG_FMT_CSR, (s.rowptr, s.col, s.val)), (cgmi.CG_FMT_SYM_CSR, up),
                      (cgmi.CG_FMT_CSC, (s.rowptr, s.col, s.val))):
        st, stats = cgmi.cg_analyze(fmt, s.n, *arrs)
        assert st == 0 and stats["slices"] >= 1 and stats["cached_loads"] == 1
    n = 5_500_000                      # tridiagonal: 16.5 M positions, 165 MB + 40 B per row > 336 MiB
    lens = np.full(n, 3)
    lens[0] = lens[-1] = 2
    ptr = np.zeros(n + 1, np.int32)
    ptr[1:] = np.cumsum(lens)
    i = np.repeat(np.arange(n), lens)
    col = (i + np.arange(ptr[-1]) - ptr[i] - (i > 0)).astype(np.int32)
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSR, n, ptr, col, None)
    assert st == 0 and stats["slices"] == 2 and stats["cached_loads"] == 0
    monkeypatch.setenv("CGMI_MATRIX_LOADS", "cached")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSR, n, ptr, col, None)
    assert st == 0 and stats["cached_loads"] == 1
    monkeypatch.setenv("CGMI_MATRIX_LOADS", "stream")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSR, s.n, s.rowptr, s.col, s.val)
    assert st == 0 and stats["cached_loads"] == 0
    monkeypatch.setenv("CGMI_ROW_LAYOUT", "rows")          # only the sliced kernels have the choice
    monkeypatch.setenv("CGMI_MATRIX_LOADS", "cached")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_CSR, s.n, s.rowptr, s.col, s.val)
    assert st == 0 and stats["slices"] == 0 and stats["cached_loads"] == 0


def _expected_targets(fmt, ptr, idx, e0, e1, l0, l1):
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))[e0:e1]
    cols = idx[e0:e1]
    if fmt == cgmi.CG_FMT_SYM_CSR:
        off = cols != rows
        contrib = cols[off]                        # mirror products land on column index
        return set(range(l0, l1)) | set(contrib.tolist()), contrib
    return set(cols.tolist()), cols


def check_scatter_plan(fmt, ptr, idx):
    n = len(ptr) - 1
    st, P = cgmi.cg_analyze_export(fmt, n, ptr, idx)
    assert st == 0, cgmi.cg_last_error(None)
    nb = P["stats"]["scatter_blocks"]
    assert P["stats"]["colors"] == P["color"].max() + 1
    # blocks tile the lines and the entries contiguously (a long line may be split)
    assert P["line0"][0] == 0 and P["line1"][-1] == n
    assert P["entry0"][0] == 0 and P["entry1"][-1] == ptr[-1]
    assert np.all(P["entry0"][1:] == P["entry1"][:-1])
    assert np.all(P["line0"][1:] >= P["line0"][:-1]) and np.all(P["line1"] > P["line0"])
    for b in range(nb):
        assert ptr[P["line0"][b]] <= P["entry0"][b] and P["entry1"][b] <= ptr[P["line1"][b]]
    writers = {}
    for b in range(nb):
        s0, s1 = P["slot0"][b], P["slot0"][b + 1]
        tg = P["target"][s0:s1]
        assert len(set(tg.tolist())) == len(tg), "duplicate slot in a block"
        exp, contrib = _expected_targets(fmt, ptr, idx, P["entry0"][b], P["entry1"][b], P["line0"][b],
                                         P["line1"][b])
        extra = set(tg.tolist()) - exp
        assert exp <= set(tg.tolist())
        # extra slots only for rows that no entry at all writes (empty rows, CSC)
        for r in extra:
            assert fmt == cgmi.CG_FMT_CSC and not np.any(idx == r)
        cnt = dict(zip(*np.unique(contrib, return_counts=True)))
        for t, c in zip(tg, P["count"][s0:s1]):
            assert c == cnt.get(t, 0)
        for t in tg:
            writers.setdefault(int(t), []).append(b)
    assert set(writers) == set(range(n)), "a row of y is never written"
    for t, bs in writers.items():
        cols = [P["color"][b] for b in bs]
        assert len(set(cols)) == len(cols), f"row {t} written twice in one colour"
    # first / last writer flags
    for b in range(nb):
        s0, s1 = P["slot0"][b], P["slot0"][b + 1]
        for t, f in zip(P["target"][s0:s1], P["flags"][s0:s1]):
            cols = [P["color"][bb] for bb in writers[int(t)]]
            assert bool(f & 1) == (P["color"][b] == min(cols))
            assert bool(f & 2) == (P["color"][b] == max(cols))
    return P


def test_scatter_plan_fem_symcsr(monkeypatch):
    monkeypatch.setenv("CGMI_SYM_PLAN", "colour")   # the coloured plan of contiguous line ranges
    s = W.fem_p1_system(12, 10, 9, seed=3)
    up, uc, _ = W.upper_triangle(s.rowptr, s.col, s.val)
    P = check_scatter_plan(cgmi.CG_FMT_SYM_CSR, up, uc)
    assert P["stats"]["colors"] <= 8 and P["stats"]["compact"] == 0


def check_compact_plan(ptr, idx, base=0):
    """Re-derives the compact-block plan of a symmetric (upper) matrix from
    its block assignment and compares every slot and count."""
    n = len(ptr) - 1
    st, P = cgmi.cg_analyze_compact(n, ptr, idx, base)
    assert st == 0, cgmi.cg_last_error(None)
    p0 = np.asarray(ptr, np.int64) - base
    i0 = np.asarray(idx, np.int64) - base
    rows = np.repeat(np.arange(n), np.diff(p0))
    bo = P["block_of"]
    nb = P["stats"]["scatter_blocks"]
    assert P["stats"]["compact"] == 1 and P["stats"]["colors"] == 1
    assert bo.min() == 0 and bo.max() == nb - 1
    sizes = np.bincount(bo, minlength=nb)
    assert np.array_equal(sizes, P["lines"]) and sizes.max() <= 512 and sizes.min() >= 1
    # blocks are numbered by their lowest row
    firsts = np.array([np.flatnonzero(bo == b)[0] for b in range(nb)])
    assert np.all(np.diff(firsts) > 0)
    off = rows != i0
    mir_src, mir_dst = rows[off], i0[off]          # mirrored product of (i, j) lands on row j
    own_rows = set()
    parked = 0
    for b in range(nb):
        s0, s1 = P["slot0"][b], P["slot0"][b + 1]
        tg, cnt = P["target"][s0:s1], P["count"][s0:s1]
        mine = np.flatnonzero(bo == b)
        nl = mine.size
        assert np.array_equal(tg[:nl], mine), "own rows first, ascending"
        sel = bo[mir_src] == b
        dst = mir_dst[sel]
        outside = np.unique(dst[bo[dst] != b])
        assert np.array_equal(tg[nl:], outside), "parked slots = rows outside reached by its mirrors"
        want = dict(zip(*np.unique(dst, return_counts=True)))
        assert all(c == want.get(t, 0) for t, c in zip(tg.tolist(), cnt.tolist()))
        own_rows |= set(mine.tolist())
        parked += outside.size
        # every block is connected in the graph of A
        adj = {}
        for a_, c_ in zip(rows[off].tolist(), i0[off].tolist()):
            if bo[a_] == b and bo[c_] == b:
                adj.setdefault(a_, []).append(c_)
                adj.setdefault(c_, []).append(a_)
        seen, todo = {int(mine[0])}, [int(mine[0])]
        while todo:
            for c_ in adj.get(todo.pop(), []):
                if c_ not in seen:
                    seen.add(c_)
                    todo.append(c_)
        assert seen == set(mine.tolist()), f"block {b} is not connected"
    assert own_rows == set(range(n))
    assert parked == P["stats"]["parked"] and P["stats"]["slots"] == n + parked
    return P


def test_compact_plan_fem_symcsr():
    s = W.fem_p1_system(12, 10, 9, seed=3)
    up, uc, _ = W.upper_triangle(s.rowptr, s.col, s.val)
    P = check_compact_plan(up, uc)
    assert P["stats"]["parked"] <= 1.2 * s.n   # contiguous 256-row ranges park ~2x more here


def test_compact_plan_fewer_parked_than_line_ranges(monkeypatch):
    # a 40^3 grid: compact blocks park under half of what line ranges need
    s = W.fem_p1_system(40, 40, 40, seed=4, with_rhs=False)
    up, uc, _ = W.upper_triangle(s.rowptr, s.col, s.val)
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, up, uc, None)
    assert st == 0 and stats["compact"] == 1
    monkeypatch.setenv("CGMI_SYM_PLAN", "colour")
    st, P = cgmi.cg_analyze_export(cgmi.CG_FMT_SYM_CSR, s.n, up, uc)
    assert st == 0
    colour_parked = int(np.sum(P["color"][np.searchsorted(P["slot0"], np.arange(P["stats"]["slots"]),
                                                           side="right") - 1] > 0))
    assert stats["parked"] < 0.5 * colour_parked, (stats["parked"], colour_parked)


def test_compact_plan_ragged_and_one_based():
    # random SPD pattern with rows of at most 8 stored entries, 1-based input
    ptr, col, val = W.random_spd_sparse(900, density=0.004, seed=5)
    up, uc, uv = W.upper_triangle(ptr, col, val)
    assert np.diff(up).max() <= 8
    P0 = check_compact_plan(up, uc)
    st, P1 = cgmi.cg_analyze_compact(900, up + 1, uc + 1, 1)
    assert st == 0
    for k in ("block_of", "slot0", "target", "count"):
        assert np.array_equal(P0[k], P1[k])


def test_compact_plan_refused_for_long_rows():
    up, uc = _arrow_upper(50)                      # row 0 has 50 entries: coloured plan
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, 50, up, uc, None)
    assert st == 0 and stats["compact"] == 0
    st, _ = cgmi.cg_analyze_compact(50, up, uc)
    assert st == cgmi.CG_ERR_ARG


def check_panel_plan(ptr, idx, base=0):
    """Re-derives the CSC column-panel plan from the arrays and compares."""
    n = len(ptr) - 1
    st, P = cgmi.cg_analyze_panels(n, ptr, idx, base)
    assert st == 0, cgmi.cg_last_error(None)
    p0 = np.asarray(ptr, np.int64) - base
    i0 = np.asarray(idx, np.int64) - base
    nnz = int(p0[-1])
    col_of = np.repeat(np.arange(n), np.diff(p0))             # column of each stored entry
    bw = int(np.max(np.abs(i0 - col_of))) if nnz else 0
    W = P["width"]
    assert W >= min(n, 2 * bw + 1) and W >= min(n, 4096)
    src = P["entry_src"]
    assert np.array_equal(np.sort(src), np.arange(nnz)), "entries lost or duplicated"
    rows, cols = i0[src], col_of[src]
    ns = P["target"].size
    sp = P["slot_ptr"]
    assert sp[0] == 0 and sp[-1] == nnz and np.all(np.diff(sp) > 0)
    seen = set()
    for s_ in range(ns):
        seg = slice(sp[s_], sp[s_ + 1])
        pk = int(P["panel"][s_])
        assert np.all(rows[seg] == P["target"][s_])
        assert np.all(cols[seg] // W == pk)
        assert np.all(np.diff(cols[seg]) > 0), "segment not in ascending column order"
        key = (pk, int(P["target"][s_]))
        assert key not in seen
        seen.add(key)
    # every (panel, row) pair with entries is exactly one slot
    assert seen == set(zip((col_of // W).tolist(), i0.tolist()))
    # colour 0 = even panels first, then odd; same-colour panels never share a row
    fp = P["first_parked"]
    assert np.all(P["panel"][:fp] % 2 == 0) and np.all(P["panel"][fp:] % 2 == 1)
    for colour in (0, 1):
        tg = P["target"][:fp] if colour == 0 else P["target"][fp:]
        assert len(set(tg.tolist())) == tg.size, f"row written twice in colour {colour}"
    # chunks tile the slots: <= 2048 entries and <= 256 slots, or one long slot
    cs = P["chunk_slot"]
    assert cs[0] == 0 and cs[-1] == ns and np.all(np.diff(cs) > 0)
    for c in range(cs.size - 1):
        ne = sp[cs[c + 1]] - sp[cs[c]]
        assert (ne <= 2048 and cs[c + 1] - cs[c] <= 256) or cs[c + 1] - cs[c] == 1
    assert P["stats"]["scatter_blocks"] == cs.size - 1 and P["stats"]["slots"] == ns
    return P


def test_panel_plan_fem_csc():
    s = W.fem_p1_system(12, 10, 9, seed=3)
    P = check_panel_plan(s.rowptr, s.col)                     # symmetric: CSC arrays == CSR arrays
    assert P["stats"]["colors"] == 1                          # n = 1080 < 4096 columns: one panel


def test_panel_plan_fem_two_colours():
    s = W.fem_p1_system(30, 28, 26, seed=9)                   # n = 21 840, bw = 871
    P = check_panel_plan(s.rowptr, s.col)
    assert P["width"] == 4096 and P["stats"]["colors"] == 2 and P["first_parked"] < P["target"].size


def test_panel_plan_wide_band():
    s = W.fem_p1_system(70, 70, 8, seed=10)                   # bw = 4971 > 4096/2: width = 2 bw + 1
    P = check_panel_plan(s.rowptr, s.col)
    assert P["width"] == 2 * (70 * 70 + 70 + 1) + 1


def test_panel_plan_ragged_nonsymmetric_csc():
    ptr, col, val = W.random_sparse(300, density=0.03, seed=5, empty_rows=20, long_rows=2, long_len=250)
    # read as CSC arrays: 2 columns of 250 entries, 20 empty columns; rows without entries exist too
    check_panel_plan(ptr, col)
    one = check_panel_plan(ptr + 1, col + 1, base=1)
    assert one["target"].size > 0


def test_panel_plan_banded_multi_panel():
    ptr, idx, _ = W.banded_sparse(10000, 1500, density=0.004, seed=11, empty=300)
    P = check_panel_plan(ptr, idx)
    assert P["width"] == 4096 and P["stats"]["colors"] == 2


def test_panel_plan_long_slot_and_banded():
    # a column panel holding one row with 3000 entries (a dense row): its slot is a chunk of its own
    n = 5000
    cols = [[j] for j in range(n)]
    for j in range(n):
        if j != 7:
            cols[j] = sorted(set(cols[j] + [7]))
    ptr = np.zeros(n + 1, np.int32)
    ptr[1:] = np.cumsum([len(c) for c in cols])
    idx = np.concatenate([np.array(c) for c in cols]).astype(np.int32)
    P = check_panel_plan(ptr, idx)
    lens = np.diff(P["slot_ptr"])
    assert lens.max() == n and P["stats"]["max_block_entries"] == n


def test_panel_width_override(monkeypatch):
    s = W.fem_p1_system(30, 28, 26, seed=9)
    monkeypatch.setenv("CGMI_PANEL_WIDTH", "9000")
    P = check_panel_plan(s.rowptr, s.col)
    assert P["width"] == 9000 and P["stats"]["colors"] == 2
    monkeypatch.setenv("CGMI_PANEL_WIDTH", "10")                # never below 2 bw + 1 / 4096
    assert check_panel_plan(s.rowptr, s.col)["width"] == 4096
    monkeypatch.setenv("CGMI_PANEL_WIDTH", str(s.n))            # one panel: one colour, nothing parked
    P = check_panel_plan(s.rowptr, s.col)
    assert P["stats"]["colors"] == 1 and P["first_parked"] == P["target"].size == s.n


def test_analyze_export_refuses_csc():
    s = W.fem_p1_system(4, 4, 4, seed=1)
    st, _ = cgmi.cg_analyze_export(cgmi.CG_FMT_CSC, s.n, s.rowptr, s.col)
    assert st == cgmi.CG_ERR_ARG and "panel" in cgmi.cg_last_error(None)


def _arrow_upper(n):
    """Upper triangle of an arrow matrix: row 0 couples to every column,
    the other rows to their right neighbour."""
    rows = [np.arange(n)] + [np.array([i, i + 1]) if i + 1 < n else np.array([i]) for i in range(1, n)]
    ptr = np.zeros(n + 1, np.int32)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    return ptr, np.concatenate(rows).astype(np.int32)


def test_scatter_plan_long_rows_symcsr(monkeypatch):
    monkeypatch.setenv("CGMI_SCATTER_ENTRIES", "32")
    up, uc = _arrow_upper(200)
    P = check_scatter_plan(cgmi.CG_FMT_SYM_CSR, up, uc)
    split = [b for b in range(P["stats"]["scatter_blocks"]) if P["line0"][b] == 0 and P["line1"][b] == 1]
    assert len(split) == 7                         # 200 entries of row 0 in blocks of 32


def test_scatter_plan_too_many_colours_is_an_error(monkeypatch):
    monkeypatch.setenv("CGMI_SCATTER_ENTRIES", "32")
    up, uc = _arrow_upper(4000)                   # 125 pieces of row 0 all write y_0
    st, _ = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, 4000, up, uc)
    assert st == cgmi.CG_ERR_UNSUPPORTED and "colours" in cgmi.cg_last_error(None)


def test_one_based_input_same_plan(monkeypatch):
    monkeypatch.setenv("CGMI_SYM_PLAN", "colour")
    s = W.fem_p1_system(6, 5, 4, seed=7)
    up, uc, _ = W.upper_triangle(s.rowptr, s.col, s.val)
    st0, P0 = cgmi.cg_analyze_export(cgmi.CG_FMT_SYM_CSR, s.n, up, uc, 0)
    st1, P1 = cgmi.cg_analyze_export(cgmi.CG_FMT_SYM_CSR, s.n, up + 1, uc + 1, 1)
    assert st0 == st1 == 0
    for k in ("color", "target", "flags", "count", "slot0"):
        assert np.array_equal(P0[k], P1[k])


def _lower_arrays(s):
    import scipy.sparse as sp
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    L = sp.tril(A, format="csr")
    L.sort_indices()
    return L.indptr.astype(np.int32), L.indices.astype(np.int32), L.data.copy()


def test_lower_triangle_input_paper_storage():
    # the paper stores L + D by rows, 1-based; CG_LOWER accepts exactly that
    s = W.fem_p1_system(6, 5, 4, seed=8)
    lp, lc, lv = _lower_arrays(s)
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, lp + 1, lc + 1, lv, 1, cgmi.CG_LOWER)
    assert st == 0 and stats["nnz"] == len(lc)
    up, uc, uv = W.upper_triangle(s.rowptr, s.col, s.val)
    st_up, stats_up = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, up, uc, uv)
    assert stats["colors"] == stats_up["colors"] and stats["slots"] == stats_up["slots"]
    # without the flag the lower layout is malformed, and upper arrays are malformed with it
    assert cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, lp, lc, lv)[0] == cgmi.CG_ERR_STRUCTURE
    assert cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, up, uc, uv, 0, cgmi.CG_LOWER)[0] == cgmi.CG_ERR_STRUCTURE


def test_batch_create_validation_on_host():
    # structure errors are reported before any device work
    s1 = W.fem_p1_system(3, 3, 2, seed=1)
    s2 = W.fem_p1_system(2, 2, 2, seed=2)
    so, ptr, col, val = W.block_diagonal([(s1.rowptr, s1.col, s1.val), (s2.rowptr, s2.col, s2.val)])
    bad = col.copy()
    bad[0] = so[1]                       # row 0 of system 0 couples into system 1 (unsorted too)
    st, h = cgmi.cg_batch_create(so, ptr, np.sort(bad[:ptr[1]]).tolist() + bad[ptr[1]:].tolist(), val)
    assert st == cgmi.CG_ERR_STRUCTURE and h is None and "another system" in cgmi.cg_batch_last_error(None)
    st, h = cgmi.cg_batch_create(np.array([0, 5, 5, so[-1]]), ptr, col, val)
    assert st == cgmi.CG_ERR_STRUCTURE
    st, h = cgmi.cg_batch_create(so, ptr, col, val, nrhs=3)
    assert st == cgmi.CG_ERR_ARG


def test_block_diagonal_helper():
    s1 = W.fem_p1_system(3, 3, 2, seed=1)
    s2 = W.fem_p1_system(2, 2, 2, seed=2)
    so, ptr, col, val = W.block_diagonal([(s1.rowptr, s1.col, s1.val), (s2.rowptr, s2.col, s2.val)])
    assert list(so) == [0, s1.n, s1.n + s2.n]
    assert ptr[-1] == s1.nnz + s2.nnz and col[ptr[s1.n]] >= s1.n


@pytest.mark.sym_expanded
def test_sym_expanded_plan_choice(monkeypatch):
    # small symmetric systems (vector kernels of <= 256 workgroups): the
    # triangle expanded into full rows, sliced like CSR -- the same positions
    # and bytes as the CSR plan of the full matrix; larger ones keep the
    # compact blocks; CGMI_SYM_EXPAND=0 keeps them on small ones too
    s = W.fem_config("fem32x32x30")
    up = W.upper_triangle(s.rowptr, s.col, s.val)
    st, sym = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, *up)
    st2, csr = cgmi.cg_analyze(cgmi.CG_FMT_CSR, s.n, s.rowptr, s.col, s.val)
    assert st == st2 == 0 and sym["compact"] == 0 and sym["slices"] == 2 and sym["parked"] == 0
    assert sym["plan_bytes"] == csr["plan_bytes"] and sym["spmv_blocks"] == csr["spmv_blocks"]
    big = W.fem_p1_system(42, 42, 40, seed=3)
    ub = W.upper_triangle(big.rowptr, big.col, big.val)
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, big.n, *ub)
    assert st == 0 and big.n > 65536 and stats["compact"] == 1
    monkeypatch.setenv("CGMI_SYM_EXPAND", "0")
    st, stats = cgmi.cg_analyze(cgmi.CG_FMT_SYM_CSR, s.n, *up)
    assert st == 0 and stats["compact"] == 1

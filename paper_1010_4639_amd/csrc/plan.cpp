// Host planner: validation and the coloured scatter plan (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "../../include/cgmi.h"

namespace cgmi {

int64_t Plan::device_bytes() const
{
    // slices: offsets + entry source, column (or 16-bit offset), value per position
    const int64_t sl = (int64_t)sl_off.size() * 4 + (int64_t)sl_src.size() * (4 + (sl_d16.empty() ? 4 : 2) + 8);
    if (format == kCsr || sym_expanded) // row-block starts or slices
        return (int64_t)csr_rb.size() * 4 + sl;
    if (panel && slices) // slices; slot targets; parked sums and flags by row
        return sl + (int64_t)pn_slot_target.size() * 4 + n * 9;
    if (panel) // entry source + column + reordered value; slot target / pointer; chunks; parked sums, flags
        return nnz * (4 + 4 + 8) + (int64_t)pn_slot_target.size() * (4 + 4) + (int64_t)pn_chunk_slot.size() * 4 +
               n * 9;
    if (sym_compact) // descriptors; slot targets, slot starts; LDS ranks; parked sums, their per-row
                     // lists; positions (source, column, value)
        return (int64_t)cp_blocks.size() * sizeof(CompactBlock) + (int64_t)slot_target.size() * 4 +
               (int64_t)seg.size() * 2 + (int64_t)cp_rank.size() * 2 + cp_parked * (8 + 4) + (n + 1) * 4 +
               (int64_t)ss_src.size() * (4 + 4 + 8);
    // descriptors, slot target / flag / segment offsets, contributions, parked
    // sums and their per-row index (upper bounds: every slot counted); sliced
    // blocks: positions (source, column, value) and their block offsets
    return (int64_t)blocks.size() * sizeof(ScatterBlock) + (int64_t)slot_target.size() * (4 + 1 + 8 + 4) +
           (int64_t)seg.size() * 2 + (int64_t)tl.size() * 2 + n * 5 + (int64_t)ss_pos.size() * 8 +
           (int64_t)ss_src.size() * (4 + 4 + 8);
}

int64_t Plan::slice_stream_bytes() const
{
    if (slices) // positions, slice offsets; CSC: slot targets, parked sums written and read
        return (int64_t)sl_src.size() * (sl_d16.empty() ? 12 : 10) + (int64_t)sl_off.size() * 4 +
               (panel ? (int64_t)pn_slot_target.size() * 4 + n * 17 : 0);
    if (sym_compact) // positions; slot targets, starts; LDS ranks; parked sums written and read, row lists
        return (int64_t)ss_src.size() * 12 + (int64_t)slot_target.size() * (4 + 2) + (int64_t)cp_rank.size() * 2 +
               cp_parked * (8 + 8 + 4) + (n + 1) * 4;
    if (sym_slices) // positions; slot targets, segments, flags; contributions; parked sums and row lists
        return (int64_t)ss_src.size() * 12 + (int64_t)slot_target.size() * (4 + 2 + 1 + 8 + 8 + 4) +
               (int64_t)tl.size() * 2 + n * 5;
    return 0;
}

static bool decide_cached(const Plan &p)
{
    const int64_t mb = p.slice_stream_bytes();
    bool c = mb > 0 && mb + 40 * p.n <= kCacheResidentBytes;
    if (const char *e = std::getenv("CGMI_MATRIX_LOADS"))
        c = mb > 0 && (std::strcmp(e, "cached") == 0 ? true : std::strcmp(e, "stream") == 0 ? false : c);
    return c;
}

int lanes_for_mean_length(double mean_len)
{
    int w = 4;
    while (w < 64 && w < mean_len)
        w *= 2;
    return w;
}

int validate_and_normalise(int fmt, int64_t n, const int32_t *ptr, const int32_t *idx, const double *vals,
                           int base, uint32_t flags, std::vector<int32_t> &ptr0, std::vector<int32_t> &idx0,
                           std::string &err, std::vector<int32_t> *perm)
{
    if (perm)
        perm->clear();
    if (fmt < 0 || fmt > 2) {
        err = "unknown format";
        return CG_ERR_ARG;
    }
    if (n < 0 || n > INT32_MAX - 1) {
        err = "n out of range";
        return CG_ERR_ARG;
    }
    if (base != 0 && base != 1) {
        err = "index_base must be 0 or 1";
        return CG_ERR_ARG;
    }
    ptr0.assign((size_t)n + 1, 0);
    idx0.clear();
    if (n == 0)
        return CG_OK;
    if (!ptr) {
        err = "ptr is NULL";
        return CG_ERR_ARG;
    }
    if (ptr[0] != base) {
        err = "ptr[0] != index_base";
        return CG_ERR_STRUCTURE;
    }
    for (int64_t i = 0; i < n; ++i)
        if (ptr[i + 1] < ptr[i]) {
            err = "ptr decreases at line " + std::to_string(i);
            return CG_ERR_STRUCTURE;
        }
    const int64_t nnz = (int64_t)ptr[n] - base;
    if (nnz > 0 && !idx) {
        err = "idx is NULL";
        return CG_ERR_ARG;
    }
    for (int64_t i = 0; i <= n; ++i)
        ptr0[i] = ptr[i] - base;
    idx0.resize((size_t)nnz);
    for (int64_t l = 0; l < n; ++l) {
        const int64_t b = ptr0[l], e = ptr0[l + 1];
        for (int64_t k = b; k < e; ++k) {
            const int64_t j = (int64_t)idx[k] - base;
            if (j < 0 || j >= n) {
                err = "index out of range at entry " + std::to_string(k);
                return CG_ERR_STRUCTURE;
            }
            if (k > b && idx[k] <= idx[k - 1]) {
                err = "indices not strictly increasing in line " + std::to_string(l);
                return CG_ERR_STRUCTURE;
            }
            if (fmt == kSymCsr && !(flags & CG_LOWER) && k == b && j != l) {
                err = "symmetric CSR row " + std::to_string(l) + " does not start with its diagonal";
                return CG_ERR_STRUCTURE;
            }
            if (fmt == kSymCsr && (flags & CG_LOWER) && k == e - 1 && j != l) {
                err = "lower symmetric CSR row " + std::to_string(l) + " does not end with its diagonal";
                return CG_ERR_STRUCTURE;
            }
            idx0[k] = (int32_t)j;
        }
        if (fmt == kSymCsr && e == b) {
            err = "symmetric CSR row " + std::to_string(l) + " is empty";
            return CG_ERR_STRUCTURE;
        }
    }
    if (vals) {
        for (int64_t k = 0; k < nnz; ++k)
            if (!std::isfinite(vals[k])) {
                err = "non-finite value at entry " + std::to_string(k);
                return CG_ERR_NONFINITE;
            }
    }
    if (fmt == kSymCsr && (flags & CG_LOWER)) {
        // lower triangle by rows == upper triangle by columns: transpose the
        // structure (stable counting sort) into the upper-by-rows layout;
        // the caller's values are permuted the same way by the creator
        std::vector<int32_t> tp((size_t)n + 1, 0), ti((size_t)nnz), src((size_t)nnz);
        for (int64_t k = 0; k < nnz; ++k)
            tp[idx0[k] + 1]++;
        for (int64_t i = 0; i < n; ++i)
            tp[i + 1] += tp[i];
        std::vector<int32_t> next(tp.begin(), tp.end() - 1);
        for (int64_t l = 0; l < n; ++l)
            for (int64_t k = ptr0[l]; k < ptr0[l + 1]; ++k) {
                const int32_t d = next[idx0[k]]++;
                ti[d] = (int32_t)l;
                src[d] = (int32_t)k;
            }
        ptr0.swap(tp);
        idx0.swap(ti);
        if (perm)
            perm->swap(src);
    }
    if ((flags & CG_CHECK_SYMMETRY) && fmt != kSymCsr) {
        // transpose by counting sort and compare entry by entry
        std::vector<int32_t> tp((size_t)n + 1, 0), ti((size_t)nnz), src((size_t)nnz);
        for (int64_t k = 0; k < nnz; ++k)
            tp[idx0[k] + 1]++;
        for (int64_t i = 0; i < n; ++i)
            tp[i + 1] += tp[i];
        std::vector<int32_t> next(tp.begin(), tp.end() - 1);
        for (int64_t l = 0; l < n; ++l)
            for (int64_t k = ptr0[l]; k < ptr0[l + 1]; ++k) {
                const int32_t d = next[idx0[k]]++;
                ti[d] = (int32_t)l;
                src[d] = (int32_t)k;
            }
        for (int64_t i = 0; i <= n; ++i)
            if (tp[i] != ptr0[i]) {
                err = "matrix is not symmetric (pattern)";
                return CG_ERR_STRUCTURE;
            }
        for (int64_t k = 0; k < nnz; ++k) {
            if (ti[k] != idx0[k]) {
                err = "matrix is not symmetric (pattern)";
                return CG_ERR_STRUCTURE;
            }
            if (vals && std::memcmp(&vals[k], &vals[src[k]], sizeof(double)) != 0) {
                err = "matrix is not symmetric (values)";
                return CG_ERR_STRUCTURE;
            }
        }
    }
    return CG_OK;
}

// Entries per block for the row-block kernels: the full 2048 (8 per thread)
// once the matrix gives >= 1024 such blocks, smaller for small matrices so
// that the launch still spreads over every compute unit (they are bound by
// latency, not bytes), never below `floor`.
static int64_t block_entries(int64_t nnz, int64_t floor)
{
    return std::max<int64_t>(floor, std::min<int64_t>(kStreamEntries, (nnz + 1023) / 1024));
}

static void plan_vectors(Plan &p)
{
    // 1024 elements per workgroup on large vectors, in every format (at
    // 100^3, with the vector kernels' registers sized to the chunk, 512 per
    // workgroup measured 3-7 % slower per iteration in all three); small
    // vectors use down to 256 per workgroup so that more compute units take
    // part
    const int64_t n = p.n;
    const int64_t per = 1024;
    int64_t g = std::max<int64_t>((n + per - 1) / per, std::min<int64_t>((n + 255) / 256, 512));
    g = std::max<int64_t>(1, std::min<int64_t>(g, kMaxVecBlocks));
    p.vec_blocks = (int)g;
    p.vec_chunk = (int)((n + g - 1) / g);
}

// Slices (see plan.h) over `nl` lines whose entries are seg_ptr[l] ..
// seg_ptr[l + 1] - 1, with columns seg_col and caller entries seg_src (null:
// the position itself).  mode: 0 = when lines are short and the padding is
// small, 1 = whenever the padded size fits 32-bit positions.
static bool plan_slices(Plan &p, int64_t nl, const int32_t *seg_ptr, const int32_t *seg_col, const int32_t *seg_src,
                        int mode)
{
    const int64_t nnz = nl > 0 ? seg_ptr[nl] : 0;
    const int64_t ns = (nl + kSliceRows - 1) / kSliceRows;
    std::vector<int64_t> off((size_t)ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t w = 0;
        for (int64_t r = s * kSliceRows; r < std::min(nl, (s + 1) * kSliceRows); ++r)
            w = std::max<int64_t>(w, (int64_t)seg_ptr[r + 1] - seg_ptr[r]);
        off[s + 1] = off[s] + w * kSliceRows;
    }
    const int64_t padded = off[ns];
    if (padded > INT32_MAX || nl > INT32_MAX)
        return false;
    if (mode == 0 && (nl == 0 || (double)nnz / (double)nl > kStreamMaxMeanRow ||
                      (double)(padded - nnz) > kSliceMaxPadding * nnz))
        return false;
    p.slices = true;
    p.sl_lines = nl;
    p.sl_off.assign(off.begin(), off.end());
    p.sl_src.assign((size_t)padded, -1);
    p.sl_col.assign((size_t)padded, -1);
    for (int64_t r = 0; r < nl; ++r) {
        const int64_t sl = r / kSliceRows, lane = r % kSliceRows;
        const int64_t w = (off[sl + 1] - off[sl]) / kSliceRows;
        for (int64_t k = seg_ptr[r]; k < seg_ptr[r + 1]; ++k) {
            const int64_t q = off[sl] + slice_position(k - seg_ptr[r], lane, w);
            p.sl_src[q] = seg_src ? seg_src[k] : (int32_t)k;
            p.sl_col[q] = seg_col[k];
        }
    }
    // one slice per wavefront up to kMaxSliceWgs workgroups, then each wave
    // takes several (contiguous per workgroup)
    const int64_t g = (ns + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t cap = kMaxSliceWgs;
    if (const char *e = std::getenv("CGMI_SLICE_WGS")) // experiments: fewer workgroups (dot partials)
        cap = std::max<int64_t>(1, std::min<int64_t>(cap, std::atoll(e)));
    p.csr_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
    p.csr_rows_per_block = 0;
    return true;
}

// experiments: CGMI_ROW_LAYOUT = rows (CSR row blocks / lanes per row, CSC
// panel chunks) or slices (the sliced layout whatever its padding)
static int slice_mode()
{
    const char *e = std::getenv("CGMI_ROW_LAYOUT");
    if (!e)
        return 0;
    return std::strcmp(e, "slices") == 0 ? 1 : std::strcmp(e, "rows") == 0 ? -1 : 0;
}

// 16-bit column offsets of CSR slices or CSC panel-slot slices (plan.h) when
// every column is within 32767 of the row its line adds to (line_row: the
// row of each line; null: the line itself, CSR); experiments: CGMI_COL16=0
// keeps 32-bit columns.
static void plan_col16(Plan &p, const int32_t *line_row)
{
    if (const char *e = std::getenv("CGMI_COL16"))
        if (std::strcmp(e, "0") == 0)
            return;
    const int64_t ns = (int64_t)p.sl_off.size() - 1;
    std::vector<int16_t> d16(p.sl_col.size(), kPad16);
    for (int64_t sl = 0; sl < ns; ++sl) {
        const int64_t w = (p.sl_off[sl + 1] - p.sl_off[sl]) / kSliceRows;
        for (int64_t lane = 0; lane < kSliceRows; ++lane)
            for (int64_t k = 0; k < w; ++k) {
                const int64_t q = p.sl_off[sl] + slice_position(k, lane, w);
                if (p.sl_col[q] < 0)
                    continue;
                const int64_t l = sl * kSliceRows + lane;
                const int64_t d = (int64_t)p.sl_col[q] - (line_row ? line_row[l] : l);
                if (d < -32767 || d > 32767)
                    return;
                d16[q] = (int16_t)d;
            }
    }
    p.sl_d16.swap(d16);
}

static void plan_csr(Plan &p, const int32_t *ptr, const int32_t *idx)
{
    const int64_t n = p.n;
    const double mean = (double)p.nnz / (double)n;
    const int mode = slice_mode();
    if (mode >= 0 && plan_slices(p, n, ptr, idx, nullptr, mode)) {
        plan_col16(p, nullptr);
        return;
    }
    if (mean <= kStreamMaxMeanRow) {
        // row blocks: <= `be` entries (<= kStreamEntries) and <= kStreamRows
        // rows; a row longer than kStreamEntries is a block of its own
        const int64_t be = block_entries(p.nnz, kBlock);
        p.csr_stream = true;
        p.csr_rb.clear();
        p.csr_rb.push_back(0);
        int64_t r0 = 0;
        for (int64_t r = 0; r < n; ++r) {
            const int64_t len = (int64_t)ptr[r + 1] - ptr[r];
            if (r > r0 && ((int64_t)ptr[r + 1] - ptr[r0] > be || r - r0 >= kStreamRows || len > kStreamEntries)) {
                p.csr_rb.push_back((int32_t)r);
                r0 = r;
            }
            if (len > kStreamEntries) {
                p.csr_rb.push_back((int32_t)(r + 1));
                r0 = r + 1;
            }
        }
        if (p.csr_rb.back() != n)
            p.csr_rb.push_back((int32_t)n);
        const int64_t nrb = (int64_t)p.csr_rb.size() - 1;
        p.csr_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(nrb, kMaxSpmvBlocks));
        p.csr_rows_per_block = 0;
        return;
    }
    const int rows_per_pass = (kBlock / p.lanes) * 4; // 4 row tiles per lane group and pass
    int64_t g = (n + rows_per_pass - 1) / rows_per_pass;
    g = std::max<int64_t>(1, std::min<int64_t>(g, kMaxSpmvBlocks));
    p.csr_blocks = (int)g;
    p.csr_rows_per_block = (int)((n + g - 1) / g);
}

// CSC column panels (see plan.h).
static int plan_panels(Plan &p, const int32_t *ptr, const int32_t *idx, std::string &err)
{
    const int64_t n = p.n, nnz = p.nnz;
    int64_t bw = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = ptr[j]; k < ptr[j + 1]; ++k)
            bw = std::max<int64_t>(bw, std::llabs((int64_t)idx[k] - j));
    int64_t W = std::max<int64_t>(2 * bw + 1, kPanelMinWidth);
    // experiments: a wider panel (never narrower than 2 bw + 1, which the
    // two-colour guarantee needs); at n the product is one row-ordered panel
    if (const char *e = std::getenv("CGMI_PANEL_WIDTH"))
        W = std::max<int64_t>(W, std::atoll(e));
    W = std::min<int64_t>(n, W);
    const int64_t np = (n + W - 1) / W;
    p.panel = true;
    p.pn_width = W;
    p.pn_npanels = (int)np;
    p.pn_src.resize((size_t)nnz);
    p.pn_col.resize((size_t)nnz);
    p.pn_slot_target.clear();
    p.pn_slot_panel.clear();
    p.pn_slot_ptr.assign(1, 0);
    std::vector<int64_t> cnt;
    int64_t pos = 0;
    for (int parity = 0; parity < 2; ++parity) {
        if (parity == 1)
            p.pn_first_parked = (int32_t)p.pn_slot_target.size();
        for (int64_t k = parity; k < np; k += 2) {
            const int64_t c0 = k * W, c1 = std::min(n, c0 + W);
            const int64_t rlo = std::max<int64_t>(0, c0 - bw), rhi = std::min(n, c1 + bw);
            cnt.assign((size_t)(rhi - rlo + 1), 0);
            for (int64_t j = c0; j < c1; ++j)
                for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e)
                    cnt[idx[e] - rlo + 1]++;
            for (int64_t r = 0; r < rhi - rlo; ++r) {
                if (cnt[r + 1] > 0) {
                    p.pn_slot_target.push_back((int32_t)(rlo + r));
                    p.pn_slot_panel.push_back((int32_t)k);
                    p.pn_slot_ptr.push_back((int32_t)(pos + cnt[r] + cnt[r + 1]));
                }
                cnt[r + 1] += cnt[r];
            }
            // stable placement: columns ascending, so each row's segment is in column order
            for (int64_t j = c0; j < c1; ++j)
                for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
                    const int64_t q = pos + cnt[idx[e] - rlo]++;
                    p.pn_src[q] = (int32_t)e;
                    p.pn_col[q] = (int32_t)j;
                }
            pos += cnt[rhi - rlo];
        }
    }
    if (np < 2)
        p.pn_first_parked = (int32_t)p.pn_slot_target.size();
    if (pos != nnz) {
        err = "internal: panel placement lost entries";
        return CG_ERR_HIP;
    }
    // chunks: consecutive slots, <= ce entries (<= kPanelChunkEntries) and
    // <= kPanelChunkSlots slots; a slot longer than kPanelChunkEntries is a
    // chunk of its own
    const int64_t ns = (int64_t)p.pn_slot_target.size();
    const int64_t ce = block_entries(nnz, kBlock);
    p.pn_chunk_slot.assign(1, 0);
    int64_t s0 = 0;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t len = (int64_t)p.pn_slot_ptr[s + 1] - p.pn_slot_ptr[s];
        if (s > s0 && ((int64_t)p.pn_slot_ptr[s + 1] - p.pn_slot_ptr[s0] > ce || s - s0 >= kPanelChunkSlots ||
                       len > kPanelChunkEntries)) {
            p.pn_chunk_slot.push_back((int32_t)s);
            s0 = s;
        }
        if (len > kPanelChunkEntries) {
            p.pn_chunk_slot.push_back((int32_t)(s + 1));
            s0 = s + 1;
        }
    }
    if (p.pn_chunk_slot.back() != ns)
        p.pn_chunk_slot.push_back((int32_t)ns);
    const int64_t nch = (int64_t)p.pn_chunk_slot.size() - 1;
    p.nblocks = (int)nch;
    p.ncolors = np >= 2 && p.pn_first_parked < ns ? 2 : (ns > 0 ? 1 : 0);
    p.max_entries = 0;
    for (int64_t c = 0; c < nch; ++c)
        p.max_entries = std::max<int>(p.max_entries, p.pn_slot_ptr[p.pn_chunk_slot[c + 1]] -
                                                         p.pn_slot_ptr[p.pn_chunk_slot[c]]);
    p.max_slots = kPanelChunkSlots;
    p.max_lines = 0;
    const int mode = slice_mode();
    if (mode >= 0)
        if (plan_slices(p, ns, p.pn_slot_ptr.data(), p.pn_col.data(), p.pn_src.data(), mode))
            plan_col16(p, p.pn_slot_target.data());
    return CG_OK;
}

static int plan_scatter(Plan &p, const int32_t *ptr, const int32_t *idx, int target_entries, std::string &err)
{
    const int64_t n = p.n;
    const bool sym = p.format == kSymCsr;
    const int E = target_entries;

    // 1. blocks: contiguous lines, <= E entries and <= kMaxBlockLines lines;
    //    a line longer than E gets blocks of its own, E entries each
    std::vector<ScatterBlock> &B = p.blocks;
    B.clear();
    auto push = [&](int64_t l0, int64_t l1, int64_t k0, int64_t k1) {
        ScatterBlock b{};
        b.line0 = (int32_t)l0;
        b.line1 = (int32_t)l1;
        b.k0 = (int32_t)k0;
        b.k1 = (int32_t)k1;
        b.id = (int32_t)B.size();
        B.push_back(b);
    };
    {
        int64_t l0 = 0;
        for (int64_t l = 0; l < n; ++l) {
            const int64_t len = (int64_t)ptr[l + 1] - ptr[l];
            if (len > E) {
                if (l > l0)
                    push(l0, l, ptr[l0], ptr[l]);
                for (int64_t k = ptr[l]; k < ptr[l + 1]; k += E)
                    push(l, l + 1, k, std::min<int64_t>(k + E, ptr[l + 1]));
                l0 = l + 1;
                continue;
            }
            if (l > l0 && ((int64_t)ptr[l + 1] - ptr[l0] > E || l - l0 >= kMaxBlockLines)) {
                push(l0, l, ptr[l0], ptr[l]);
                l0 = l;
            }
        }
        if (n > l0)
            push(l0, n, ptr[l0], ptr[n]);
    }
    const int nb = (int)B.size();
    p.nblocks = nb;

    // 2. slots and contributions of every block; rows nobody writes are
    //    attached to the block covering the same line index (they receive 0)
    std::vector<int32_t> slot_of((size_t)n, -1);
    std::vector<uint8_t> touched((size_t)n, 0);
    std::vector<std::vector<int32_t>> targets(nb);
    for (int b = 0; b < nb; ++b) {
        const ScatterBlock &bk = B[b];
        std::vector<int32_t> &t = targets[b];
        if (sym) {
            for (int32_t l = bk.line0; l < bk.line1; ++l)
                t.push_back(l);
            std::vector<int32_t> remote;
            for (int64_t l = bk.line0; l < bk.line1; ++l) {
                const int64_t s = std::max<int64_t>(ptr[l], bk.k0), e = std::min<int64_t>(ptr[l + 1], bk.k1);
                for (int64_t k = s; k < e; ++k)
                    if (idx[k] >= bk.line1)
                        remote.push_back(idx[k]);
            }
            std::sort(remote.begin(), remote.end());
            remote.erase(std::unique(remote.begin(), remote.end()), remote.end());
            t.insert(t.end(), remote.begin(), remote.end());
        } else {
            for (int64_t k = bk.k0; k < bk.k1; ++k)
                t.push_back(idx[k]);
            std::sort(t.begin(), t.end());
            t.erase(std::unique(t.begin(), t.end()), t.end());
        }
        for (int32_t r : t)
            touched[r] = 1;
    }
    if (!sym) {
        // a row with no entry at all (empty row of A) still needs y_i = 0
        int b = 0;
        for (int64_t r = 0; r < n; ++r) {
            if (touched[r])
                continue;
            while (b + 1 < nb && B[b].line1 <= r)
                ++b;
            targets[b].push_back((int32_t)r);
            touched[r] = 1;
        }
    }

    // 3. greedy colouring in block order on the write-set conflict graph
    std::vector<uint64_t> used((size_t)n, 0);
    p.block_color.assign(nb, 0);
    int ncol = 0;
    for (int b = 0; b < nb; ++b) {
        uint64_t forbid = 0;
        for (int32_t r : targets[b])
            forbid |= used[r];
        if (forbid == ~0ull) {
            err = "scatter plan needs more than 64 colours (a row shared by too many blocks); use CSR";
            return CG_ERR_UNSUPPORTED;
        }
        int c = 0;
        while (forbid & (1ull << c))
            ++c;
        p.block_color[b] = c;
        ncol = std::max(ncol, c + 1);
        for (int32_t r : targets[b])
            used[r] |= 1ull << c;
    }
    p.ncolors = ncol;

    // 4. slot arrays, FIRST / LAST flags, contributions (counting sort per block)
    std::vector<int8_t> minc((size_t)n, 127), maxc((size_t)n, -1);
    for (int b = 0; b < nb; ++b)
        for (int32_t r : targets[b]) {
            minc[r] = (int8_t)std::min<int>(minc[r], p.block_color[b]);
            maxc[r] = (int8_t)std::max<int>(maxc[r], p.block_color[b]);
        }
    int64_t total_slots = 0, total_tl = 0;
    for (int b = 0; b < nb; ++b) {
        total_slots += (int64_t)targets[b].size();
        total_tl += B[b].k1 - B[b].k0;
    }
    if (total_slots + nb + 1 >= INT32_MAX || total_tl >= INT32_MAX) {
        err = "scatter plan too large for 32-bit offsets";
        return CG_ERR_UNSUPPORTED;
    }
    p.slot_target.clear();
    p.slot_flag.clear();
    p.slot_count.clear();
    p.seg.clear();
    p.tl.clear();
    p.slot_target.reserve(total_slots);
    p.slot_flag.reserve(total_slots);
    p.slot_count.reserve(total_slots);
    p.seg.reserve(total_slots + nb);
    p.tl.reserve(total_tl);
    p.max_entries = 0;
    p.max_lines = 0;
    p.max_slots = 0;
    std::vector<int32_t> cnt;
    for (int b = 0; b < nb; ++b) {
        ScatterBlock &bk = B[b];
        const std::vector<int32_t> &t = targets[b];
        bk.slot0 = (int32_t)p.slot_target.size();
        bk.nslots = (int32_t)t.size();
        bk.tl0 = (int32_t)p.tl.size();
        const int c = p.block_color[b];
        for (size_t s = 0; s < t.size(); ++s) {
            slot_of[t[s]] = (int32_t)s;
            p.slot_target.push_back(t[s]);
            uint8_t f = 0;
            if (minc[t[s]] == c)
                f |= kSlotFirst;
            if (maxc[t[s]] == c)
                f |= kSlotLast;
            p.slot_flag.push_back(f);
        }
        // contributions: (slot, local entry) in ascending entry order
        cnt.assign(t.size() + 1, 0);
        auto for_each_contrib = [&](auto &&fn) {
            for (int64_t l = bk.line0; l < bk.line1; ++l) {
                const int64_t s = std::max<int64_t>(ptr[l], bk.k0), e = std::min<int64_t>(ptr[l + 1], bk.k1);
                for (int64_t k = s; k < e; ++k) {
                    if (sym && idx[k] == l)
                        continue; // the diagonal has no mirror
                    fn(slot_of[idx[k]], (int32_t)(k - bk.k0));
                }
            }
        };
        for_each_contrib([&](int32_t s, int32_t) { cnt[s + 1]++; });
        for (size_t s = 0; s < t.size(); ++s)
            cnt[s + 1] += cnt[s];
        const size_t base = p.tl.size();
        p.tl.resize(base + cnt[t.size()]);
        for (size_t s = 0; s <= t.size(); ++s)
            p.seg.push_back((uint16_t)cnt[s]);
        for (size_t s = 0; s < t.size(); ++s)
            p.slot_count.push_back(cnt[s + 1] - cnt[s]);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for_each_contrib([&](int32_t s, int32_t k) { p.tl[base + fill[s]++] = (uint16_t)k; });
        for (int32_t r : t)
            slot_of[r] = -1;
        bk.ntl = cnt[t.size()];
        p.max_entries = std::max(p.max_entries, bk.k1 - bk.k0);
        p.max_lines = std::max(p.max_lines, bk.line1 - bk.line0);
        p.max_slots = std::max(p.max_slots, bk.nslots);
    }

    // 5. phase order: block ids sorted by colour, block order within a colour
    p.color_off.assign(ncol + 1, 0);
    for (int b = 0; b < nb; ++b)
        p.color_off[p.block_color[b] + 1]++;
    for (int c = 0; c < ncol; ++c)
        p.color_off[c + 1] += p.color_off[c];
    p.phase_blocks.assign(nb, 0);
    std::vector<int32_t> pos(p.color_off.begin(), p.color_off.end() - 1);
    for (int b = 0; b < nb; ++b)
        p.phase_blocks[pos[p.block_color[b]]++] = b;
    return CG_OK;
}

// Symmetric CSR, sliced blocks (plan.h): every block keeps its lines and
// slots; only the order of its entries changes (k-th entries of its lines
// contiguous), so that thread l holds line l's entries in registers.  Taken
// when no line of any block has more than kStreamPerThread entries (and, by
// default, the padding stays small).
static void plan_sym_slices(Plan &p, const int32_t *ptr, const int32_t *idx, int mode)
{
    if (p.format != kSymCsr || mode < 0 || p.nblocks == 0)
        return;
    const int nb = p.nblocks;
    std::vector<int32_t> pos((size_t)nb + 1, 0);
    int64_t total = 0;
    for (int b = 0; b < nb; ++b) {
        const ScatterBlock &bk = p.blocks[b];
        const int64_t nl = bk.line1 - bk.line0;
        int64_t L = 0;
        for (int64_t l = bk.line0; l < bk.line1; ++l)
            L = std::max<int64_t>(L, std::min<int64_t>(ptr[l + 1], bk.k1) - std::max<int64_t>(ptr[l], bk.k0));
        if (L > kStreamPerThread || nl > kBlock)
            return;
        total += nl * L;
        if (total > INT32_MAX)
            return;
        pos[b + 1] = (int32_t)total;
    }
    if (mode == 0 && (double)(total - p.nnz) > kSliceMaxPadding * (double)p.nnz)
        return;
    p.ss_pos = pos;
    p.ss_src.assign((size_t)total, -1);
    p.ss_idx.assign((size_t)total, -1);
    p.ss_tl = p.tl;
    std::vector<uint16_t> local;
    for (int b = 0; b < nb; ++b) {
        const ScatterBlock &bk = p.blocks[b];
        const int64_t nl = bk.line1 - bk.line0;
        local.assign((size_t)(bk.k1 - bk.k0), 0);
        for (int64_t l = bk.line0; l < bk.line1; ++l) {
            const int64_t e0 = std::max<int64_t>(ptr[l], bk.k0), e1 = std::min<int64_t>(ptr[l + 1], bk.k1);
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t lp = (e - e0) * nl + (l - bk.line0);
                p.ss_src[pos[b] + lp] = (int32_t)e;
                p.ss_idx[pos[b] + lp] = idx[e];
                local[e - bk.k0] = (uint16_t)lp;
            }
        }
        for (int32_t i = bk.tl0; i < bk.tl0 + bk.ntl; ++i)
            p.ss_tl[i] = local[p.tl[i]];
    }
    p.sym_slices = true;
}

// experiments: CGMI_SYM_PLAN = colour selects the contiguous, coloured plan
// for symmetric CSR even where compact blocks apply
static bool compact_allowed()
{
    const char *e = std::getenv("CGMI_SYM_PLAN");
    return !(e && std::strcmp(e, "colour") == 0);
}

// Lines per compact block: kCompactLines on large matrices; on small ones
// fewer, so that there are about 512 blocks to spread over the 256 compute
// units (a small system's iteration is bound by latency, not bytes).
// Experiments: CGMI_COMPACT_LINES overrides (16 .. kCompactLines).
static int compact_block_lines(int64_t n)
{
    int lines = kCompactLines;
    while (lines > 64 && n / lines < 512)
        lines /= 2;
    if (const char *e = std::getenv("CGMI_COMPACT_LINES"))
        lines = std::max(16, std::min(kCompactLines, std::atoi(e)));
    return lines;
}

// Symmetric CSR, compact blocks (plan.h).  Returns false (plan untouched)
// when some line has more than kStreamPerThread entries.
static bool plan_sym_compact(Plan &p, const int32_t *ptr, const int32_t *idx)
{
    const int64_t n = p.n;
    const int cap = compact_block_lines(n);
    for (int64_t l = 0; l < n; ++l)
        if ((int64_t)ptr[l + 1] - ptr[l] > kStreamPerThread)
            return false;
    // graph of A without the diagonal: the stored triangle and its mirror
    std::vector<int32_t> ap((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (idx[k] != i) {
                ap[i + 1]++;
                ap[idx[k] + 1]++;
            }
    for (int64_t i = 0; i < n; ++i)
        ap[i + 1] += ap[i];
    std::vector<int32_t> ai((size_t)ap[n]);
    {
        std::vector<int32_t> fill(ap.begin(), ap.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
                if (idx[k] != i) {
                    ai[fill[i]++] = idx[k];
                    ai[fill[idx[k]]++] = (int32_t)i;
                }
    }
    // 1. growth: from the lowest free line; nearest to the seed first, then
    //    most couplings into the block, then the lowest line number
    std::vector<int32_t> blk((size_t)n, -1), gain((size_t)n, 0), dist((size_t)n, 0), stamp((size_t)n, -1);
    struct Cand {
        int64_t key;
        int32_t line;
        bool operator<(const Cand &o) const { return key < o.key || (key == o.key && line > o.line); }
    };
    auto key = [&](int32_t j) { return -(int64_t)dist[j] * 4096 + gain[j]; };
    std::vector<Cand> heap;
    int32_t nb = 0;
    int64_t seed = 0;
    while (true) {
        while (seed < n && blk[seed] >= 0)
            ++seed;
        if (seed >= n)
            break;
        heap.clear();
        dist[seed] = 0;
        gain[seed] = 0;
        stamp[seed] = nb;
        heap.push_back({key((int32_t)seed), (int32_t)seed});
        int lines = 0;
        while (!heap.empty() && lines < cap) {
            std::pop_heap(heap.begin(), heap.end());
            const Cand c = heap.back();
            heap.pop_back();
            const int32_t i = c.line;
            if (blk[i] >= 0 || stamp[i] != nb || c.key != key(i))
                continue; // taken, or a stale entry
            blk[i] = nb;
            ++lines;
            for (int32_t q = ap[i]; q < ap[i + 1]; ++q) {
                const int32_t j = ai[q];
                if (blk[j] >= 0)
                    continue;
                if (stamp[j] != nb) {
                    stamp[j] = nb;
                    gain[j] = 0;
                    dist[j] = dist[i] + 1;
                }
                gain[j]++;
                heap.push_back({key(j), j});
                std::push_heap(heap.begin(), heap.end());
            }
        }
        ++nb;
    }
    // 2. merge small pockets into the neighbour they couple to most (with room)
    std::vector<int32_t> bl((size_t)nb, 0);
    for (int64_t i = 0; i < n; ++i)
        bl[blk[i]]++;
    {
        std::vector<std::vector<int32_t>> mem((size_t)nb);
        for (int64_t i = 0; i < n; ++i)
            mem[blk[i]].push_back((int32_t)i);
        std::vector<int32_t> order((size_t)nb);
        for (int32_t b = 0; b < nb; ++b)
            order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return bl[a] < bl[b]; });
        std::vector<int32_t> cnt((size_t)nb, 0), touched;
        for (int32_t b : order) {
            if (bl[b] == 0 || bl[b] >= cap / 2)
                continue;
            touched.clear();
            for (int32_t i : mem[b])
                for (int32_t q = ap[i]; q < ap[i + 1]; ++q) {
                    const int32_t c = blk[ai[q]];
                    if (c == b)
                        continue;
                    if (cnt[c]++ == 0)
                        touched.push_back(c);
                }
            int32_t best = -1;
            for (int32_t c : touched)
                if (bl[c] + bl[b] <= cap &&
                    (best < 0 || cnt[c] > cnt[best] || (cnt[c] == cnt[best] && c < best)))
                    best = c;
            for (int32_t c : touched)
                cnt[c] = 0;
            if (best < 0)
                continue;
            for (int32_t i : mem[b]) {
                blk[i] = best;
                mem[best].push_back(i);
            }
            mem[b].clear();
            bl[best] += bl[b];
            bl[b] = 0;
        }
    }
    // 3. block order: by lowest line; lines ascending inside a block
    std::vector<int32_t> first((size_t)nb, INT32_MAX), rank((size_t)nb, -1), ids;
    for (int64_t i = n - 1; i >= 0; --i)
        first[blk[i]] = (int32_t)i;
    for (int32_t b = 0; b < nb; ++b)
        if (bl[b] > 0)
            ids.push_back(b);
    std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) { return first[a] < first[b]; });
    for (size_t k = 0; k < ids.size(); ++k)
        rank[ids[k]] = (int32_t)k;
    const int32_t nbk = (int32_t)ids.size();
    p.cp_block_of.resize((size_t)n);
    std::vector<int32_t> lp((size_t)nbk + 1, 0), lines((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        p.cp_block_of[i] = rank[blk[i]];
        lp[rank[blk[i]] + 1]++;
    }
    for (int32_t b = 0; b < nbk; ++b)
        lp[b + 1] += lp[b];
    {
        std::vector<int32_t> fill(lp.begin(), lp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            lines[fill[p.cp_block_of[i]]++] = (int32_t)i; // ascending inside each block
    }
    // 4. per block: positions, slots (own lines, then the rows reached
    //    outside), contributions grouped by slot (line order within a slot)
    p.cp_blocks.assign((size_t)nbk, CompactBlock{});
    p.cp_rank.assign((size_t)n * kStreamPerThread, 0xffff);
    p.slot_target.clear();
    p.slot_count.clear();
    p.seg.clear();
    p.ss_tl.clear();
    p.ss_src.clear();
    p.ss_idx.clear();
    p.ss_pos.assign((size_t)nbk + 1, 0);
    std::vector<int32_t> local((size_t)n, -1); // row -> local slot while its block is built
    std::vector<int32_t> remote, cs;
    std::vector<std::pair<int32_t, int32_t>> contrib; // (slot, position)
    int64_t pos = 0, parked = 0;
    p.max_slots = 0;
    p.max_entries = 0;
    p.max_lines = 0;
    p.cp_perm = lines; // blocks' lines in block order: the device numbering
    for (int32_t b = 0; b < nbk; ++b) {
        const int32_t l0 = lp[b], nl = lp[b + 1] - lp[b];
        int32_t len = 0;
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t i = lines[l0 + t];
            len = std::max<int32_t>(len, ptr[i + 1] - ptr[i]);
            local[i] = t;
        }
        remote.clear();
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t i = lines[l0 + t];
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
                if (idx[k] != i && local[idx[k]] < 0)
                    remote.push_back(idx[k]);
        }
        std::sort(remote.begin(), remote.end());
        remote.erase(std::unique(remote.begin(), remote.end()), remote.end());
        for (size_t r = 0; r < remote.size(); ++r)
            local[remote[r]] = nl + (int32_t)r;
        const int32_t ns = nl + (int32_t)remote.size();
        contrib.clear();
        if (pos + (int64_t)nl * len > INT32_MAX)
            return false;
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t i = lines[l0 + t];
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
                const int32_t q = (int32_t)((k - ptr[i]) * nl + t); // LDS slot of its mirror product
                if (idx[k] != i)
                    contrib.push_back({local[idx[k]], q});
            }
        }
        std::stable_sort(contrib.begin(), contrib.end(),
                         [](const std::pair<int32_t, int32_t> &a, const std::pair<int32_t, int32_t> &c) {
                             return a.first < c.first;
                         });
        CompactBlock &cb = p.cp_blocks[b];
        cb.pos0 = (int32_t)pos;
        cb.len = len;
        cb.nl = nl;
        cb.slot0 = (int32_t)p.slot_target.size();
        cb.nslots = ns;
        cb.seg0 = (int32_t)p.seg.size();
        cb.line0 = l0;
        cb.park0 = (int32_t)parked;
        for (int32_t t = 0; t < nl; ++t)
            p.slot_target.push_back(lines[l0 + t]);
        for (int32_t r : remote)
            p.slot_target.push_back(r);
        cs.assign((size_t)ns + 1, 0);
        for (const auto &c : contrib)
            cs[c.first + 1]++;
        for (int32_t s = 0; s < ns; ++s)
            cs[s + 1] += cs[s];
        for (int32_t s = 0; s <= ns; ++s)
            p.seg.push_back((uint16_t)cs[s]);
        while (p.seg.size() % 8 != 0) // the next block's starts begin 16-byte aligned
            p.seg.push_back(0);
        for (int32_t s = 0; s < ns; ++s)
            p.slot_count.push_back(cs[s + 1] - cs[s]);
        for (size_t r = 0; r < contrib.size(); ++r) { // LDS place = rank in the slot-grouped order
            const int32_t q = contrib[r].second, t = q % nl, k = q / nl;
            p.cp_rank[(size_t)(l0 + t) * kStreamPerThread + k] = (uint16_t)r;
        }
        // positions: entries k and k + 1 of line t side by side (pairs, as in
        // the slices with nl lines), padding -1; every block starts at an
        // even position, so a pair is one aligned 8- / 16-byte load
        const int64_t npos = ((int64_t)nl * len + 1) & ~int64_t(1);
        p.ss_src.resize((size_t)(pos + npos), -1);
        p.ss_idx.resize((size_t)(pos + npos), -1);
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t i = lines[l0 + t];
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
                const int64_t kk = k - ptr[i];
                const int64_t q = pos + (kk < (len & ~1) ? (kk >> 1) * 2 * nl + 2 * t + (kk & 1) : kk * nl + t);
                p.ss_src[q] = (int32_t)k;
                p.ss_idx[q] = idx[k];
            }
        }
        pos += npos;
        p.ss_pos[b + 1] = (int32_t)pos;
        parked += (int64_t)remote.size();
        for (int32_t t = 0; t < nl; ++t)
            local[lines[l0 + t]] = -1;
        for (int32_t r : remote)
            local[r] = -1;
        p.max_slots = std::max(p.max_slots, ns);
        p.max_entries = std::max(p.max_entries, nl * len);
        p.max_lines = std::max(p.max_lines, nl);
    }
    if ((int64_t)p.slot_target.size() + nbk + 1 >= INT32_MAX || parked >= INT32_MAX)
        return false;
    p.nblocks = nbk;
    p.ncolors = 1;
    p.cp_parked = parked;
    p.blocks.clear();
    p.block_color.assign((size_t)nbk, 0);
    p.color_off = {0, nbk};
    p.phase_blocks.clear();
    p.sym_compact = true;
    return true;
}

// Symmetric CSR on a small system (vector kernels of at most 256
// workgroups, n <= 65 536): there the product is bound by its launch and
// its chain of dependent steps, not by the bytes the triangle saves, and the
// scatter's mirror products through LDS and parked sums lengthen that chain.
// The triangle is expanded into full rows -- an off-diagonal entry stored at
// (i, j) and (j, i), both positions naming the caller's one entry -- and
// sliced like CSR; row i's entries come in ascending column order (mirrored
// ones first).  Experiments: CGMI_SYM_EXPAND=0 keeps the scatter plans.
static bool plan_sym_expanded(Plan &p, const int32_t *ptr, const int32_t *idx)
{
    if (p.vec_blocks > kBlock)
        return false;
    if (const char *e = std::getenv("CGMI_SYM_EXPAND"))
        if (std::strcmp(e, "0") == 0)
            return false;
    const int64_t n = p.n;
    std::vector<int32_t> fptr((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            fptr[i + 1]++;
            if (idx[k] != i)
                fptr[idx[k] + 1]++;
        }
    for (int64_t i = 0; i < n; ++i)
        fptr[i + 1] += fptr[i];
    if (fptr[n] > INT32_MAX / 2)
        return false;
    std::vector<int32_t> fcol((size_t)fptr[n]), fsrc((size_t)fptr[n]), next(fptr.begin(), fptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = idx[k];
            fcol[next[i]] = j;
            fsrc[next[i]++] = (int32_t)k;
            if (j != i) {
                fcol[next[j]] = (int32_t)i;
                fsrc[next[j]++] = (int32_t)k;
            }
        }
    if (!plan_slices(p, n, fptr.data(), fcol.data(), fsrc.data(), slice_mode()))
        return false;
    plan_col16(p, nullptr);
    p.sym_expanded = true;
    return true;
}

int build_plan(int fmt, int64_t n, const int32_t *ptr0, const int32_t *idx0, int target_entries, Plan &p,
               std::string &err)
{
    p = Plan{};
    p.format = fmt;
    p.n = n;
    p.nnz = n > 0 ? ptr0[n] : 0;
    if (n == 0)
        return CG_OK;
    const double mean = (double)p.nnz / (double)n;
    p.lanes = lanes_for_mean_length(mean);
    plan_vectors(p);
    if (fmt == kCsr) {
        plan_csr(p, ptr0, idx0);
        p.cached = decide_cached(p);
        return CG_OK;
    }
    if (fmt == kCsc) {
        const int st = plan_panels(p, ptr0, idx0, err);
        p.cached = st == CG_OK && decide_cached(p);
        return st;
    }
    if (target_entries <= 0 && compact_allowed() && slice_mode() >= 0 && plan_sym_expanded(p, ptr0, idx0)) {
        p.cached = decide_cached(p);
        return CG_OK;
    }
    if (target_entries <= 0 && compact_allowed() && slice_mode() >= 0 && plan_sym_compact(p, ptr0, idx0)) {
        p.cached = decide_cached(p);
        return CG_OK;
    }
    if (target_entries <= 0)
        target_entries = (int)block_entries(p.nnz, 512);
    target_entries = std::min(target_entries, kMaxScatterEntries);
    const int st = plan_scatter(p, ptr0, idx0, target_entries, err);
    if (st == CG_OK) {
        plan_sym_slices(p, ptr0, idx0, slice_mode());
        p.cached = decide_cached(p);
    }
    return st;
}

} // namespace cgmi

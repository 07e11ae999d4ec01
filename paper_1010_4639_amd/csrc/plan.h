// Host-side planning of the sparse product: structure validation, index-base
// conversion, and the atomic-free scatter plan for the formats whose product
// writes rows other than the one being read (symmetric CSR, CSC).
//
// Scatter plan.  The lines (rows of the stored triangle, or columns) are cut
// into contiguous blocks of at most `target_entries` entries.  A block's write
// set is the list of y rows it produces ("slots", sorted ascending); each slot
// gets the list of the block's products that land on it ("contributions",
// ascending entry order), so one workgroup can sum them in local memory with
// no atomics and in a fixed order.  Blocks whose write sets intersect are
// given different colours by a greedy pass in block order; the blocks of one
// colour run as one kernel, colours one after another.  Every slot carries
// two flags: FIRST (no earlier colour writes that row, so the block stores
// instead of read-modify-write) and LAST (no later colour writes it, so the
// block holds the final y_i and adds p_i y_i to the fused dot product).
//
// CSC plan ("column panels").  The columns are cut into panels of W >= 2 bw + 1
// consecutive columns (bw = the largest |i - j| of a stored entry), so panel
// k only writes rows within bw of its columns and panels k and k + 2 never
// share a row: even panels form colour 0, odd panels colour 1.  Inside a
// panel the entries are ordered by row, then column, so every (panel, row)
// pair -- a write slot -- is one contiguous segment summed in ascending column
// order, and consecutive slots are grouped into chunks (<= 2048 entries,
// <= 256 slots) for the workgroups.  Slots of colour 0 come first and write
// y; colour-1 slots are parked and added row by row afterwards.  This is the
// two-dimensional blocking of compressed-sparse-blocks storage applied to
// the transpose product: column blocks for the scatter, row order inside.
//
// Compact blocks (symmetric CSR whose lines have at most kStreamPerThread
// entries; the default there).  Contiguous line ranges are a poor unit for
// the mirrored product: in a mesh numbered plane by plane, almost every
// mirror product of a range lands outside it.  Instead blocks are grown on
// the graph of A: from the lowest-numbered free line, breadth first (lines
// nearer the seed first, then those with more couplings into the block,
// then the lowest number), up to kCompactLines (512) lines -- fewer on small
// matrices, so that there are about 512 blocks; leftover pockets of fewer
// than half that many lines are merged into the neighbouring block
// they couple to most when it has room.  Each line belongs to exactly one
// block, and that block OWNS the line's row of y: its first slots are its
// own lines (ascending), whose sums -- the stored row itself plus the mirror
// products landing on it from the block's other lines -- it stores in y.
// Its remaining slots are the rows outside the block that its mirror
// products reach; their sums are parked and added to y row by row
// afterwards, in ascending block order.  No two blocks write one location,
// so no colouring is needed.  On the device the rows are renumbered block
// by block (the lines of block b become the consecutive numbers
// line0 .. line0 + nl - 1, in their original order), so a block's own rows
// of x and y are contiguous: its y stores and own x loads are whole cache
// lines, and its gathers stay near them.  The plan itself (and its export)
// keeps the caller's numbering; cg_solve / cg_spmv move the caller's
// vectors in and out of the block order.  The entries of a block are stored like a
// slice of nl lines (entries 2j, 2j + 1 of line t side by side at
// pos0 + 2 nl j + 2 t, the last entries of an odd width at
// pos0 + nl (len - 1) + t).
//
// Slices.  Rows (CSR) or write slots (CSC panels: one (panel, row) segment
// each) are grouped in slices of 64 consecutive lines, one per wavefront
// lane; lines shorter than the slice's longest (w entries) are padded with
// source -1.  Inside a slice the entries are stored in pairs: entries 2j and
// 2j + 1 of the line of lane l sit side by side at off + 128 j + 2 l (+ 1),
// and when w is odd the last entries of all lines follow at
// off + 64 (w - 1) + l.  One 8- or 16-byte load per lane thus brings two
// entries, and a wave's load is 512 or 1024 contiguous bytes.  This is the
// sliced ELLPACK layout (SELL-C-sigma, Kreutzer et al. 2014) with C = 64, no
// sorting and two-entry packing: for a stencil-like matrix the lanes of one
// load read neighbouring x entries, so the gather of x becomes a
// near-contiguous load.  Chosen when the padding stays small; each line is
// still summed left to right by one lane.  When every column lies within
// 32767 of the row its line adds to (the CSR row, or the CSC slot's target
// row; any banded numbering, e.g. a 3D grid numbered lexicographically up to
// 181 x 181 nodes a plane) each column is stored as its 16-bit offset from
// that row (-32768 = padding) instead of the 32-bit index: 10 instead of 12
// bytes per FP64 entry, 6 instead of 8 per FP32 one.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace cgmi {

constexpr int kBlock = 256;             // threads per workgroup in every kernel
constexpr int16_t kPad16 = -32768;      // padding in 16-bit column offsets
constexpr int kDefaultScatterEntries = 2048;
constexpr int kMaxScatterEntries = 2048;   // 8 entries per thread held in registers
constexpr int kMaxBlockLines = 256;
constexpr int kMaxColors = 64;
constexpr int kMaxSpmvBlocks = 2048;    // CSR product workgroups (= dot partials)
constexpr int kMaxVecBlocks = 2048;
constexpr int kStreamPerThread = 8;                    // CSR row-block kernel: entries per thread
constexpr int kStreamEntries = kBlock * kStreamPerThread; // entries per CSR row block
constexpr int kStreamRows = kBlock;                    // rows per CSR row block (one thread each)
constexpr double kStreamMaxMeanRow = 32.0;             // longer mean rows use lanes-per-row
constexpr int kSliceRows = 64;          // slices: lines per slice (one wavefront, a line per lane)
constexpr int kWavesPerBlock = kBlock / kSliceRows;
constexpr int kMaxSliceWgs = 4 * kMaxSpmvBlocks; // slice kernel workgroups (= dot partials)
constexpr double kSliceMaxPadding = 0.125; // slices only while padding <= this fraction of nnz
// Sliced products read the matrix with ordinary (cache-allocating) loads
// while the bytes of one iteration (matrix side + 40 B per row of vectors)
// stay below this, so the matrix stays resident in the 256 MB Infinity Cache
// from one CG iteration to the next; non-temporal loads above.  Measured on
// FEM systems: at 110^3 (~325 MB) ordinary loads are 6-12 % faster per
// iteration, at 120^3 (~378 MB) 4-14 % slower.
constexpr int64_t kCacheResidentBytes = 336ll << 20;
constexpr int kPanelMinWidth = 4096;    // CSC panels span at least this many columns
constexpr int kPanelChunkEntries = kStreamEntries; // entries per CSC panel chunk
constexpr int kPanelChunkSlots = kBlock;           // slots per CSC panel chunk (one thread each)
constexpr int kCompactThreads = 512;     // compact blocks: workgroup size (one line per thread)
constexpr int kCompactLines = kCompactThreads;             // lines per compact block at most
constexpr int kCompactEntries = kCompactLines * kStreamPerThread; // entries per compact block at most
constexpr uint8_t kSlotFirst = 1;
constexpr uint8_t kSlotLast = 2;

enum Format { kCsr = 0, kSymCsr = 1, kCsc = 2 };

// Offset inside a slice of width w (entries per line) of the k-th entry of
// the line of lane `lane` (the pair packing above).
inline int64_t slice_position(int64_t k, int64_t lane, int64_t w)
{
    return k < (w & ~int64_t(1)) ? (k >> 1) * (2 * kSliceRows) + 2 * lane + (k & 1) : k * kSliceRows + lane;
}

struct ScatterBlock {
    int32_t line0, line1;  // lines [line0, line1)
    int32_t k0, k1;        // entries [k0, k1) (a line longer than the block limit is split)
    int32_t slot0, nslots; // slots [slot0, slot0 + nslots); seg of this block starts at slot0 + id
    int32_t tl0, id;       // contributions start; block id (index of its dot partial)
    int32_t ntl;           // number of contributions
    int32_t pad;           // device copy: colour of the block
};

// A compact block of the symmetric format (device layout).  Its mirror
// products are placed in LDS grouped by the slot they add to: slot s sums
// the products at [seg[seg0 + s], seg[seg0 + s + 1]); the place of the
// product of line t's k-th entry is cp_rank[8 (line0 + t) + k].
struct CompactBlock {
    int32_t pos0;   // first position of its entries (even)
    int32_t len;    // entries per line (its longest line; shorter lines padded)
    int32_t nl;     // own lines = its first nl slots
    int32_t slot0;  // slots [slot0, slot0 + nslots) of slot_target
    int32_t nslots;
    int32_t seg0;   // nslots + 1 slot starts seg[seg0 ..] (seg0 a multiple of 8)
    int32_t line0;  // its lines' ranks at cp_rank[8 line0 ..]
    int32_t park0;  // parked-sum index of its slot nl (its first non-own slot)
};

struct Plan {
    int format = 0;
    int64_t n = 0, nnz = 0;
    int lanes = 16;                       // lanes sharing one line
    // CSR: either row blocks (short rows: entries staged in LDS, one thread
    // sums each row) or `lanes` lanes per row over contiguous row ranges
    int csr_blocks = 0, csr_rows_per_block = 0;
    bool csr_stream = false;
    std::vector<int32_t> csr_rb;          // row-block starts (nrb + 1), stream mode
    // sliced layout of the CSR rows or of the CSC panel slots (replaces row
    // blocks / lanes per row / panel chunks); workgroups in csr_blocks
    bool slices = false;
    int64_t sl_lines = 0;                 // rows (CSR) or slots (CSC)
    std::vector<int32_t> sl_off;          // [slices + 1] first position of each slice (multiple of 64)
    std::vector<int32_t> sl_src;          // [positions] caller entry (0-based) at each position, -1 = padding
    std::vector<int32_t> sl_col;          // [positions] column at each position, -1 = padding
    std::vector<int16_t> sl_d16;          // banded: column - (row of the line) at each position, kPad16 = padding (else empty)
    // scatter formats
    int nblocks = 0, ncolors = 0, max_entries = 0, max_lines = 0, max_slots = 0;
    std::vector<ScatterBlock> blocks;     // by block id
    std::vector<int32_t> color_off;       // ncolors + 1
    std::vector<int32_t> phase_blocks;    // block ids ordered by colour (stable)
    std::vector<int32_t> block_color;
    std::vector<int32_t> slot_target;
    std::vector<uint8_t> slot_flag;
    std::vector<int32_t> slot_count;      // contributions per slot (export / checks only)
    std::vector<uint16_t> seg;            // per block nslots + 1 local offsets into its contributions
    std::vector<uint16_t> tl;             // local entry index (k - k0) of every contribution
    // symmetric CSR, sliced blocks (every line of every block <= 8 entries):
    // block b's entries at positions ss_pos[b] + k * nl_b + l (line l of the
    // block, its k-th entry), padded with source -1; contributions then name
    // local positions (ss_tl) instead of local entries
    bool sym_slices = false;
    std::vector<int32_t> ss_pos;          // [nblocks + 1] by block id
    std::vector<int32_t> ss_src;          // [positions] caller entry (0-based), -1 = padding
    std::vector<int32_t> ss_idx;          // [positions] column, -1 = padding
    std::vector<uint16_t> ss_tl;          // [contributions] local position of each contribution
    // symmetric CSR, compact blocks (plan.h); positions in ss_src / ss_idx,
    // contributions (local positions) in ss_tl, slots in slot_target / seg
    bool sym_compact = false;
    // symmetric CSR on a small system: the triangle expanded into full rows
    // and sliced like CSR (sl_src names the caller's entry of each position,
    // an off-diagonal entry twice)
    bool sym_expanded = false;
    std::vector<CompactBlock> cp_blocks;  // [nblocks] in block order
    std::vector<uint16_t> cp_rank;        // [8 n] LDS place of each entry's mirror product (0xffff: none)
    std::vector<int32_t> cp_perm;         // [n] block order: device row k is the caller's row cp_perm[k]
    std::vector<int32_t> cp_block_of;     // [n] block of each line
    int64_t cp_parked = 0;                // parked sums (slots that are not own lines)
    // CSC column panels (format kCsc): entries in panel order
    bool panel = false;
    int64_t pn_width = 0;
    int pn_npanels = 0;
    std::vector<int32_t> pn_src;          // [nnz] caller entry (0-based) of each panel-order entry
    std::vector<int32_t> pn_col;          // [nnz] column of each panel-order entry
    std::vector<int32_t> pn_slot_target;  // [slots] row written
    std::vector<int32_t> pn_slot_ptr;     // [slots + 1] entries of each slot (panel order)
    std::vector<int32_t> pn_slot_panel;   // [slots] panel of each slot (export / checks)
    std::vector<int32_t> pn_chunk_slot;   // [chunks + 1] slots of each chunk
    int32_t pn_first_parked = 0;          // slots >= this belong to colour 1
    // vector kernels
    int vec_blocks = 0, vec_chunk = 0;

    // bytes one sliced product reads from the matrix side (positions, slot
    // descriptors, contribution lists, parked sums); 0 if not sliced
    int64_t slice_stream_bytes() const;
    // ordinary instead of non-temporal matrix loads (kCacheResidentBytes;
    // experiments: CGMI_MATRIX_LOADS = cached | stream); decided once by
    // build_plan
    bool cached = false;
    bool matrix_cached() const { return cached; }
    int scatter_wgs() const { return nblocks < kMaxSpmvBlocks ? nblocks : kMaxSpmvBlocks; }
    int spmv_blocks() const { return format == kCsr || slices ? csr_blocks : scatter_wgs(); }
    int64_t device_bytes() const;
};

// Validates (rules of cg_create) and returns 0-based copies.  vals may be null.
// With CG_LOWER the structure is returned in the upper layout and *perm (if
// given) maps each new entry position to the caller's entry index.
int validate_and_normalise(int fmt, int64_t n, const int32_t *ptr, const int32_t *idx, const double *vals,
                           int base, uint32_t flags, std::vector<int32_t> &ptr0, std::vector<int32_t> &idx0,
                           std::string &err, std::vector<int32_t> *perm = nullptr);

// Builds the plan for 0-based arrays.  target_entries <= 0 selects the default.
int build_plan(int fmt, int64_t n, const int32_t *ptr0, const int32_t *idx0, int target_entries, Plan &plan,
               std::string &err);

int lanes_for_mean_length(double mean_len);

} // namespace cgmi

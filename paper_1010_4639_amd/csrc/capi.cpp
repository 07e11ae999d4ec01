// C-ABI of the cgmi library: handle lifetime, upload, the device-resident CG
// driver and the host-only planning entry points.  Declared in include/cgmi.h.
//
// Solve schedule.  Initialisation (r0 = b - A x0, p0 = r0, ||b||, r0'r0) is
// enqueued once; the iteration then runs from a HIP graph holding `batch`
// iterations (product + fused p'q, r update + fused r'r, x/p update) and a
// final convergence check.  All scalars stay on the device; every kernel
// reads the device status at entry and returns at once when the loop has
// stopped, so the host only looks at a 48-byte state copy after each graph
// launch.  Two launches are kept in flight, so the GPU never waits for the
// host; the extra launch issued after the stop costs only early returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cgmi.h"
#include "kernels.h"
#include "plan.h"

using namespace cgmi;

// The static scratch array of cg_spmv_static (see static_scratch below).
static __device__ __align__(256) double scratch[(32u << 20) / sizeof(double)];

struct cg_handle {
    Plan plan;
    DevMatrix dm;
    int device = 0;
    hipStream_t stream = nullptr;  // caller's stream (null stream by default)
    hipStream_t capture = nullptr; // private stream used only to record the graph
    std::vector<void *> allocs;
    size_t dev_bytes = 0; // sum of the allocations
    double *r = nullptr, *p = nullptr, *q = nullptr, *xw = nullptr;
    double *bp = nullptr; // b in the device row order (renumbered plans)
    // two kernels per CG iteration (small CSR-slice or compact plans): the
    // product forms the direction, which alternates between p and p2
    bool fused = false;
    double *p2 = nullptr;
    double *sig = nullptr, *sig_spmv = nullptr, *rho = nullptr, *bb = nullptr;
    DevState *st = nullptr;
    DevState *host_st = nullptr; // pinned, 2 entries
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int batch = 32;
    int graph_batch = 0;
    // mixed precision (CG_MIXED)
    bool mixed = false;
    DevState *st_in = nullptr; // state of the inner FP32 solves
    float *p32 = nullptr;      // inner search direction, FP32
    double *rout = nullptr;    // outer residual b - A x, FP64
    hipGraph_t graph32 = nullptr;
    hipGraphExec_t gexec32 = nullptr;
    int graph32_batch = 0;
    // caller entry order -> normalised order (lower-triangle input), device copy
    int32_t *perm = nullptr;
    int32_t *flag = nullptr; // device word for checks made by kernels
    std::string err;
};

namespace {

thread_local std::string g_err;

int hip_fail(std::string &err, hipError_t e, const char *what)
{
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CG_ERR_NOMEM : CG_ERR_HIP;
}

#define HIP_TRY(h, call)                                                                                           \
    do {                                                                                                           \
        hipError_t e_ = (call);                                                                                    \
        if (e_ != hipSuccess)                                                                                      \
            return hip_fail((h)->err, e_, #call);                                                                  \
    } while (0)

template <class T>
int dalloc(cg_handle *h, T **out, size_t count)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        return hip_fail(h->err, e, "hipMalloc");
    h->allocs.push_back(p);
    h->dev_bytes += bytes;
    *out = static_cast<T *>(p);
    return CG_OK;
}

template <class T>
int upload(cg_handle *h, T **out, const T *src, size_t count)
{
    int st = dalloc(h, out, count);
    if (st != CG_OK)
        return st;
    if (count) {
        hipError_t e = hipMemcpy(*out, src, count * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_fail(h->err, e, "hipMemcpy");
    }
    return CG_OK;
}

void release(cg_handle *h)
{
    if (h->gexec)
        (void)hipGraphExecDestroy(h->gexec);
    if (h->graph)
        (void)hipGraphDestroy(h->graph);
    if (h->gexec32)
        (void)hipGraphExecDestroy(h->gexec32);
    if (h->graph32)
        (void)hipGraphDestroy(h->graph32);
    for (auto &e : h->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (h->host_st)
        (void)hipHostFree(h->host_st);
    for (void *p : h->allocs)
        (void)hipFree(p);
    if (h->capture)
        (void)hipStreamDestroy(h->capture);
    h->allocs.clear();
}

int upload_all(cg_handle *h, const std::vector<int32_t> &ptr0, const std::vector<int32_t> &idx0, const double *vals)
{
    const Plan &p = h->plan;
    DevMatrix &m = h->dm;
    const int64_t n = p.n;
    m.format = p.format;
    m.n = (int)n;
    m.lanes = p.lanes;
    m.csr_blocks = p.csr_blocks;
    m.csr_rows_per_block = p.csr_rows_per_block;
    m.nblocks = p.nblocks;
    m.ncolors = p.ncolors;
    m.lds_entries = p.max_entries;
    m.lds_lines = p.max_lines;
    m.max_slots = p.max_slots;
    m.color_off = p.color_off;
    m.vec_blocks = p.vec_blocks;
    m.vec_chunk = p.vec_chunk;
    m.matrix_cached = p.matrix_cached();
    int st;
    int32_t *dptr, *didx;
    double *dval;
    if ((st = upload(h, &dptr, ptr0.data(), ptr0.size())) != CG_OK)
        return st;
    if ((st = upload(h, &didx, idx0.data(), idx0.size())) != CG_OK)
        return st;
    if ((st = upload(h, &dval, vals, idx0.size())) != CG_OK)
        return st;
    m.ptr = dptr;
    m.idx = didx;
    m.val = dval;
    if (p.format == kCsr && p.csr_stream) {
        int32_t *rb;
        int2 *rbe;
        std::vector<int2> bnd(p.csr_rb.size());
        for (size_t i = 0; i < bnd.size(); ++i)
            bnd[i] = make_int2(p.csr_rb[i], ptr0[p.csr_rb[i]]);
        if ((st = upload(h, &rb, p.csr_rb.data(), p.csr_rb.size())) != CG_OK ||
            (st = upload(h, &rbe, bnd.data(), bnd.size())) != CG_OK)
            return st;
        m.csr_stream = true;
        m.csr_rb = rb;
        m.csr_rbe = rbe;
        m.csr_nrb = (int)p.csr_rb.size() - 1;
    }
    if (p.slices) {
        int32_t *off, *col = nullptr, *src;
        int16_t *d16 = nullptr;
        double *sv;
        if ((st = upload(h, &off, p.sl_off.data(), p.sl_off.size())) != CG_OK ||
            (p.sl_d16.empty() ? (st = upload(h, &col, p.sl_col.data(), p.sl_col.size()))
                              : (st = upload(h, &d16, p.sl_d16.data(), p.sl_d16.size()))) != CG_OK ||
            (st = upload(h, &src, p.sl_src.data(), p.sl_src.size())) != CG_OK ||
            (st = dalloc(h, &sv, std::max<size_t>(p.sl_src.size(), 1))) != CG_OK)
            return st;
        m.slices = true;
        m.sl_lines = (int)p.sl_lines;
        m.nslices = (int)p.sl_off.size() - 1;
        m.sl_off = off;
        m.sl_col = col;
        m.sl_d16 = d16;
        m.sl_src = src;
        m.sl_val = sv;
        if (h->mixed && (st = dalloc(h, &m.sl_val32, std::max<size_t>(p.sl_src.size(), 1))) != CG_OK)
            return st;
    }
    if (p.panel && n > 0) {
        // CSC column panels: slots of colour 0 first (see plan.h).  A row
        // meets at most two panels, one of each colour (W >= 2 bw + 1), so it
        // has at most one parked sum: parked sums are stored by row, and one
        // flag byte per row says which of y_i (bit 0) and part_i (bit 1) hold
        // a share of (A x)_i.
        const int64_t ns = (int64_t)p.pn_slot_target.size();
        const int32_t fp = p.pn_first_parked;
        std::vector<uint8_t> c0((size_t)n, 0);
        for (int64_t q = 0; q < ns; ++q) {
            const uint8_t bit = q < fp ? 1 : 2;
            if (c0[p.pn_slot_target[q]] & bit) {
                h->err = "internal: a row has two panel slots of one colour";
                return CG_ERR_HIP;
            }
            c0[p.pn_slot_target[q]] |= bit;
        }
        bool gather = false;
        for (int64_t i = 0; i < n; ++i)
            gather = gather || c0[i] != 1;
        int32_t *cs = nullptr, *sp = nullptr, *stg, *pc = nullptr, *src = nullptr;
        uint8_t *dc0;
        double *pv = nullptr, *part;
        if (!p.slices && // chunk kernel: slot pointers, chunks and the entries in panel order
            ((st = upload(h, &cs, p.pn_chunk_slot.data(), p.pn_chunk_slot.size())) != CG_OK ||
             (st = upload(h, &sp, p.pn_slot_ptr.data(), p.pn_slot_ptr.size())) != CG_OK ||
             (st = upload(h, &pc, p.pn_col.data(), p.pn_col.size())) != CG_OK ||
             (st = upload(h, &src, p.pn_src.data(), p.pn_src.size())) != CG_OK ||
             (st = dalloc(h, &pv, p.pn_src.size())) != CG_OK))
            return st;
        if ((st = upload(h, &stg, p.pn_slot_target.data(), p.pn_slot_target.size())) != CG_OK ||
            (st = dalloc(h, &part, (size_t)n)) != CG_OK || (st = upload(h, &dc0, c0.data(), c0.size())) != CG_OK)
            return st;
        m.panel = true;
        m.pn_gather = gather;
        m.pn_chunk_slot = cs;
        m.pn_slot_ptr = sp;
        m.pn_slot_target = stg;
        m.pn_col = pc;
        m.pn_src = src;
        m.pn_val = pv;
        m.pn_first_parked = fp;
        m.part = part;
        m.part_doubles = n;
        m.has_c0 = dc0;
        m.scatter_wgs = p.scatter_wgs();
        if (h->mixed && !p.slices && (st = dalloc(h, &m.pn_val32, p.pn_src.size())) != CG_OK)
            return st;
    } else if (p.sym_compact && n > 0) {
        // compact blocks (plan.h), rows renumbered in block order: row
        // indices (columns, slot targets) converted to it; per row, its
        // parked sums in ascending block order for the row pass
        std::vector<int32_t> inv((size_t)n);
        for (int64_t k = 0; k < n; ++k)
            inv[p.cp_perm[k]] = (int32_t)k;
        std::vector<int32_t> dtg(p.slot_target.size()), didx(p.ss_idx.size());
        for (size_t q = 0; q < dtg.size(); ++q)
            dtg[q] = inv[p.slot_target[q]];
        for (size_t q = 0; q < didx.size(); ++q)
            didx[q] = p.ss_idx[q] < 0 ? -1 : inv[p.ss_idx[q]];
        // parked sums stored by row: row i's sums (ascending block order) at
        // part[rsp[i] .. rsp[i + 1]); each parked slot gets its place there
        std::vector<int32_t> rsp((size_t)n + 1, 0), dest((size_t)p.cp_parked);
        for (const CompactBlock &b : p.cp_blocks)
            for (int32_t s = b.nl; s < b.nslots; ++s)
                rsp[dtg[b.slot0 + s] + 1]++;
        for (int64_t i = 0; i < n; ++i)
            rsp[i + 1] += rsp[i];
        {
            std::vector<int32_t> next(rsp.begin(), rsp.end() - 1);
            for (const CompactBlock &b : p.cp_blocks)
                for (int32_t s = b.nl; s < b.nslots; ++s)
                    dest[b.park0 + (s - b.nl)] = next[dtg[b.slot0 + s]]++;
        }
        CompactBlock *cb;
        int32_t *tg, *drsp, *ddst, *sidx, *ssrc, *vp, *vi;
        uint16_t *sg, *rk;
        double *part, *sv;
        // parked-slot rows padded by one: the product reads a block's first
        // one unguarded, also when the block has none
        dest.push_back(0);
        const size_t np = std::max<size_t>(p.ss_src.size(), 1);
        if ((st = upload(h, &cb, p.cp_blocks.data(), p.cp_blocks.size())) != CG_OK ||
            (st = upload(h, &tg, dtg.data(), dtg.size())) != CG_OK ||
            (st = upload(h, &vp, p.cp_perm.data(), p.cp_perm.size())) != CG_OK ||
            (st = upload(h, &vi, inv.data(), inv.size())) != CG_OK ||
            (st = dalloc(h, &h->bp, (size_t)n)) != CG_OK ||
            (st = upload(h, &sg, p.seg.data(), p.seg.size())) != CG_OK ||
            (st = upload(h, &rk, p.cp_rank.data(), p.cp_rank.size())) != CG_OK ||
            (st = dalloc(h, &part, (size_t)p.cp_parked)) != CG_OK ||
            (st = upload(h, &drsp, rsp.data(), rsp.size())) != CG_OK ||
            (st = upload(h, &ddst, dest.data(), dest.size())) != CG_OK ||
            (st = upload(h, &sidx, didx.data(), didx.size())) != CG_OK ||
            (st = upload(h, &ssrc, p.ss_src.data(), p.ss_src.size())) != CG_OK || (st = dalloc(h, &sv, np)) != CG_OK)
            return st;
        m.compact = true;
        m.vperm = vp;
        m.vinv = vi;
        m.cblocks = cb;
        m.parked = p.cp_parked;
        m.part_doubles = p.cp_parked;
        m.slot_target = tg;
        m.seg = sg;
        m.cp_rank = rk;
        m.part = part;
        m.rs_ptr = drsp;
        m.rs_idx = nullptr; // parked sums already by row
        m.cp_dest = ddst;
        m.has_c0 = nullptr;
        m.ss_idx = sidx;
        m.ss_src = ssrc;
        m.ss_val = sv;
        m.ss_positions = (int64_t)p.ss_src.size();
        m.scatter_wgs = p.scatter_wgs();
        if (h->mixed && (st = dalloc(h, &m.ss_val32, np)) != CG_OK)
            return st;
    } else if (p.format != kCsr && !p.sym_expanded && n > 0) {
        // device arrays in colour order: the blocks of one colour, and their
        // write slots, are contiguous
        const int nb = p.nblocks;
        std::vector<ScatterBlock> ob(nb);
        std::vector<int32_t> otg, cso(p.ncolors + 1, 0);
        std::vector<uint8_t> ofl;
        std::vector<uint16_t> osg;
        otg.reserve(p.slot_target.size());
        ofl.reserve(p.slot_flag.size());
        osg.reserve(p.seg.size());
        for (int i = 0; i < nb; ++i) {
            const ScatterBlock &src = p.blocks[p.phase_blocks[i]];
            ScatterBlock d = src;
            d.slot0 = (int32_t)otg.size();
            d.id = i;
            d.pad = p.block_color[src.id];
            for (int s = 0; s < src.nslots; ++s) {
                otg.push_back(p.slot_target[src.slot0 + s]);
                ofl.push_back(p.slot_flag[src.slot0 + s]);
            }
            for (int s = 0; s <= src.nslots; ++s)
                osg.push_back(p.seg[src.slot0 + src.id + s]);
            cso[d.pad + 1] += src.nslots;
            ob[i] = d;
        }
        for (int c = 0; c < p.ncolors; ++c)
            cso[c + 1] += cso[c];
        // per row: its parked slots (colours >= 1) in ascending colour order,
        // and whether a colour-0 block writes it
        std::vector<int32_t> rsp((size_t)n + 1, 0), rsi;
        std::vector<uint8_t> c0((size_t)n, 0);
        const int32_t first_parked = cso.size() > 1 ? cso[1] : 0;
        for (size_t q = 0; q < otg.size(); ++q) {
            if ((int32_t)q < first_parked)
                c0[otg[q]] = 1;
            else
                rsp[otg[q] + 1]++;
        }
        for (int64_t i = 0; i < n; ++i)
            rsp[i + 1] += rsp[i];
        rsi.resize(rsp[n]);
        {
            std::vector<int32_t> next(rsp.begin(), rsp.end() - 1);
            for (size_t q = first_parked; q < otg.size(); ++q)
                rsi[next[otg[q]]++] = (int32_t)q;
        }
        ScatterBlock *b;
        int32_t *tg, *drsp, *drsi;
        uint8_t *fl, *dc0;
        uint16_t *sg, *tl;
        double *part;
        if ((st = upload(h, &b, ob.data(), ob.size())) != CG_OK ||
            (st = upload(h, &tg, otg.data(), otg.size())) != CG_OK ||
            (st = upload(h, &fl, ofl.data(), ofl.size())) != CG_OK ||
            (st = upload(h, &sg, osg.data(), osg.size())) != CG_OK ||
            (st = upload(h, &tl, (p.sym_slices ? p.ss_tl : p.tl).data(), p.tl.size())) != CG_OK ||
            (st = dalloc(h, &part, otg.size())) != CG_OK || (st = upload(h, &drsp, rsp.data(), rsp.size())) != CG_OK ||
            (st = upload(h, &drsi, rsi.data(), rsi.size())) != CG_OK ||
            (st = upload(h, &dc0, c0.data(), c0.size())) != CG_OK)
            return st;
        m.rs_ptr = drsp;
        m.rs_idx = drsi;
        m.has_c0 = dc0;
        m.blocks = b;
        m.slot_target = tg;
        m.slot_flag = fl;
        m.part_doubles = (int64_t)otg.size();
        m.seg = sg;
        m.tl = tl;
        m.part = part;
        m.color_slot_off = cso;
        m.scatter_wgs = p.scatter_wgs();
        if (p.sym_slices) {
            // per device block (colour order): first position, entries per line
            std::vector<int2> sb(nb);
            for (int i = 0; i < nb; ++i) {
                const ScatterBlock &src = p.blocks[p.phase_blocks[i]];
                const int32_t q0 = p.ss_pos[src.id], q1 = p.ss_pos[src.id + 1];
                sb[i] = make_int2(q0, (q1 - q0) / (src.line1 - src.line0));
            }
            int2 *dsb;
            int32_t *sidx, *ssrc;
            double *sv;
            const size_t np = std::max<size_t>(p.ss_src.size(), 1);
            if ((st = upload(h, &dsb, sb.data(), sb.size())) != CG_OK ||
                (st = upload(h, &sidx, p.ss_idx.data(), p.ss_idx.size())) != CG_OK ||
                (st = upload(h, &ssrc, p.ss_src.data(), p.ss_src.size())) != CG_OK ||
                (st = dalloc(h, &sv, np)) != CG_OK)
                return st;
            m.sym_slices = true;
            m.ss_blk = dsb;
            m.ss_idx = sidx;
            m.ss_src = ssrc;
            m.ss_val = sv;
            m.ss_positions = (int64_t)p.ss_src.size();
            if (h->mixed && (st = dalloc(h, &m.ss_val32, np)) != CG_OK)
                return st;
        }
    }
    const size_t nv = (size_t)std::max<int64_t>(n, 1);
    if ((st = dalloc(h, &h->r, nv)) != CG_OK || (st = dalloc(h, &h->p, nv)) != CG_OK ||
        (st = dalloc(h, &h->q, nv)) != CG_OK || (st = dalloc(h, &h->xw, nv)) != CG_OK)
        return st;
    // Two kernels per iteration where launches, not bytes, bound the
    // iteration: vector kernels of at most 256 workgroups (n <= 65 536).
    // There every product workgroup reducing the r'r partials and gathering
    // r and p costs less than the third launch; on large systems it costs
    // more.  Experiments: CGMI_FUSED=0 / 1 (1: wherever the plan allows).
    bool fuse = p.vec_blocks <= kBlock;
    if (const char *e = std::getenv("CGMI_FUSED"))
        fuse = std::strcmp(e, "0") != 0;
    h->fused = fuse && n > 0 && ((m.slices && !m.panel) || m.compact);
    if (h->fused && (st = dalloc(h, &h->p2, nv)) != CG_OK)
        return st;
    const size_t ns = (size_t)std::max(1, std::max(p.spmv_blocks(), p.vec_blocks));
    if ((st = dalloc(h, &h->sig, ns)) != CG_OK || (st = dalloc(h, &h->sig_spmv, ns)) != CG_OK ||
        (st = dalloc(h, &h->rho, ns)) != CG_OK || (st = dalloc(h, &h->bb, ns)) != CG_OK ||
        (st = dalloc(h, &h->st, 1)) != CG_OK)
        return st;
    if (h->mixed && n > 0) {
        // FP32 copy of D^-1/2 A D^-1/2 and D^-1/2 itself: filled by mixed_rescale
        float *dv32;
        double *dsc;
        if ((st = dalloc(h, &dv32, idx0.size())) != CG_OK || (st = dalloc(h, &dsc, (size_t)n)) != CG_OK ||
            (st = dalloc(h, &h->p32, nv)) != CG_OK || (st = dalloc(h, &h->rout, nv)) != CG_OK ||
            (st = dalloc(h, &h->st_in, 1)) != CG_OK)
            return st;
        m.val32 = dv32;
        m.dscale = dsc;
    }
    hipError_t e = hipHostMalloc((void **)&h->host_st, 2 * sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess)
        return hip_fail(h->err, e, "hipHostMalloc");
    std::memset(h->host_st, 0, 2 * sizeof(DevState));
    for (auto &ev : h->ev)
        HIP_TRY(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(h, hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
    return CG_OK;
}

void fill_stats(const Plan &p, cg_plan_stats *s)
{
    std::memset(s, 0, sizeof(*s));
    s->n = p.n;
    s->nnz = p.nnz;
    s->format = p.format;
    s->lanes_per_line = p.lanes;
    s->spmv_blocks = p.spmv_blocks();
    s->scatter_blocks = p.nblocks;
    s->vec_blocks = p.vec_blocks;
    s->colors = p.ncolors;
    s->max_block_entries = p.max_entries;
    s->slices = !p.sl_d16.empty() ? 2 : p.slices || p.sym_slices || p.sym_compact ? 1 : 0;
    s->compact = p.sym_compact ? 1 : 0;
    s->parked = p.sym_compact ? p.cp_parked : 0;
    s->cached_loads = p.matrix_cached() ? 1 : 0;
    s->slots = p.panel ? (int64_t)p.pn_slot_target.size() : (int64_t)p.slot_target.size();
    s->plan_bytes = p.device_bytes();
}

// experiments: CGMI_MIXED_RESTART=1 restarts every inner solve from p = r
// instead of keeping the previous inner solve's next direction
bool restart_inner()
{
    const char *e = std::getenv("CGMI_MIXED_RESTART");
    return e && std::atoi(e) != 0;
}

int scatter_entries_override()
{
    const char *e = std::getenv("CGMI_SCATTER_ENTRIES");
    return e ? std::atoi(e) : 0;
}

// One CG iteration on the handle's vectors, in CG (gated) mode.
void enqueue_iteration(cg_handle *h, hipStream_t s, int parity)
{
    IterCtx c;
    c.st = h->st;
    c.rho_part = h->rho;
    c.n_rho = h->dm.vec_blocks;
    c.defer_rows = true;
    if (h->fused) {
        // product with the direction update (p_(k-1) in one buffer, p_k
        // written to the other), then the r update
        c.fused = true;
        c.pold = parity ? h->p2 : h->p;
        c.pnew = parity ? h->p : h->p2;
        c.r = h->r;
        c.x = h->xw;
        launch_spmv(h->dm, c.pold, h->q, h->sig, c, s);
        launch_update_r(h->dm, h->r, h->q, h->st, h->sig, h->rho, s, true, true);
        return;
    }
    launch_spmv(h->dm, h->p, h->q, h->sig, c, s);
    launch_update_r(h->dm, h->r, h->q, h->st, h->sig, h->rho, s, true);
    launch_update_xp(h->dm, h->xw, h->p, h->r, h->st, h->rho, s);
}

// One inner (mixed-precision) iteration: FP32 product, FP64 r update, FP64 c
// update with the FP32 search direction.
void enqueue_iteration32(cg_handle *h, hipStream_t s)
{
    IterCtx c;
    c.st = h->st_in;
    c.defer_rows = true;
    launch_spmv32(h->dm, h->p32, h->q, h->sig, c, s);
    launch_update_r(h->dm, h->r, h->q, h->st_in, h->sig, h->rho, s, true);
    launch_update_xp32(h->dm, h->p, h->p32, h->r, h->st_in, h->rho, s);
}

int build_graph_generic(cg_handle *h, bool mixed)
{
    hipGraph_t &g = mixed ? h->graph32 : h->graph;
    hipGraphExec_t &ge = mixed ? h->gexec32 : h->gexec;
    int &gb = mixed ? h->graph32_batch : h->graph_batch;
    if (ge && gb == h->batch)
        return CG_OK;
    if (ge) {
        (void)hipGraphExecDestroy(ge);
        ge = nullptr;
    }
    if (g) {
        (void)hipGraphDestroy(g);
        g = nullptr;
    }
    HIP_TRY(h, hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
    // The inner solves of mixed precision are short (about 100 iterations at
    // inner tolerance 1e-2), and the launches that run past each one's stop
    // are paid at every refinement step: their graph holds at most 8
    // iterations (160^3, CSR: 72.5 ms with 32, 68.8 with 16, 67.8 with 8).
    // Experiments: CGMI_MIXED_BATCH = iterations per launch of the inner solves.
    int nb = mixed ? std::min(h->batch, 8) : h->batch;
    if (mixed)
        if (const char *e = std::getenv("CGMI_MIXED_BATCH"))
            nb = std::max(1, std::atoi(e));
    const bool fused = !mixed && h->fused;
    if (fused) // the directions alternate between two buffers: an even count
        nb += nb & 1;
    for (int i = 0; i < nb; ++i) {
        if (mixed)
            enqueue_iteration32(h, h->capture);
        else
            enqueue_iteration(h, h->capture, i & 1);
    }
    // (the fused iteration records its stops in its own r update)
    if (!fused)
        launch_check(h->dm, mixed ? h->st_in : h->st, h->rho, h->capture);
    hipError_t e = hipStreamEndCapture(h->capture, &g);
    if (e != hipSuccess)
        return hip_fail(h->err, e, "hipStreamEndCapture");
    HIP_TRY(h, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    gb = h->batch;
    return CG_OK;
}

int build_graph(cg_handle *h)
{
    return build_graph_generic(h, false);
}

// Replays `ge` (two launches in flight) until the device status of `st`
// leaves kRun; returns the final status through *status.
int run_until_stop(cg_handle *h, hipGraphExec_t ge, DevState *st, int32_t *status)
{
    hipStream_t s = h->stream;
    hipError_t e;
    auto launch = [&](int slot) -> hipError_t {
        hipError_t r = hipGraphLaunch(ge, s);
        if (r == hipSuccess)
            r = hipMemcpyAsync(&h->host_st[slot], st, sizeof(DevState), hipMemcpyDeviceToHost, s);
        if (r == hipSuccess)
            r = hipEventRecord(h->ev[slot], s);
        return r;
    };
    if ((e = launch(0)) != hipSuccess)
        return hip_fail(h->err, e, "hipGraphLaunch");
    for (int i = 0;; ++i) {
        if ((e = launch((i + 1) & 1)) != hipSuccess)
            return hip_fail(h->err, e, "hipGraphLaunch");
        if ((e = hipEventSynchronize(h->ev[i & 1])) != hipSuccess)
            return hip_fail(h->err, e, "hipEventSynchronize");
        *status = h->host_st[i & 1].status;
        if (*status != kRun)
            return CG_OK;
    }
}

int read_state(cg_handle *h, DevState *st, DevState *out)
{
    hipError_t e;
    if ((e = hipMemcpyAsync(&h->host_st[0], st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return hip_fail(h->err, e, "state readback");
    *out = h->host_st[0];
    return CG_OK;
}

// Mixed precision: D^-1/2 and the FP32 copy of D^-1/2 A D^-1/2 from the
// current FP64 values (each scaled value formed in FP64, rounded once), on
// the handle's stream; blocks to read the diagonal check.
int mixed_rescale(cg_handle *h)
{
    hipStream_t s = h->stream;
    HIP_TRY(h, hipMemsetAsync(h->flag, 0, sizeof(int32_t), s));
    double *sc = const_cast<double *>(h->dm.dscale);
    if (h->dm.vperm != nullptr) // D^-1/2 by the caller's rows first, then in the device order
        sc = h->q;
    launch_mx_rescale(h->dm, sc, const_cast<float *>(h->dm.val32), h->flag, s);
    if (h->dm.vperm != nullptr)
        launch_permute(h->dm.n, sc, h->dm.vperm, const_cast<double *>(h->dm.dscale), s);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(&h->host_st[0].pad, h->flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (h->host_st[0].pad) {
        h->err = "CG_MIXED needs a positive, finite diagonal entry in every line";
        return CG_ERR_ARG;
    }
    return CG_OK;
}

// Every array derived from the FP64 values (CSC panel order, the mixed
// FP32 scaled copy) rebuilt from dm.val, on the handle's stream.
int refresh_values(cg_handle *h)
{
    DevMatrix &m = h->dm;
    const int64_t nnz = h->plan.nnz;
    if (m.panel && !m.slices)
        launch_permute(nnz, m.val, m.pn_src, m.pn_val, h->stream);
    if (m.slices)
        launch_permute((int64_t)h->plan.sl_src.size(), m.val, m.sl_src, m.sl_val, h->stream);
    if (m.sym_slices || m.compact)
        launch_permute(m.ss_positions, m.val, m.ss_src, m.ss_val, h->stream);
    HIP_TRY(h, hipGetLastError());
    if (h->mixed && m.n > 0) {
        const int st = mixed_rescale(h);
        if (st != CG_OK)
            return st;
        if (m.panel && !m.slices)
            launch_permute(nnz, m.val32, m.pn_src, m.pn_val32, h->stream);
        if (m.slices)
            launch_permute((int64_t)h->plan.sl_src.size(), m.val32, m.sl_src, m.sl_val32, h->stream);
        if (m.sym_slices || m.compact)
            launch_permute(m.ss_positions, m.val32, m.ss_src, m.ss_val32, h->stream);
        HIP_TRY(h, hipGetLastError());
    }
    return CG_OK;
}

// Scratch of cg_spmv_static (dot partials and parked sums of one product):
// a fixed array in device memory, one copy on every GPU the library runs on,
// held until the process ends.  Host code never uses the name itself as an
// address: static_scratch looks up each device's copy once.
constexpr size_t kStaticScratchDoubles = (32u << 20) / sizeof(double); // 32 MiB
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the static scratch on the handle's device, which must
// be the current device.
int static_scratch(cg_handle *h, double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(h->err, e, "hipGetDevice");
    if (dev != h->device || dev < 0 || dev >= kMaxScratchDevices) {
        h->err = "cg_spmv_static: the current device is not the handle's";
        return CG_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(h->err, e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CG_OK;
}

// Vectors in and out of the device row order (compact symmetric plans
// renumber their rows; every other plan keeps the caller's order).
// into(): src in the caller's order -> dst in the device order; returns the
// vector the device uses.  out_of(): device order -> caller's order.
const double *vec_into(cg_handle *h, const double *src, double *dst)
{
    if (h->dm.vperm == nullptr)
        return src;
    launch_permute(h->dm.n, src, h->dm.vperm, dst, h->stream);
    return dst;
}

hipError_t vec_out_of(cg_handle *h, const double *src, double *dst)
{
    if (h->dm.vinv == nullptr)
        return hipMemcpyAsync(dst, src, sizeof(double) * (size_t)h->dm.n, hipMemcpyDeviceToDevice, h->stream);
    launch_permute(h->dm.n, src, h->dm.vinv, dst, h->stream);
    return hipGetLastError();
}

int status_to_code(int32_t s)
{
    switch (s) {
    case kConverged:
    case kZeroRhs: return CG_OK;
    case kMaxit: return CG_NOT_CONVERGED;
    case kBreakdown: return CG_ERR_BREAKDOWN;
    case kNonfinite: return CG_ERR_NONFINITE;
    default: return CG_ERR_HIP;
    }
}

} // namespace

extern "C" {

int cg_analyze(int format, int64_t n, const int32_t *ptr, const int32_t *idx, const double *vals, int index_base,
               uint32_t flags, cg_plan_stats *stats)
{
    std::vector<int32_t> p0, i0;
    std::string err;
    int st;
    try {
        st = validate_and_normalise(format, n, ptr, idx, vals, index_base, flags, p0, i0, err);
        if (st == CG_OK) {
            Plan plan;
            st = build_plan(format, n, p0.data(), i0.data(), scatter_entries_override(), plan, err);
            if (st == CG_OK && stats)
                fill_stats(plan, stats);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed";
        st = CG_ERR_NOMEM;
    }
    g_err = st == CG_OK ? std::string() : err;
    return st;
}

int cg_analyze_export(int format, int64_t n, const int32_t *ptr, const int32_t *idx, int index_base,
                      int32_t *blk_color, int32_t *blk_line0, int32_t *blk_line1, int32_t *blk_entry0,
                      int32_t *blk_entry1, int64_t *blk_slot0, int32_t *slot_target, uint8_t *slot_flags,
                      int32_t *slot_count)
{
    if (format == kCsr) {
        g_err = "CSR has no scatter plan";
        return CG_ERR_ARG;
    }
    if (format == kCsc) {
        g_err = "CSC uses the column-panel plan (cg_analyze_panels)";
        return CG_ERR_ARG;
    }
    std::vector<int32_t> p0, i0;
    std::string err;
    int st;
    try {
        st = validate_and_normalise(format, n, ptr, idx, nullptr, index_base, 0, p0, i0, err);
        Plan plan;
        if (st == CG_OK)
            st = build_plan(format, n, p0.data(), i0.data(), scatter_entries_override(), plan, err);
        if (st == CG_OK && plan.sym_compact) {
            err = "this symmetric matrix is planned in compact blocks (cg_analyze_compact)";
            st = CG_ERR_ARG;
        }
        if (st == CG_OK) {
            for (int b = 0; b < plan.nblocks; ++b) {
                const ScatterBlock &bk = plan.blocks[b];   // block-id order
                if (blk_color) blk_color[b] = plan.block_color[b];
                if (blk_line0) blk_line0[b] = bk.line0;
                if (blk_line1) blk_line1[b] = bk.line1;
                if (blk_entry0) blk_entry0[b] = bk.k0;
                if (blk_entry1) blk_entry1[b] = bk.k1;
                if (blk_slot0) blk_slot0[b] = bk.slot0;
            }
            if (blk_slot0) blk_slot0[plan.nblocks] = (int64_t)plan.slot_target.size();
            const size_t ns = plan.slot_target.size();
            if (slot_target) std::memcpy(slot_target, plan.slot_target.data(), ns * 4);
            if (slot_flags) std::memcpy(slot_flags, plan.slot_flag.data(), ns);
            if (slot_count) std::memcpy(slot_count, plan.slot_count.data(), ns * 4);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed";
        st = CG_ERR_NOMEM;
    }
    g_err = st == CG_OK ? std::string() : err;
    return st;
}

int cg_analyze_compact(int64_t n, const int32_t *ptr, const int32_t *idx, int index_base, int32_t *block_of,
                       int64_t *blk_slot0, int32_t *blk_lines, int32_t *slot_target, int32_t *slot_count)
{
    std::vector<int32_t> p0, i0;
    std::string err;
    int st;
    try {
        st = validate_and_normalise(kSymCsr, n, ptr, idx, nullptr, index_base, 0, p0, i0, err);
        Plan plan;
        if (st == CG_OK)
            st = build_plan(kSymCsr, n, p0.data(), i0.data(), scatter_entries_override(), plan, err);
        if (st == CG_OK && !plan.sym_compact) {
            err = "this matrix is not planned in compact blocks";
            st = CG_ERR_ARG;
        }
        if (st == CG_OK) {
            if (block_of)
                std::memcpy(block_of, plan.cp_block_of.data(), (size_t)n * 4);
            for (int b = 0; b < plan.nblocks; ++b) {
                if (blk_slot0)
                    blk_slot0[b] = plan.cp_blocks[b].slot0;
                if (blk_lines)
                    blk_lines[b] = plan.cp_blocks[b].nl;
            }
            if (blk_slot0)
                blk_slot0[plan.nblocks] = (int64_t)plan.slot_target.size();
            const size_t ns = plan.slot_target.size();
            if (slot_target)
                std::memcpy(slot_target, plan.slot_target.data(), ns * 4);
            if (slot_count)
                std::memcpy(slot_count, plan.slot_count.data(), ns * 4);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed";
        st = CG_ERR_NOMEM;
    }
    g_err = st == CG_OK ? std::string() : err;
    return st;
}

int cg_analyze_panels(int64_t n, const int32_t *ptr, const int32_t *idx, int index_base, int64_t *width,
                      int32_t *entry_src, int32_t *slot_target, int32_t *slot_ptr, int32_t *slot_panel,
                      int32_t *chunk_slot, int32_t *first_parked)
{
    std::vector<int32_t> p0, i0;
    std::string err;
    int st;
    try {
        st = validate_and_normalise(kCsc, n, ptr, idx, nullptr, index_base, 0, p0, i0, err);
        Plan plan;
        if (st == CG_OK)
            st = build_plan(kCsc, n, p0.data(), i0.data(), 0, plan, err);
        if (st == CG_OK) {
            const size_t ns = plan.pn_slot_target.size();
            if (width) *width = plan.pn_width;
            if (first_parked) *first_parked = plan.pn_first_parked;
            if (entry_src) std::memcpy(entry_src, plan.pn_src.data(), plan.pn_src.size() * 4);
            if (slot_target) std::memcpy(slot_target, plan.pn_slot_target.data(), ns * 4);
            if (slot_ptr) std::memcpy(slot_ptr, plan.pn_slot_ptr.data(), plan.pn_slot_ptr.size() * 4);
            if (slot_panel) std::memcpy(slot_panel, plan.pn_slot_panel.data(), ns * 4);
            if (chunk_slot) std::memcpy(chunk_slot, plan.pn_chunk_slot.data(), plan.pn_chunk_slot.size() * 4);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed";
        st = CG_ERR_NOMEM;
    }
    g_err = st == CG_OK ? std::string() : err;
    return st;
}

int cg_create(cg_handle **out, int format, int64_t n, const int32_t *ptr, const int32_t *idx, const double *vals,
              int index_base, uint32_t flags)
{
    if (!out) {
        g_err = "out is NULL";
        return CG_ERR_ARG;
    }
    *out = nullptr;
    std::unique_ptr<cg_handle> h;
    try {
        h.reset(new cg_handle());
        std::vector<int32_t> p0, i0, perm;
        int st = validate_and_normalise(format, n, ptr, idx, vals, index_base, flags, p0, i0, h->err, &perm);
        if (st == CG_OK && n > 0 && p0[n] > 0 && !vals) {
            h->err = "vals is NULL";
            st = CG_ERR_ARG;
        }
        std::vector<double> pvals;
        if (st == CG_OK && !perm.empty()) { // lower-triangle input: values follow the transposed layout
            pvals.resize(perm.size());
            for (size_t k = 0; k < perm.size(); ++k)
                pvals[k] = vals[perm[k]];
            vals = pvals.data();
        }
        if (st == CG_OK)
            st = build_plan(format, n, p0.data(), i0.data(), scatter_entries_override(), h->plan, h->err);
        h->mixed = (flags & CG_MIXED) != 0;
        if (st == CG_OK) {
            hipError_t e = hipGetDevice(&h->device);
            st = e == hipSuccess ? upload_all(h.get(), p0, i0, vals) : hip_fail(h->err, e, "hipGetDevice");
        }
        if (st == CG_OK && !perm.empty())
            st = upload(h.get(), &h->perm, perm.data(), perm.size());
        if (st == CG_OK)
            st = dalloc(h.get(), &h->flag, 1);
        if (st == CG_OK)
            st = refresh_values(h.get());
        if (st != CG_OK) {
            g_err = h->err;
            release(h.get());
            return st;
        }
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        if (h)
            release(h.get());
        return CG_ERR_NOMEM;
    }
    g_err.clear();
    *out = h.release();
    return CG_OK;
}

int cg_set_stream(cg_handle *h, void *hip_stream)
{
    if (!h)
        return CG_ERR_ARG;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return CG_OK;
}

int cg_set_batch(cg_handle *h, int32_t iters_per_launch)
{
    if (!h || iters_per_launch < 1 || iters_per_launch > 4096)
        return CG_ERR_ARG;
    h->batch = iters_per_launch;
    return CG_OK;
}

int cg_spmv(cg_handle *h, const double *x, double *y)
{
    if (!h)
        return CG_ERR_ARG;
    if (h->dm.n == 0)
        return CG_OK;
    if (!x || !y || x == y) {
        h->err = "x / y NULL or aliased";
        return CG_ERR_ARG;
    }
    if (h->dm.vperm != nullptr) { // through the device row order
        launch_spmv(h->dm, vec_into(h, x, h->p), h->q, h->sig_spmv, IterCtx{}, h->stream);
        HIP_TRY(h, vec_out_of(h, h->q, y));
    } else {
        launch_spmv(h->dm, x, y, h->sig_spmv, IterCtx{}, h->stream);
    }
    HIP_TRY(h, hipGetLastError());
    return CG_OK;
}

int cg_spmv_static(cg_handle *h, const double *x, double *y)
{
    if (!h)
        return CG_ERR_ARG;
    if (h->dm.n == 0)
        return CG_OK;
    if (!x || !y || x == y) {
        h->err = "x / y NULL or aliased";
        return CG_ERR_ARG;
    }
    // dot partials first (rounded up to 256 bytes), then the parked sums
    const int64_t nsig = ((int64_t)std::max(1, h->dm.spmv_blocks()) + 31) / 32 * 32;
    const int64_t need = nsig + h->dm.part_doubles;
    if (need > (int64_t)kStaticScratchDoubles) {
        h->err = "cg_spmv_static: the product needs " + std::to_string(need * 8) + " scratch bytes, more than the " +
                 std::to_string(kStaticScratchDoubles * 8) + " of the static array (use cg_spmv)";
        return CG_ERR_ARG;
    }
    double *base = nullptr;
    const int st = static_scratch(h, &base);
    if (st != CG_OK)
        return st;
    IterCtx c;
    c.part = h->dm.part_doubles > 0 ? base + nsig : nullptr;
    if (h->dm.vperm != nullptr) { // through the device row order (the handle's own vectors, no allocation)
        launch_spmv(h->dm, vec_into(h, x, h->p), h->q, base, c, h->stream);
        HIP_TRY(h, vec_out_of(h, h->q, y));
    } else {
        launch_spmv(h->dm, x, y, base, c, h->stream);
    }
    HIP_TRY(h, hipGetLastError());
    return CG_OK;
}

int cg_solve(cg_handle *h, const double *b, double *x, double tol, int32_t maxit, cg_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    cg_info loc{};
    if (!info)
        info = &loc;
    std::memset(info, 0, sizeof(*info));
    auto done = [&](int code) {
        info->status = code;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return code;
    };
    if (!h)
        return done(CG_ERR_ARG);
    if (!(tol >= 0.0) || maxit < 0) {
        h->err = "tol must be >= 0 and maxit >= 0";
        return done(CG_ERR_ARG);
    }
    const int n = h->dm.n;
    if (n == 0)
        return done(CG_OK);
    if (!b || !x || b == x) {
        h->err = "b / x NULL or the same buffer";
        return done(CG_ERR_ARG);
    }
    hipStream_t s = h->stream;
    int st = build_graph(h);
    if (st != CG_OK)
        return done(st);
    // initialisation (b and x0 in the device row order)
    const double *bi = vec_into(h, b, h->bp);
    const double *x0 = vec_into(h, x, h->xw);
    launch_spmv(h->dm, x0, h->q, h->sig_spmv, IterCtx{}, s);
    launch_init_vec(h->dm, bi, x0, h->q, h->r, h->p, h->xw, h->rho, h->bb, s);
    launch_init_state(h->dm, h->st, h->bb, h->rho, tol, maxit, s);
    if (h->fused) // the first fused step forms p_0 = r_0 + beta * 0
        launch_fill(n, h->p, 0.0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return done(hip_fail(h->err, e, "launch"));
    // iteration: two graph launches in flight, poll the older one's state
    int32_t status = kRun;
    if ((st = run_until_stop(h, h->gexec, h->st, &status)) != CG_OK)
        return done(st);
    // finish: copy x out, true residual of the returned x
    if (status == kConverged || status == kMaxit || status == kBreakdown) {
        e = vec_out_of(h, h->xw, x);
        if (e != hipSuccess)
            return done(hip_fail(h->err, e, "copy-out"));
        launch_spmv(h->dm, h->xw, h->q, h->sig_spmv, IterCtx{}, s);
        launch_true_residual(h->dm, bi, h->q, h->bb, h->st, s);
    } else if (status == kZeroRhs) {
        launch_fill(n, x, 0.0, s);
    }
    if ((e = hipMemcpyAsync(&h->host_st[0], h->st, sizeof(DevState), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(hip_fail(h->err, e, "final state readback"));
    const DevState &d = h->host_st[0];
    info->iters = d.iters;
    info->relres = d.nb > 0.0 ? std::sqrt(d.rho) / d.nb : 0.0;
    info->relres_true = d.res_true;
    if (d.status == kNonfinite) {
        info->relres = 0.0;
        h->err = "b has a non-finite entry";
    } else if (d.status == kBreakdown) {
        h->err = "p'Ap <= 0 or non-finite: matrix not SPD";
    }
    return done(status_to_code(d.status));
}

int cg_solve_mixed(cg_handle *h, const double *b, double *x, double tol, int32_t maxit, double inner_tol,
                   int32_t max_outer, cg_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    cg_info loc{};
    if (!info)
        info = &loc;
    std::memset(info, 0, sizeof(*info));
    auto done = [&](int code) {
        info->status = code;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return code;
    };
    if (!h)
        return done(CG_ERR_ARG);
    if (!h->mixed) {
        h->err = "handle was created without CG_MIXED";
        return done(CG_ERR_ARG);
    }
    if (!(tol >= 0.0) || maxit < 0 || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1) {
        h->err = "need tol >= 0, maxit >= 0, 0 < inner_tol < 1, max_outer >= 1";
        return done(CG_ERR_ARG);
    }
    const int n = h->dm.n;
    if (n == 0)
        return done(CG_OK);
    if (!b || !x || b == x) {
        h->err = "b / x NULL or the same buffer";
        return done(CG_ERR_ARG);
    }
    hipStream_t s = h->stream;
    int st = build_graph_generic(h, true);
    if (st != CG_OK)
        return done(st);
    // outer start: r = b - A x0, ||b||, ||r|| (FP64 product; device row order)
    const double *bi = vec_into(h, b, h->bp);
    const double *x0 = vec_into(h, x, h->xw);
    launch_spmv(h->dm, x0, h->q, h->sig_spmv, IterCtx{}, s);
    launch_init_vec(h->dm, bi, x0, h->q, h->rout, h->p, h->xw, h->rho, h->bb, s);
    launch_init_state(h->dm, h->st, h->bb, h->rho, tol, maxit, s);
    DevState out;
    if ((st = read_state(h, h->st, &out)) != CG_OK)
        return done(st);
    if (out.status == kNonfinite) {
        h->err = "b has a non-finite entry";
        return done(CG_ERR_NONFINITE);
    }
    if (out.status == kZeroRhs) {
        launch_fill(n, x, 0.0, s);
        (void)hipStreamSynchronize(s);
        return done(CG_OK);
    }
    const double nb = out.nb;
    double relres = std::sqrt(out.rho) / nb;
    int total = 0, outer = 0, code = CG_NOT_CONVERGED;
    bool keep_p = false; // the previous inner solve converged: its next direction carries over
    while (true) {
        if (relres <= tol) {
            code = CG_OK;
            break;
        }
        if (outer >= max_outer || total >= maxit)
            break;
        // inner solve of (D^-1/2 A D^-1/2) c = D^-1/2 r in FP32 storage
        launch_mx_init(h->dm, h->rout, h->r, h->p32, h->p, h->rho, h->bb, s, keep_p && !restart_inner());
        launch_init_state(h->dm, h->st_in, h->bb, h->rho, inner_tol, maxit - total, s);
        int32_t status = kRun;
        if ((st = run_until_stop(h, h->gexec32, h->st_in, &status)) != CG_OK)
            return done(st);
        DevState in;
        if ((st = read_state(h, h->st_in, &in)) != CG_OK)
            return done(st);
        total += in.iters;
        ++outer;
        keep_p = in.status == kConverged && in.iters > 0;
        if (in.status == kBreakdown && in.iters == 0) {
            h->err = "inner FP32 solve broke down before any step";
            code = CG_ERR_BREAKDOWN;
            break;
        }
        // x += D^-1/2 c; r = b - A x (FP64 product), true residual norm
        launch_mx_apply(h->dm, h->xw, h->p, s);
        launch_spmv(h->dm, h->xw, h->q, h->sig_spmv, IterCtx{}, s);
        launch_init_vec(h->dm, bi, h->xw, h->q, h->rout, h->p, h->xw, h->rho, h->bb, s);
        launch_outer_norm(h->dm, h->st, h->rho, s);
        if ((st = read_state(h, h->st, &out)) != CG_OK)
            return done(st);
        relres = std::sqrt(out.rho) / nb;
        if (!std::isfinite(relres)) {
            h->err = "refinement produced a non-finite residual";
            code = CG_ERR_BREAKDOWN;
            break;
        }
    }
    hipError_t e = vec_out_of(h, h->xw, x);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return done(hip_fail(h->err, e, "copy-out"));
    info->iters = total;
    info->outer = outer;
    info->relres = relres;
    info->relres_true = relres;
    return done(code);
}

int cg_set_values(cg_handle *h, const double *vals)
{
    if (!h)
        return CG_ERR_ARG;
    const int64_t nnz = h->plan.nnz;
    if (nnz == 0)
        return CG_OK;
    if (!vals) {
        h->err = "vals is NULL";
        return CG_ERR_ARG;
    }
    hipStream_t s = h->stream;
    launch_set_values(nnz, vals, h->perm, const_cast<double *>(h->dm.val), s);
    HIP_TRY(h, hipGetLastError());
    return refresh_values(h);
}

int cg_pattern_grad(cg_handle *h, const double *lam, const double *x, double *grad)
{
    if (!h)
        return CG_ERR_ARG;
    if (h->plan.nnz == 0)
        return CG_OK;
    if (!lam || !x || !grad) {
        h->err = "lam / x / grad NULL";
        return CG_ERR_ARG;
    }
    launch_pattern_grad(h->dm, lam, x, h->perm, grad, h->stream);
    HIP_TRY(h, hipGetLastError());
    return CG_OK;
}

int cg_get_stats(const cg_handle *h, cg_plan_stats *stats)
{
    if (!h || !stats)
        return CG_ERR_ARG;
    fill_stats(h->plan, stats);
    stats->device_bytes = (int64_t)h->dev_bytes;
    return CG_OK;
}

void cg_destroy(cg_handle *h)
{
    if (!h)
        return;
    (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
}

const char *cg_status_string(int status)
{
    switch (status) {
    case CG_OK: return "converged";
    case CG_NOT_CONVERGED: return "maxit reached before tol";
    case CG_ERR_ARG: return "invalid argument";
    case CG_ERR_STRUCTURE: return "malformed sparse structure";
    case CG_ERR_BREAKDOWN: return "breakdown: p'Ap <= 0 (matrix not SPD)";
    case CG_ERR_NONFINITE: return "non-finite value";
    case CG_ERR_NOMEM: return "out of memory";
    case CG_ERR_HIP: return "HIP runtime error";
    case CG_ERR_UNSUPPORTED: return "structure not supported by the scatter plan";
    default: return "unknown status";
    }
}

const char *cg_last_error(const cg_handle *h)
{
    return h ? h->err.c_str() : g_err.c_str();
}

} // extern "C"

// HIP kernels for gfx950 (CDNA4, wave64): sparse products over CSR, symmetric
// CSR and CSC, and the fused vector / reduction steps of conjugate gradient.
//
// All kernels use 256-thread workgroups.  Every reduction is a fixed tree
// (butterfly inside a wavefront, waves summed in index order, partials summed
// by a fixed per-thread stride), so results are bitwise reproducible.  No
// floating-point atomics anywhere; the only cross-workgroup communication is
// through per-workgroup partials read by a later kernel.
#include "kernels.h"
#include "devutil.h"

#include <cmath>
#include <cstdlib>
#include <cstring>

namespace cgmi {

namespace {

using namespace dev;

// Loads of the matrix streams.  NT: non-temporal (read once per product, do
// not displace the vectors); otherwise ordinary loads, so that a matrix that
// fits the 256 MB Infinity Cache together with the vectors stays resident
// from one CG iteration to the next.
template <bool NT, class T>
__device__ __forceinline__ T matrix_load(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Two-element vectors for the paired loads of the sliced layout (native
// vector types, which the non-temporal load builtin accepts).
typedef int int2v __attribute__((ext_vector_type(2)));
typedef unsigned int uint4v __attribute__((ext_vector_type(4)));
template <class T>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<int32_t> {
    typedef int32_t type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<int16_t> {
    typedef int16_t type __attribute__((ext_vector_type(2)));
};

// Column of a slice entry: stored as is (int32_t, -1 = padding) or as its
// offset from the line's row (int16_t, kPad16 = padding).
__device__ __forceinline__ int col_of(int32_t raw, int) { return raw; }
__device__ __forceinline__ int col_of(int16_t raw, int row) { return raw == kPad16 ? -1 : row + raw; }

// Start of an iteration (before its product): stop when the current residual
// meets the tolerance (decided and published by the previous x/p update, or by
// the initialisation) or maxit products are done.  Every workgroup reads the
// same state; only workgroup 0 records the decision.
__device__ bool iter_gate(DevState *st)
{
    // all fields read before the first decision, and the common case taken
    // on one test of all of them (one memory round trip)
    const int status = st->status, k = st->k, maxit = st->maxit, conv = st->conv_next;
    const double rho = st->rho_next;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if ((status == kRun) & (conv == 0) & (k < maxit)) {
        if (lead)
            st->rho = rho;
        return true;
    }
    if (status != kRun)
        return false;
    // converged (checked first) or out of iterations
    if (lead) {
        st->rho = rho;
        st->iters = k;
        st->status = conv ? kConverged : kMaxit;
    }
    return false;
}

// Two kernels per iteration (IterCtx::fused): what the product needs besides
// its matrix -- the previous direction, the residual, the vectors it writes,
// and the r update's partials of r'r.
struct FusedDir {
    const double *pold = nullptr, *r = nullptr;
    double *pnew = nullptr, *x = nullptr;
    const double *rho_part = nullptr;
    int n_rho = 0;
};

struct FusedStep {
    bool xupd;    // this iteration's x += alpha p_prev is still to be applied
    bool run;     // and the iteration goes on (product, new direction)
    double alpha; // alpha of the previous iteration (0 before the first)
    double beta;  // rho_k / rho_(k-1)
};

// Start of iteration k in the fused form: r'r of the current residual from
// the r update's partials (fixed order: the bits the x/p update computes),
// the unfused gate's decision (converged first, then maxit), and beta.
// Workgroup 0 publishes r'r and the decision; the r update that follows
// records a stop (no workgroup of this kernel reads those fields, and no
// status changes here, so every workgroup applies the x update it owes).
// TB: threads of the calling kernel's workgroup (red: TB / 64 entries); the
// first kBlock threads hold the partials as the x/p update's threads do, the
// others add +0.0, so the sum has the x/p update's bits.
template <int TB>
__device__ FusedStep fused_gate(DevState *st, const FusedDir &fd, double *red)
{
    const int status = st->status, k = st->k, maxit = st->maxit;
    const double rho_prev = st->rho, alpha = st->alpha, tol_nb = st->tol_nb;
    double sv = 0.0;
    if (threadIdx.x < kBlock) {
        double pv[kPartPerThread];
        partials_load(fd.rho_part, fd.n_rho, pv);
#pragma unroll
        for (int j = 0; j < kPartPerThread; ++j)
            if ((int)threadIdx.x + j * kBlock < fd.n_rho)
                sv += pv[j];
    }
    const double rho = block_sum_n<TB>(sv, red);
    FusedStep f{status == kRun, false, alpha, 0.0};
    if (!f.xupd)
        return f;
    const int stop = sqrt(rho) <= tol_nb ? 1 : (k >= maxit ? 2 : 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho_next = rho;
        st->conv_next = stop;
    }
    f.run = stop == 0;
    f.beta = f.run ? rho / rho_prev : 0.0;
    return f;
}

// p_k[c] = r[c] + beta p_(k-1)[c] for a gathered column (0 for padding):
// the fused product's x operand, bit-identical to what the x/p update
// stores.
__device__ __forceinline__ double fused_dir(const FusedDir &fd, double beta, int c)
{
    // two guarded loads with nothing else in their branch (so neither waits
    // there, and a wave with no column skips both), then the update outside:
    // fma(beta, 0, 0) = 0 for padding
    const double po = c >= 0 ? fd.pold[c] : 0.0;
    const double rr = c >= 0 ? fd.r[c] : 0.0;
    return fma(beta, po, rr);
}

// ------------------------------------------------------------------ CSR
// W lanes per row (4..64), U rows per lane group in flight, rows of the
// workgroup's contiguous range visited in passes of (256 / W) * U rows.
// Index / value streams use non-temporal loads (read once); x is gathered
// through the cache.  Fused epilogue: partial of x'y.
// VT / PT: storage type of the values / of the input vector (double, or float
// for the FP32 product of mixed-precision refinement); arithmetic is FP64.
template <int W, int U, class VT, class PT>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int n, int rows_per_block, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col,
                                                     const VT *__restrict__ val,
                                                     const PT *__restrict__ x, double *__restrict__ y,
                                                     double *__restrict__ sig_part, DevState *st)
{
    __shared__ double red[kWaves];
    if (st != nullptr && !iter_gate(st))
        return;
    constexpr int NG = kBlock / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int r0 = blk * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    const int g = threadIdx.x / W, lane = threadIdx.x % W;
    double sig = 0.0;
    for (int base = r0 + g; base < r1; base += NG * U) {
        int rs[U], re[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = base + u * NG;
            const bool ok = r < r1;
            rs[u] = ok ? __builtin_nontemporal_load(ptr + r) : 0;
            re[u] = ok ? __builtin_nontemporal_load(ptr + r + 1) : 0;
        }
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            acc[u] = 0.0;
        for (int off = lane;; off += W) {
            bool any = false;
            int c[U];
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = rs[u] + off;
                const bool ok = k < re[u];
                any |= ok;
                c[u] = ok ? __builtin_nontemporal_load(col + k) : -1;
                v[u] = ok ? (double)__builtin_nontemporal_load(val + k) : 0.0;
            }
            if (!any)
                break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xv = (double)gather0(x, c[u]);
                acc[u] = fma(v[u], xv, acc[u]);
            }
        }
        double yv = 0.0;
        int row = r1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double t = group_sum<W>(acc[u]);
            if (lane == u) {
                yv = t;
                row = base + u * NG;
            }
        }
        if (lane < U && row < r1) {
            y[row] = yv;
            sig = fma((double)x[row], yv, sig);
        }
    }
    sig = block_sum(sig, red);
    if (threadIdx.x == 0)
        sig_part[blk] = sig;
}

// ------------------------------------------------- CSR row blocks
// Short rows (the FEM case): a workgroup takes a contiguous range of row
// blocks (<= 256 rows, <= 2048 entries each).  The boundaries {first row,
// first entry} of every block are precomputed (uniform: scalar loads, no
// dependent read of the row pointers).  For each block every thread first
// issues its 8 index / value loads (fully coalesced, non-temporal) and its
// row's local pointer, then the 8 gathers of x, parks the products in LDS,
// and after one barrier each row is summed left to right by one thread -- the
// same order as the textbook loop, so y is bit-identical to a serial
// row-by-row product.  A row longer than a block is summed by the whole
// workgroup (fixed tree).  (Prefetching the next block into registers was
// measured slower: the extra registers cut the resident workgroups by more
// than the latency it hides.)
template <class VT, class PT>
__global__ __launch_bounds__(kBlock) void k_spmv_csr_rows(int nrb, const int2 *__restrict__ rbe,
                                                          const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ col,
                                                          const VT *__restrict__ val,
                                                          const PT *__restrict__ x, double *__restrict__ y,
                                                          double *__restrict__ sig_part, DevState *st)
{
    constexpr int E = kStreamPerThread;
    __shared__ double prod[kStreamEntries];
    __shared__ int32_t lptr[kStreamRows + 1];
    __shared__ double red[kWaves];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    if (st != nullptr && !iter_gate(st))
        return;
    const int b0 = (int)((int64_t)wg * nrb / gridDim.x);
    const int b1 = (int)((int64_t)(wg + 1) * nrb / gridDim.x);
    const int t = threadIdx.x;
    double sig = 0.0;
    for (int b = b0; b < b1; ++b) {
        const int2 lo = rbe[b], hi = rbe[b + 1];
        const int r0 = lo.x, nr = hi.x - lo.x;
        const int e0 = lo.y, e1 = hi.y;
        if (e1 - e0 > kStreamEntries) { // one long row
            double a = 0.0;
            for (int e = e0 + t; e < e1; e += kBlock)
                a = fma((double)__builtin_nontemporal_load(val + e), (double)x[__builtin_nontemporal_load(col + e)],
                        a);
            a = block_sum(a, red);
            if (t == 0) {
                y[r0] = a;
                sig = fma((double)x[r0], a, sig);
            }
            continue;
        }
        int c[E];
        double v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = e0 + t + m * kBlock;
            const bool ok = e < e1;
            c[m] = ok ? __builtin_nontemporal_load(col + e) : -1;
            v[m] = ok ? (double)__builtin_nontemporal_load(val + e) : 0.0;
        }
        if (t < nr)
            lptr[t + 1] = __builtin_nontemporal_load(ptr + r0 + t + 1) - e0;
        if (t == 0)
            lptr[0] = 0;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (c[m] >= 0)
                prod[t + m * kBlock] = v[m] * (double)x[c[m]];
        __syncthreads();
        if (t < nr) {
            double a = 0.0;
            const int k1 = lptr[t + 1];
            for (int k = lptr[t]; k < k1; ++k)
                a += prod[k];
            y[r0 + t] = a;
            sig = fma((double)x[r0 + t], a, sig);
        }
        __syncthreads();
    }
    sig = block_sum(sig, red);
    if (t == 0)
        sig_part[wg] = sig;
}

// ------------------------------------------------- slices
// Sliced layout (plan.h): one wavefront per slice of 64 lines, lane l owns
// line 64 s + l and walks its entries left to right, U positions per round
// (all index / value loads of a round first -- coalesced, non-temporal --
// then the U gathers of x, then the sums).  For a stencil-like matrix the
// k-th entries of neighbouring lines are neighbouring columns, so each gather
// touches a few cache lines instead of one per lane.  Each line is summed as
// a + v x with the product rounded before the add (no fused multiply-add), as
// the row-block kernels' LDS products are: a CSR row is bit-identical to the
// serial row-by-row loop.  With more slices than 4 x kMaxSliceWgs each wave
// takes several consecutive slices of its workgroup's range.
// PANEL = false: lines are the rows of y.  PANEL = true: lines are the CSC
// panel slots; a colour-0 slot stores y[target], a colour-1 slot parks its
// sum at part[target] for the row pass.  Fused epilogue: partial of x'y (linear in the line
// sums, so x_target * sum per line).
// FUSED (CSR, FP64): the two-kernel iteration (FusedDir): x is unused, the
// gathered operand is p_k formed from fd.pold and fd.r, and each line's row
// gets its new direction and x update.
template <bool PANEL, int S, bool NT, class VT, class PT, class CT, bool FUSED = false>
__global__ __launch_bounds__(kBlock) void k_spmv_slices(int nl, int ns, const int32_t *__restrict__ off,
                                                        const CT *__restrict__ col, const VT *__restrict__ val,
                                                        const PT *__restrict__ x, double *__restrict__ y,
                                                        const int32_t *__restrict__ target, double *__restrict__ part,
                                                        int first_parked, double *__restrict__ sig_part, DevState *st,
                                                        FusedDir fd = FusedDir{})
{
#pragma clang fp contract(off)
    static_assert(!FUSED || (!PANEL && sizeof(PT) == 8), "the fused form is for FP64 CSR rows");
    // positions per round (values and gathered x stay in their stored type
    // until the multiply); 16 in the two-kernel form of small systems, whose
    // rows then take one round instead of two (latency, not bytes, bounds it)
    constexpr int U = FUSED ? 16 : 8;
    __shared__ double red[kWaves];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int s0 = (int)((int64_t)wg * ns / gridDim.x);
    const int s1 = (int)((int64_t)(wg + 1) * ns / gridDim.x);
    FusedStep f{true, true, 0.0, 0.0};
    if constexpr (FUSED) {
        f = fused_gate<kBlock>(st, fd, red);
        if (!f.run) {
            // stopping: the x update this iteration owes, on this workgroup's rows
            if (f.xupd)
                for (int i = s0 * kSliceRows + (int)threadIdx.x; i < min(s1 * kSliceRows, nl); i += kBlock)
                    fd.x[i] = fma(f.alpha, fd.pold[i], fd.x[i]);
            return;
        }
    } else if (st != nullptr && !iter_gate(st)) {
        return;
    }
    const int lane = threadIdx.x & 63;
    double sig = 0.0;
    // S slices per wave at a time (sl, sl + kWaves, ...): their loads are
    // issued together, so a wave with several slices keeps S chains in flight
    for (int sl = s0 + (int)(threadIdx.x >> 6); sl < s1; sl += S * kWaves) {
        int e0[S], len[S], l[S], tg[S];
        double a[S];
        int lmax = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int q = sl + j * kWaves;
            const bool has = q < s1;
            e0[j] = has ? off[q] : 0;
            len[j] = has ? (off[q + 1] - e0[j]) / kSliceRows : 0;
            l[j] = has ? q * kSliceRows + lane : nl;
            tg[j] = l[j];
            if (PANEL)
                tg[j] = l[j] < nl ? matrix_load<NT>(target + l[j]) : -1;
            a[j] = 0.0;
            lmax = max(lmax, len[j]);
        }
        for (int k0 = 0; k0 < lmax; k0 += U) {
            int c[S][U];
            VT v[S][U];
            PT xv[S][U];
            // One 2-wide load per entry pair, unconditional: entries k, k + 1
            // side by side; the single last entry of an odd-width slice
            // through the aligned pair holding it (the lane's parity picks
            // the half); past the width, positions 0 and 1 (discarded).  No
            // load sits in a branch, where it would wait for the loads before
            // it; the entries are then selected.
            typename Vec2<CT>::type craw[S][U / 2];
            typename Vec2<VT>::type vraw[S][U / 2];
#pragma unroll
            for (int j = 0; j < S; ++j)
#pragma unroll
                for (int u = 0; u < U; u += 2) {
                    const int k = k0 + u;
                    const int e = k + 1 < len[j] ? e0[j] + (k >> 1) * (2 * kSliceRows) + 2 * lane
                                  : k < len[j]   ? e0[j] + k * kSliceRows + (lane & ~1)
                                                 : 0;
                    craw[j][u >> 1] = matrix_load<NT>(reinterpret_cast<const typename Vec2<CT>::type *>(col + e));
                    vraw[j][u >> 1] = matrix_load<NT>(reinterpret_cast<const typename Vec2<VT>::type *>(val + e));
                }
#pragma unroll
            for (int j = 0; j < S; ++j)
#pragma unroll
                for (int u = 0; u < U; u += 2) {
                    const int k = k0 + u;
                    const bool pair = k + 1 < len[j], hi = !pair && (lane & 1);
                    const int row = PANEL ? tg[j] : l[j]; // the row the line adds to
                    c[j][u] = k < len[j] ? col_of(hi ? craw[j][u >> 1].y : craw[j][u >> 1].x, row) : -1;
                    c[j][u + 1] = pair ? col_of(craw[j][u >> 1].y, row) : -1;
                    v[j][u] = hi ? vraw[j][u >> 1].y : vraw[j][u >> 1].x;
                    v[j][u + 1] = vraw[j][u >> 1].y;
                }
#pragma unroll
            for (int j = 0; j < S; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if constexpr (FUSED)
                        xv[j][u] = fused_dir(fd, f.beta, c[j][u]);
                    else
                        xv[j][u] = gather0(x, c[j][u]);
                }
#pragma unroll
            for (int j = 0; j < S; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (c[j][u] >= 0)
                        a[j] = a[j] + (double)v[j][u] * (double)xv[j][u];
        }
#pragma unroll
        for (int j = 0; j < S; ++j)
            if (l[j] < nl) {
                if (!PANEL || l[j] < first_parked)
                    y[tg[j]] = a[j];
                else
                    part[tg[j]] = a[j]; // parked by row: at most one colour-1 slot per row
                if constexpr (FUSED) {
                    // the row's new direction and the x update it owes
                    const double po = fd.pold[l[j]];
                    const double pk = fma(f.beta, po, fd.r[l[j]]);
                    fd.pnew[l[j]] = pk;
                    fd.x[l[j]] = fma(f.alpha, po, fd.x[l[j]]);
                    sig = fma(pk, a[j], sig);
                } else {
                    sig = fma((double)x[tg[j]], a[j], sig);
                }
            }
    }
    sig = block_sum(sig, red);
    if (threadIdx.x == 0)
        sig_part[wg] = sig;
}

// ------------------------------------------------- CSC column panels
// One launch over every chunk of every panel (chunks of colour 0 first; a
// workgroup walks a contiguous range of chunks).  A chunk is a run of write
// slots -- (panel, row) pairs, each a contiguous segment of entries in column
// order -- so it is processed like a CSR row block: coalesced index / value
// loads, the gathers of x, products parked in LDS, one thread per slot sums
// its segment left to right.  Colour-0 slots store y; colour-1 slots park the
// sum for k_scatter_gather.  x'y is linear in the slot sums, so each
// workgroup accumulates sum_slots x_row * sum.  A slot longer than a chunk
// is summed by the whole workgroup (fixed tree).
template <class VT, class PT>
__global__ __launch_bounds__(kBlock) void k_panel_rows(int nch, const int32_t *__restrict__ chunk_slot,
                                                       const int32_t *__restrict__ slot_ptr,
                                                       const int32_t *__restrict__ slot_target,
                                                       const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                       const PT *__restrict__ x, double *__restrict__ y,
                                                       double *__restrict__ part, int first_parked,
                                                       double *__restrict__ sig_part, DevState *st)
{
    constexpr int E = kStreamPerThread;
    __shared__ double prod[kStreamEntries];
    __shared__ int32_t lptr[kStreamRows + 1];
    __shared__ double red[kWaves];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    if (st != nullptr && !iter_gate(st))
        return;
    const int c0 = (int)((int64_t)wg * nch / gridDim.x);
    const int c1 = (int)((int64_t)(wg + 1) * nch / gridDim.x);
    const int t = threadIdx.x;
    double sig = 0.0;
    for (int c = c0; c < c1; ++c) {
        const int s0 = chunk_slot[c], ns = chunk_slot[c + 1] - s0;
        const int e0 = slot_ptr[s0], e1 = slot_ptr[s0 + ns];
        if (e1 - e0 > kStreamEntries) { // one long slot
            double a = 0.0;
            for (int e = e0 + t; e < e1; e += kBlock)
                a = fma((double)__builtin_nontemporal_load(val + e), (double)x[__builtin_nontemporal_load(col + e)],
                        a);
            a = block_sum(a, red);
            if (t == 0) {
                const int tg = slot_target[s0];
                if (s0 < first_parked)
                    y[tg] = a;
                else
                    part[tg] = a; // parked by row: at most one colour-1 slot per row
                sig = fma((double)x[tg], a, sig);
            }
            continue;
        }
        int cc[E];
        double v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = e0 + t + m * kBlock;
            const bool ok = e < e1;
            cc[m] = ok ? __builtin_nontemporal_load(col + e) : -1;
            v[m] = ok ? (double)__builtin_nontemporal_load(val + e) : 0.0;
        }
        int tg = -1;
        if (t < ns) {
            lptr[t + 1] = __builtin_nontemporal_load(slot_ptr + s0 + t + 1) - e0;
            tg = __builtin_nontemporal_load(slot_target + s0 + t);
        }
        if (t == 0)
            lptr[0] = 0;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (cc[m] >= 0)
                prod[t + m * kBlock] = v[m] * (double)x[cc[m]];
        const double xt = (double)gather0(x, tg);
        __syncthreads();
        if (t < ns) {
            double a = 0.0;
            const int k1 = lptr[t + 1];
            for (int k = lptr[t]; k < k1; ++k)
                a += prod[k];
            const int sl = s0 + t;
            if (sl < first_parked)
                y[tg] = a;
            else
                part[tg] = a;
            sig = fma(xt, a, sig);
        }
        __syncthreads();
    }
    sig = block_sum(sig, red);
    if (t == 0)
        sig_part[wg] = sig;
}

// dst[k] = src[perm[k]] (0 where perm[k] < 0): values into the panel order
// or the slice positions
template <class T>
__global__ __launch_bounds__(kBlock) void k_permute(int64_t nnz, const T *__restrict__ src,
                                                    const int32_t *__restrict__ perm, T *__restrict__ dst)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nnz) {
        const int32_t j = perm[k];
        dst[k] = j >= 0 ? src[j] : T(0);
    }
}

// ------------------------------------------------- coloured scatter
// Product of the symmetric format, whose stored entries also write the rows
// named by their index (the mirrored triangle).  Two kernels:
//
// k_scatter_sums -- all blocks of all colours at once (blocks stored in
//   colour order, each workgroup walks a contiguous range).  Per block every
//   independent global load is issued first (line pointers, x of the own
//   lines, the contribution list -> LDS, the index / value pairs, E per
//   thread, and the write-slot descriptors, SU per thread); then the gathers;
//   then, through one LDS product buffer: the products of the stored rows
//   themselves, a_e x_idx(e), each own row summed left to right by the thread
//   that owns that row's slot; then the mirror products a_e x_line(e), and
//   every slot's sum in the plan's fixed order.  Every value is read once and
//   used twice.  Colour-0 blocks are the first writers of all their rows and
//   store y directly; the others park their slot sums in `part`.  The dot x'y
//   is linear in the slot sums, so each workgroup accumulates
//   sum_slots x_target * sum here, before any y is final.
// k_scatter_gather -- one launch: every row adds its parked slot sums, in
//   ascending colour order, to what its colour-0 writer stored (if any).
//   Blocks of one colour write disjoint rows, so colour 0 can store without
//   conflicts; the colour order fixes the accumulation order of the rest.
//   (Inside CG iterations this pass is folded into the r update.)
template <int SU, int E, class VT, class PT>
__global__ __launch_bounds__(kBlock) void k_scatter_sums(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const VT *__restrict__ val,
    const PT *__restrict__ x, double *__restrict__ y, double *__restrict__ part, double *__restrict__ sig_part,
    const ScatterBlock *__restrict__ blocks, int nblocks, const int32_t *__restrict__ slot_target,
    const uint16_t *__restrict__ seg, const uint16_t *__restrict__ tl, int lds_entries, int lds_lines, DevState *st)
{
    // E entries per thread: E * kBlock >= the largest block
    extern __shared__ double lds[];
    __shared__ double red[kWaves];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    if (st != nullptr && !iter_gate(st))
        return;
    double *sp = lds; // own-row products first, then the mirror products
    double *xl = sp + lds_entries;
    int32_t *lp = reinterpret_cast<int32_t *>(xl + lds_lines);
    uint16_t *lm = reinterpret_cast<uint16_t *>(lp + lds_lines + 1);
    uint16_t *tv = lm + lds_entries;
    const int t = threadIdx.x;
    const int b0 = (int)((int64_t)wg * nblocks / gridDim.x);
    const int b1 = (int)((int64_t)(wg + 1) * nblocks / gridDim.x);
    double sig = 0.0;
    for (int b = b0; b < b1; ++b) {
        const ScatterBlock bk = blocks[b];
        const int nl = bk.line1 - bk.line0, ne = bk.k1 - bk.k0;
        // ---- independent loads
        for (int l = t; l <= nl; l += kBlock)
            lp[l] = min(max(ptr[bk.line0 + l] - bk.k0, 0), ne);
        for (int l = t; l < nl; l += kBlock)
            xl[l] = (double)x[bk.line0 + l];
        for (int i = t; i < bk.ntl; i += kBlock)
            tv[i] = tl[bk.tl0 + i];
        int c[E];
        double v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = t + m * kBlock;
            const bool ok = e < ne;
            c[m] = ok ? __builtin_nontemporal_load(idx + bk.k0 + e) : -1;
            v[m] = ok ? (double)__builtin_nontemporal_load(val + bk.k0 + e) : 0.0;
        }
        int tg[SU], lo[SU], hi[SU];
        const uint16_t *sg = seg + bk.slot0 + bk.id;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int s = t + u * kBlock;
            const bool ok = s < bk.nslots;
            tg[u] = ok ? slot_target[bk.slot0 + s] : -1;
            lo[u] = ok ? sg[s] : 0;
            hi[u] = ok ? sg[s + 1] : 0;
        }
        // ---- gathers
        double xg[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            xg[m] = (double)gather0(x, c[m]);
        double xt[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u)
            xt[u] = (double)gather0(x, tg[u]);
        __syncthreads();
        // ---- line of every entry
        for (int l = t; l < nl; l += kBlock)
            for (int k = lp[l]; k < lp[l + 1]; ++k)
                lm[k] = (uint16_t)l;
        // ---- own rows, stored entries left to right; the sum of row l stays
        //      in thread l, which owns that row's slot (l < 256)
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (c[m] >= 0)
                sp[t + m * kBlock] = v[m] * xg[m];
        __syncthreads();
        double own = 0.0;
        if (t < nl)
            for (int k = lp[t]; k < lp[t + 1]; ++k)
                own += sp[k];
        __syncthreads();
        // ---- mirror products (the diagonal has none)
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = t + m * kBlock;
            if (c[m] >= 0) {
                const int l = lm[e];
                if (c[m] != bk.line0 + l)
                    sp[e] = v[m] * xl[l];
            }
        }
        __syncthreads();
        // ---- slot sums
        const bool first_colour = bk.pad == 0;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            if (tg[u] < 0)
                continue;
            const int s = t + u * kBlock;
            double a = s < nl ? own : 0.0; // s < nl <= 256 implies u == 0 and s == t
            for (int i = lo[u]; i < hi[u]; ++i)
                a += sp[tv[i]];
            if (first_colour)
                y[tg[u]] = a;
            else
                part[bk.slot0 + s] = a;
            sig = fma(xt[u], a, sig);
        }
        __syncthreads(); // LDS is reused by the next block
    }
    sig = block_sum(sig, red);
    if (t == 0)
        sig_part[wg] = sig;
}

// Sliced blocks of the symmetric format: the same blocks, slots, colours and
// contribution lists as k_scatter_sums, with each block's entries stored
// k-th-entry-major (position k * nl + l for line l), so thread l loads line
// l's entries itself (coalesced over l, and so are the gathers of x for a
// stencil-like matrix), sums its own row in registers left to right from
// rounded products (the same bits as the LDS sum), and parks only the mirror
// products a_e x_l in LDS, where the slot sums read them through the
// contribution list (local positions).  Two barriers per block, no line map.
template <int SU, bool NT, class VT, class PT>
__global__ __launch_bounds__(kBlock) void k_scatter_slices(
    const int32_t *__restrict__ sidx, const VT *__restrict__ sval, const int2 *__restrict__ sblk,
    const PT *__restrict__ x, double *__restrict__ y, double *__restrict__ part, double *__restrict__ sig_part,
    const ScatterBlock *__restrict__ blocks, int nblocks, const int32_t *__restrict__ slot_target,
    const uint16_t *__restrict__ seg, const uint16_t *__restrict__ tl, DevState *st)
{
#pragma clang fp contract(off)
    constexpr int E = kStreamPerThread;
    __shared__ double sp[kMaxScatterEntries];
    __shared__ uint16_t tv[kMaxScatterEntries];
    __shared__ double red[kWaves];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    if (st != nullptr && !iter_gate(st))
        return;
    const int t = threadIdx.x;
    const int b0 = (int)((int64_t)wg * nblocks / gridDim.x);
    const int b1 = (int)((int64_t)(wg + 1) * nblocks / gridDim.x);
    double sig = 0.0;
    for (int b = b0; b < b1; ++b) {
        const ScatterBlock bk = blocks[b];
        const int2 sb = sblk[b];
        const int nl = bk.line1 - bk.line0, L = sb.y;
        const bool mine = t < nl;
        // ---- independent loads
        for (int i = t; i < bk.ntl; i += kBlock)
            tv[i] = tl[bk.tl0 + i];
        int c[E];
        double v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const bool ok = mine && m < L;
            const int q = sb.x + m * nl + t;
            c[m] = ok ? matrix_load<NT>(sidx + q) : -1;
            v[m] = ok ? (double)matrix_load<NT>(sval + q) : 0.0;
        }
        const double xo = (double)gather0(x, mine ? bk.line0 + t : -1);
        // ---- gathers
        double xg[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            xg[m] = (double)gather0(x, c[m]);
        // ---- own row in registers; mirror products (not the diagonal) to LDS
        double own = 0.0;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (c[m] >= 0) {
                own = own + v[m] * xg[m];
                if (c[m] != bk.line0 + t)
                    sp[m * nl + t] = v[m] * xo;
            }
        __syncthreads();
        // ---- slot descriptors, loaded only now: held across the first phase
        //      they cost 22 VGPRs (91 instead of 69, 5 instead of 7 waves per
        //      SIMD), more than their latency here (45.5 instead of 47.5 us)
        int tg[SU], lo[SU], hi[SU];
        const uint16_t *sg = seg + bk.slot0 + bk.id;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int s = t + u * kBlock;
            const bool ok = s < bk.nslots;
            tg[u] = ok ? slot_target[bk.slot0 + s] : -1;
            lo[u] = ok ? sg[s] : 0;
            hi[u] = ok ? sg[s + 1] : 0;
        }
        double xt[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u)
            xt[u] = (double)gather0(x, tg[u]);
        // ---- slot sums
        const bool first_colour = bk.pad == 0;
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            if (tg[u] < 0)
                continue;
            const int s = t + u * kBlock;
            double a = s < nl ? own : 0.0; // s < nl <= 256 implies u == 0 and s == t
            for (int i = lo[u]; i < hi[u]; ++i)
                a += sp[tv[i]];
            if (first_colour)
                y[tg[u]] = a;
            else
                part[bk.slot0 + s] = a;
            sig = fma(xt[u], a, sig);
        }
        __syncthreads(); // LDS is reused by the next block
    }
    sig = block_sum(sig, red);
    if (t == 0)
        sig_part[wg] = sig;
}

// Compact blocks of the symmetric format (plan.h): thread t holds own line
// t of the block (row line0 + t of the block order), loads that
// line's entries (two per load, coalesced over t) and the LDS places of
// their mirror products (one 16-byte load), sums the stored row in registers
// left to right from rounded products, and puts each mirror product a_e x_t
// at its place -- the products are grouped there by the slot they add to.
// The block's slot starts are staged in LDS (16 bytes per thread).  After
// one barrier each slot sums its contiguous run of products in the plan's
// order: own-line slots add it to their row's sum and store y (the block
// owns those rows; nobody else stores them), the other slots park their sum
// at its place in the by-row array of the row pass.  Fused epilogue: x'y as
// sum_slots x_target * sum.
// FUSED (FP64): the two-kernel iteration (FusedDir), as in k_spmv_slices:
// every x operand is p_k formed from fd.pold and fd.r, and each own line's
// row gets its new direction and x update.
template <int SU, bool NT, class VT, class PT, bool FUSED = false>
__global__ __launch_bounds__(kCompactThreads) void k_scatter_compact(
    const int32_t *__restrict__ sidx, const VT *__restrict__ sval, const CompactBlock *__restrict__ blocks,
    int nblocks, const int32_t *__restrict__ slot_target, const uint16_t *__restrict__ seg,
    const uint16_t *__restrict__ rank, const int32_t *__restrict__ dest, const PT *__restrict__ x,
    double *__restrict__ y, double *__restrict__ part, double *__restrict__ sig_part, DevState *st,
    FusedDir fd = FusedDir{})
{
#pragma clang fp contract(off)
    constexpr int E = kStreamPerThread;
    constexpr int TB = kCompactThreads;
    // slot starts: staged through LDS (16 bytes per thread) for a streamed
    // matrix; for a cache-resident one each thread reads its slots' starts
    // itself, which frees 9 KB of LDS for a 4th workgroup per CU (a latency-
    // bound product gains from it, a bandwidth-bound one does not)
    constexpr int kStarts = NT ? ((TB + kCompactEntries + 1) + 7) / 8 * 8 : 8;
    __shared__ double sp[kCompactEntries];
    __shared__ __align__(16) uint16_t st16[kStarts];
    __shared__ double red[TB / 64];
    static_assert(!FUSED || sizeof(PT) == 8, "the fused form is FP64");
    FusedStep f{true, true, 0.0, 0.0};
    if constexpr (FUSED) {
        f = fused_gate<TB>(st, fd, red);
    } else if (st != nullptr && !iter_gate(st)) {
        return;
    }
    const int t = threadIdx.x;
    // blocks of this XCD: one contiguous eighth; its workgroups take them in
    // turn (workgroup i of the XCD: blocks i, i + G, i + 2G, ...), so the
    // blocks in flight on an XCD at any time are neighbours, whose x and y
    // lines meet in that XCD's L2
    const int nx = min(kXcds, (int)gridDim.x);
    const int xcd = blockIdx.x % nx, wi = blockIdx.x / nx;
    const int gx = ((int)gridDim.x - xcd + nx - 1) / nx;
    const int b1 = (int)((int64_t)(xcd + 1) * nblocks / nx);
    const int bfirst = (int)((int64_t)xcd * nblocks / nx) + wi;
    if constexpr (FUSED) {
        if (!f.run) {
            // stopping: the x update this iteration owes, on this workgroup's lines
            if (f.xupd)
                for (int b = bfirst; b < b1; b += gx) {
                    const CompactBlock bk = blocks[b];
                    if (t < bk.nl)
                        fd.x[bk.line0 + t] = fma(f.alpha, fd.pold[bk.line0 + t], fd.x[bk.line0 + t]);
                }
            return;
        }
    }
    double sig = 0.0;
    for (int b = bfirst; b < b1; b += gx) {
        const CompactBlock bk = blocks[b];
        const int nl = bk.nl, L = bk.len;
        const bool mine = t < nl;
        // ---- independent loads, all issued before the first wait (loads
        //      complete in issue order): slot starts, LDS places, entries,
        //      and the targets and rows of the parked slots.  None sits in a
        //      divergent branch, where it would wait before the next one is
        //      issued: indices are clamped into the block and the values
        //      selected afterwards; branches on the block's sizes are uniform.
        const int nchunk = (bk.nslots + 8) / 8; // 16-byte chunks of the nslots + 1 slot starts
        uint4v sg0 = {0u, 0u, 0u, 0u}, sg1 = {0u, 0u, 0u, 0u};
        int s0[SU], s1[SU]; // cache-resident: the run [seg[s], seg[s + 1]) of each of the thread's slots
        if constexpr (NT) {
            const uint4v *segv = reinterpret_cast<const uint4v *>(seg + bk.seg0);
            sg0 = matrix_load<NT>(segv + min(t, nchunk - 1));
            if (nchunk > TB)
                sg1 = matrix_load<NT>(segv + min(t + TB, nchunk - 1));
        } else {
#pragma unroll
            for (int u = 0; u < SU; ++u) { // index clamped to the block's nslots + 1 starts, unused past them
                const int s = t + u * TB;
                s0[u] = seg[bk.seg0 + min(s, bk.nslots)];
                s1[u] = seg[bk.seg0 + min(s + 1, bk.nslots)];
            }
        }
        const int tl = mine ? t : 0;
        const int line = mine ? bk.line0 + t : -1; // rows renumbered in block order
        const uint4v rk = matrix_load<NT>(reinterpret_cast<const uint4v *>(rank) + (bk.line0 + tl));
        // entries m, m + 1 side by side (one 8- / 16-byte load), or the
        // single last entry of an odd width through the aligned pair holding
        // it (the thread's parity picks the half), or, past the width, the
        // block's first pair (discarded)
        int2v craw[E / 2];
        typename Vec2<VT>::type vraw[E / 2];
#pragma unroll
        for (int h = 0; h < E / 2; ++h) {
            const int m = 2 * h;
            const int q = m + 1 < L ? bk.pos0 + m * nl + 2 * tl : m < L ? bk.pos0 + m * nl + (tl & ~1) : bk.pos0;
            craw[h] = matrix_load<NT>(reinterpret_cast<const int2v *>(sidx + q));
            vraw[h] = matrix_load<NT>(reinterpret_cast<const typename Vec2<VT>::type *>(sval + q));
        }
        int c[E];
        double v[E];
#pragma unroll
        for (int h = 0; h < E / 2; ++h) {
            const int m = 2 * h;
            const bool hi = m + 1 >= L && (tl & 1);
            c[m] = mine && m < L ? (hi ? craw[h].y : craw[h].x) : -1;
            c[m + 1] = mine && m + 1 < L ? craw[h].y : -1;
            v[m] = (double)(hi ? vraw[h].y : vraw[h].x);
            v[m + 1] = (double)vraw[h].y;
        }
        int tg[SU], pk[SU];
        const int npk = bk.nslots - nl; // parked slots of the block
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int s = t + u * TB;
            const bool parked = s >= nl && s < bk.nslots;
            const int ts = matrix_load<NT>(slot_target + bk.slot0 + min(max(s, nl), bk.nslots - 1));
            tg[u] = s < nl ? line : parked ? ts : -1;
            // (dest holds one element past its last parked slot)
            const int ps = matrix_load<NT>(dest + bk.park0 + min(max(s - nl, 0), max(npk - 1, 0)));
            pk[u] = parked ? ps : -1;
        }
        // ---- gathers (fused: p_k formed from the previous direction and r)
        double xo, xg[E], xt[SU];
        if constexpr (FUSED) {
            xo = fused_dir(fd, f.beta, mine ? line : -1);
#pragma unroll
            for (int m = 0; m < E; ++m)
                xg[m] = fused_dir(fd, f.beta, c[m]);
#pragma unroll
            for (int u = 0; u < SU; ++u)
                xt[u] = t + u * TB < nl ? xo : fused_dir(fd, f.beta, tg[u]);
            if (mine) { // the own line's new direction and the x update it owes
                fd.pnew[line] = xo;
                fd.x[line] = fma(f.alpha, fd.pold[line], fd.x[line]);
            }
        } else {
            xo = (double)gather0(x, mine ? line : -1);
#pragma unroll
            for (int m = 0; m < E; ++m)
                xg[m] = (double)gather0(x, c[m]);
#pragma unroll
            for (int u = 0; u < SU; ++u)
                xt[u] = t + u * TB < nl ? xo : (double)gather0(x, tg[u]);
        }
        // ---- slot starts to LDS (read after the barrier below)
        if constexpr (NT) {
            if (t < nchunk)
                *reinterpret_cast<uint4v *>(st16 + 8 * t) = sg0;
            if (nchunk > TB && t + TB < nchunk)
                *reinterpret_cast<uint4v *>(st16 + 8 * (t + TB)) = sg1;
        }
        // ---- own row in registers; mirror products (not the diagonal) to their places
        const uint32_t rw[4] = {rk.x, rk.y, rk.z, rk.w};
        double own = 0.0;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (c[m] >= 0) {
                own = own + v[m] * xg[m];
                const uint32_t place = (rw[m >> 1] >> (16 * (m & 1))) & 0xffffu;
                if (place != 0xffffu)
                    sp[place] = v[m] * xo;
            }
        __syncthreads();
        // ---- slot sums: own lines store y, the others park
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            if (tg[u] < 0)
                continue;
            const int s = t + u * TB;
            const bool own_slot = s < nl; // implies u == 0 and s == t
            double a = own_slot ? own : 0.0;
            const int lo = NT ? (int)st16[s] : s0[u], hi = NT ? (int)st16[s + 1] : s1[u];
            for (int i = lo; i < hi; ++i)
                a += sp[i];
            if (own_slot)
                y[tg[u]] = a;
            else
                part[pk[u]] = a; // by row: the row pass reads each row's sums contiguously
            sig = fma(xt[u], a, sig);
        }
        __syncthreads(); // LDS is reused by the next block
    }
    // workgroup sum of the x'y partial (fixed tree: waves, then in order)
    sig = group_sum<64>(sig);
    __syncthreads();
    if ((t & 63) == 0)
        red[t >> 6] = sig;
    __syncthreads();
    if (t == 0) {
        double a = red[0];
#pragma unroll
        for (int w = 1; w < TB / 64; ++w)
            a += red[w];
        sig_part[blockIdx.x] = a;
    }
}

// One thread per row: y_i = (y_i if a colour-0 block wrote it, else 0)
// + the row's parked slot sums in ascending colour order.  Every row is
// owned by one thread, so no atomics; the order is fixed by the plan.
__global__ __launch_bounds__(kBlock) void k_scatter_gather(int n, const int32_t *__restrict__ rs_ptr,
                                                           const int32_t *__restrict__ rs_idx,
                                                           const uint8_t *__restrict__ has_c0,
                                                           const double *__restrict__ part, double *__restrict__ y,
                                                           const DevState *st)
{
    if (st != nullptr && st->status != kRun)
        return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int k0 = rs_ptr[i], k1 = rs_ptr[i + 1];
    const bool c0 = has_c0 == nullptr || has_c0[i] != 0; // null: compact blocks, every row stored by its owner
    if (k0 == k1) {
        if (!c0)
            y[i] = 0.0; // no entry writes this row
        return;         // else written once, by its colour-0 block
    }
    double a = c0 ? y[i] : 0.0;
    for (int k = k0; k < k1; ++k)
        a += part[rs_idx != nullptr ? rs_idx[k] : k]; // null: parked sums stored by row
    y[i] = a;
}

// Row pass of the CSC panels: y_i = (colour-0 share) + (parked share), the
// same terms and order as k_scatter_gather, with the parked sum stored by
// row (flag bit 0: y_i holds a share, bit 1: part_i does; neither: no entry
// writes row i, y_i = 0).
__global__ __launch_bounds__(kBlock) void k_panel_gather(int n, const uint8_t *__restrict__ flags,
                                                         const double *__restrict__ part, double *__restrict__ y,
                                                         const DevState *st)
{
    if (st != nullptr && st->status != kRun)
        return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int f = flags[i];
    if (f == 1)
        return; // written once, by its colour-0 slot
    double a = (f & 1) ? y[i] : 0.0;
    if (f & 2)
        a += part[i];
    y[i] = a;
}

// ------------------------------------------------------ vector kernels
// Each workgroup owns a contiguous chunk (XCD-remapped).  The first KP
// elements per thread are loaded before the dot partials of the previous
// kernel are reduced, so the two memory round trips overlap.
constexpr int kPre = 8; // KP at most: a chunk of more than 8 x 256 elements takes the rest in a loop

// Rows finished by the row pass of a scatter product: GATHER folds that pass
// (k_scatter_gather's sum, same terms, same order) into the r update, so the
// product's last writes of y and their re-read are saved.
// GATHER: 0 = no row pass; 1 = per-row lists of parked slots (symmetric
// CSR, coloured plan); 2 = at most one parked sum per row, stored by row,
// with a flag byte (bit 0: y_i holds a share, bit 1: part_i does; CSC
// panels); 3 = parked sums stored by row at [rs_ptr[i], rs_ptr[i+1]), y_i
// always stored (symmetric CSR, compact blocks).
struct RowPass {
    const int32_t *rs_ptr = nullptr, *rs_idx = nullptr;
    const uint8_t *has_c0 = nullptr;
    const double *part = nullptr;
};

template <int GATHER>
__device__ __forceinline__ double q_value(const double *__restrict__ q, const RowPass &g, int i)
{
    if (GATHER == 0)
        return q[i];
    if (GATHER == 2) {
        const int f = g.has_c0[i];
        double a = (f & 1) ? q[i] : 0.0;
        if (f & 2)
            a += g.part[i];
        return a;
    }
    const int k0 = g.rs_ptr[i], k1 = g.rs_ptr[i + 1];
    if (GATHER == 3) {
        // parked sums stored by row: the first two loaded without a loop, so
        // the loads of several rows are in flight together (rarely more)
        double a = q[i];
        const double p0 = k0 < k1 ? g.part[k0] : 0.0;
        const double p1 = k0 + 1 < k1 ? g.part[k0 + 1] : 0.0;
        if (k0 < k1)
            a += p0;
        if (k0 + 1 < k1)
            a += p1;
        for (int k = k0 + 2; k < k1; ++k)
            a += g.part[k];
        return a;
    }
    double a = g.has_c0[i] ? q[i] : 0.0;
    for (int k = k0; k < k1; ++k)
        a += g.part[g.rs_idx[k]];
    return a;
}

// q (with the row pass of GATHER folded in: q_value's terms in q_value's
// order) and r of a thread's first KP rows (i0, i0 + kBlock, ...; rows from
// i1 on give 0).  The loads go out in dependency order -- row-pass indices or
// flags, then q and r, then the parked sums -- each group for every row before
// anything waits (loads complete in issue order); a parked sum is read
// unguarded (from element 0, or from q_i, when the row has none) and selected
// afterwards, so no load shares a branch with its add and waits there.
template <int GATHER, int KP>
__device__ __forceinline__ void row_values(const double *__restrict__ q, const double *__restrict__ r,
                                           const RowPass &g, int n, int i0, int i1, double (&qv)[KP],
                                           double (&rv)[KP])
{
    int k0[KP], k1[KP], fl[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int i = i0 + u * kBlock;
        const bool ok = i < i1;
        k0[u] = 0;
        k1[u] = 0;
        fl[u] = 0;
        if (GATHER == 3) { // unguarded (row clamped), then selected
            const int ic = min(i, n - 1);
            const int a = g.rs_ptr[ic], b = g.rs_ptr[ic + 1];
            k0[u] = ok ? a : 0;
            k1[u] = ok ? b : 0;
        }
        if (GATHER == 2)
            fl[u] = ok ? (int)g.has_c0[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int i = i0 + u * kBlock;
        const bool ok = i < i1;
        if (GATHER == 1)
            qv[u] = ok ? q_value<1>(q, g, i) : 0.0;
        else
            qv[u] = ok ? q[i] : 0.0;
        rv[u] = ok ? r[i] : 0.0;
    }
    if constexpr (GATHER == 2 || GATHER == 3) {
        double p0[KP], p1[KP];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            if (GATHER == 3) { // part holds at least one element
                p0[u] = g.part[k0[u] < k1[u] ? k0[u] : 0];
                p1[u] = g.part[k0[u] + 1 < k1[u] ? k0[u] + 1 : 0];
            } else {
                const int ic = min(i0 + u * kBlock, n - 1);
                p0[u] = *((fl[u] & 2) ? g.part + ic : q + ic);
                p1[u] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            double a = qv[u];
            if (GATHER == 2) {
                a = (fl[u] & 1) ? a : 0.0;
                a = (fl[u] & 2) ? a + p0[u] : a;
            } else {
                a = k0[u] < k1[u] ? a + p0[u] : a;
                a = k0[u] + 1 < k1[u] ? a + p1[u] : a;
                for (int k = k0[u] + 2; k < k1[u]; ++k) // rare: more than two parked sums
                    a += g.part[k];
            }
            qv[u] = a;
        }
    }
}

// PPT: dot partials per thread (n_sig <= PPT * 256).  FUSED: the r update
// of the two-kernel iteration: r'r of the current residual is the one the
// product published (rho_next), and a stop the product decided (conv_next)
// is recorded here.
// KP: elements per thread loaded up front (the chunk's, up to 8 x 256;
// registers sized to the chunk, so small chunks keep more waves resident).
template <int GATHER, int PPT, bool FUSED, int KP>
__global__ __launch_bounds__(kBlock) void k_update_r(int n, int chunk, double *__restrict__ r,
                                                     const double *__restrict__ q, DevState *st,
                                                     const double *__restrict__ sig_part, int n_sig,
                                                     double *__restrict__ rho_part, RowPass g)
{
    __shared__ double red[kWaves];
    // the gate, the partials and the first vector elements are loaded
    // together (one memory round trip); nothing is stored before the gate
    const int status = st->status;
    const int stop = FUSED ? st->conv_next : 0;
    const double rho = FUSED ? st->rho_next : st->rho;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    const int t = threadIdx.x;
    double pv[PPT];
    partials_load(sig_part, n_sig, pv);
    double qv[KP], rv[KP];
    row_values<GATHER, KP>(q, r, g, n, i0 + t, i1, qv, rv);
    if (status != kRun)
        return;
    const bool lead = blockIdx.x == 0 && t == 0;
    if (FUSED && stop != 0) {
        if (lead) {
            st->rho = rho;
            st->iters = st->k;
            st->status = stop == 1 ? kConverged : kMaxit;
        }
        return;
    }
    const double sigma = partials_sum(pv, n_sig, red);
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) {
            if (FUSED)
                st->rho = rho;
            st->iters = st->k;
            st->sigma = sigma;
            st->status = kBreakdown;
        }
        return;
    }
    const double alpha = rho / sigma;
    if (lead) {
        st->alpha = alpha;
        st->sigma = sigma;
        st->k = st->k + 1;
        if (FUSED)
            st->rho = rho; // r'r of the residual this step starts from (the next beta's denominator)
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int i = i0 + t + u * kBlock;
        if (i < i1) {
            const double ri = fma(-alpha, qv[u], rv[u]);
            r[i] = ri;
            acc = fma(ri, ri, acc);
        }
    }
    for (int i = i0 + t + KP * kBlock; i < i1; i += kBlock) {
        const double ri = fma(-alpha, q_value<GATHER>(q, g, i), r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, red);
    if (t == 0)
        rho_part[blk] = acc;
}

// x += alpha p and p = r + beta p; workgroup 0 publishes r'r and the
// convergence decision for the next iteration's gate (no workgroup of this
// kernel reads those two fields).
// PT: storage type of p (double; float for the inner solves of mixed
// precision, where p is rounded to FP32 after the FP64 update).
template <class PT, int PPT, int KP>
__global__ __launch_bounds__(kBlock) void k_update_xp(int n, int chunk, double *__restrict__ x,
                                                      PT *__restrict__ p, const double *__restrict__ r,
                                                      DevState *st, const double *__restrict__ rho_part,
                                                      int n_rho)
{
    __shared__ double red[kWaves];
    // the gate, the partials and the first vector elements are loaded
    // together (one memory round trip); nothing is stored before the gate
    const int status = st->status;
    const double alpha = st->alpha, rho = st->rho;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    const int t = threadIdx.x;
    double part[PPT];
    partials_load(rho_part, n_rho, part);
    double pv[KP], xv[KP], rv[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int i = i0 + t + u * kBlock;
        const bool ok = i < i1;
        pv[u] = ok ? (double)p[i] : 0.0;
        xv[u] = ok ? x[i] : 0.0;
        rv[u] = ok ? r[i] : 0.0;
    }
    if (status != kRun)
        return;
    const double rho_new = partials_sum(part, n_rho, red);
    const double beta = rho_new / rho;
    // last step: x only -- except for the FP32 directions of the mixed inner
    // solve, whose next direction carries over to the next refinement step
    const bool conv = sqrt(rho_new) <= st->tol_nb && sizeof(PT) == 8;
    if (blockIdx.x == 0 && t == 0) {
        st->rho_next = rho_new;
        st->conv_next = sqrt(rho_new) <= st->tol_nb ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int i = i0 + t + u * kBlock;
        if (i < i1) {
            x[i] = fma(alpha, pv[u], xv[u]);
            if (!conv)
                p[i] = (PT)fma(beta, pv[u], rv[u]);
        }
    }
    for (int i = i0 + t + KP * kBlock; i < i1; i += kBlock) {
        const double pi = (double)p[i];
        x[i] = fma(alpha, pi, x[i]);
        if (!conv)
            p[i] = (PT)fma(beta, pi, r[i]);
    }
}

// Mixed precision, start of an inner solve: rh = s .* r_out (scaled
// residual, FP64), p = fl32(rh), c = 0; partials of rh'rh (into both arrays:
// the inner solve's "b" is rh).
__global__ __launch_bounds__(kBlock) void k_mx_init(int n, int chunk, const double *__restrict__ r_out,
                                                    const double *__restrict__ s, double *__restrict__ rh,
                                                    float *__restrict__ p, double *__restrict__ c,
                                                    double *__restrict__ rho_part, double *__restrict__ bb_part,
                                                    int keep_p)
{
    __shared__ double red[kWaves];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    double a = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double v = s[i] * r_out[i];
        rh[i] = v;
        if (!keep_p)
            p[i] = (float)v;
        c[i] = 0.0;
        a = fma(v, v, a);
    }
    a = block_sum(a, red);
    if (threadIdx.x == 0) {
        rho_part[blk] = a;
        bb_part[blk] = a;
    }
}

// Mixed precision, end of an inner solve: x += s .* c.
__global__ __launch_bounds__(kBlock) void k_mx_apply(int n, double *__restrict__ x, const double *__restrict__ s,
                                                     const double *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        x[i] = fma(s[i], c[i], x[i]);
}

// Outer residual norm: st->rho = sum of partials, st->res_true = sqrt / nb.
__global__ __launch_bounds__(kBlock) void k_outer_norm(DevState *st, const double *__restrict__ part, int m)
{
    __shared__ double red[kWaves];
    const double rho = reduce_partials(part, m, red);
    if (threadIdx.x == 0) {
        st->rho = rho;
        st->res_true = st->nb > 0.0 ? sqrt(rho) / st->nb : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_check(DevState *st)
{
    iter_gate(st);
}

__global__ __launch_bounds__(kBlock) void k_init_vec(int n, int chunk, const double *__restrict__ b,
                                                     const double *__restrict__ x0, const double *__restrict__ q,
                                                     double *__restrict__ r, double *__restrict__ p,
                                                     double *__restrict__ xw, double *__restrict__ rho_part,
                                                     double *__restrict__ bb_part)
{
    __shared__ double red[kWaves];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    double ar = 0.0, ab = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double bi = b[i];
        const double ri = bi - q[i];
        r[i] = ri;
        p[i] = ri;
        xw[i] = x0[i];
        ar = fma(ri, ri, ar);
        ab = fma(bi, bi, ab);
    }
    ar = block_sum(ar, red);
    ab = block_sum(ab, red);
    if (threadIdx.x == 0) {
        rho_part[blk] = ar;
        bb_part[blk] = ab;
    }
}

__global__ __launch_bounds__(kBlock) void k_init_state(DevState *st, const double *__restrict__ bb_part,
                                                       const double *__restrict__ rho_part, int m, double tol,
                                                       int maxit)
{
    __shared__ double red[kWaves];
    const double nb = sqrt(reduce_partials(bb_part, m, red));
    const double rho = reduce_partials(rho_part, m, red);
    if (threadIdx.x == 0) {
        st->k = 0;
        st->iters = 0;
        st->maxit = maxit;
        st->nb = nb;
        st->rho = rho;
        st->alpha = 0.0;
        st->sigma = 0.0;
        st->res_true = 0.0;
        st->tol_nb = tol * nb;
        st->rho_next = rho;
        st->conv_next = sqrt(rho) <= tol * nb ? 1 : 0;
        st->status = !isfinite(nb) ? kNonfinite : (nb == 0.0 ? kZeroRhs : kRun);
    }
}

__global__ __launch_bounds__(kBlock) void k_resid_part(int n, int chunk, const double *__restrict__ b,
                                                       const double *__restrict__ q, double *__restrict__ part)
{
    __shared__ double red[kWaves];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    double a = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double d = b[i] - q[i];
        a = fma(d, d, a);
    }
    a = block_sum(a, red);
    if (threadIdx.x == 0)
        part[blk] = a;
}

__global__ __launch_bounds__(kBlock) void k_resid_finish(DevState *st, const double *__restrict__ part, int m)
{
    __shared__ double red[kWaves];
    const double s = reduce_partials(part, m, red);
    if (threadIdx.x == 0)
        st->res_true = st->nb > 0.0 ? sqrt(s) / st->nb : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_fill(int n, double *__restrict__ x, double v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        x[i] = v;
}

// New values for a planned matrix: val[k] = src[perm[k]] (perm = the
// normalisation's entry order, e.g. a lower triangle read as its transpose),
// or src[k] when there is none.
__global__ __launch_bounds__(kBlock) void k_gather_values(int64_t nnz, const double *__restrict__ src,
                                                          const int32_t *__restrict__ perm, double *__restrict__ val)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nnz)
        val[k] = src[perm ? perm[k] : k];
}

// Mixed precision after new values: s_l = 1 / sqrt(a_ll) per line; a line
// whose diagonal is absent, non-positive or not finite raises *bad.
__global__ __launch_bounds__(kBlock) void k_mx_diag(int n, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                    double *__restrict__ sc, int32_t *__restrict__ bad)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    double d = 0.0;
    for (int k = ptr[l]; k < ptr[l + 1]; ++k)
        if (idx[k] == l)
            d = val[k];
    if (!(d > 0.0) || !isfinite(d)) {
        *bad = 1;
        d = 1.0;
    }
    sc[l] = 1.0 / sqrt(d);
}

// Mixed precision: v32 = fl32(s_line * a * s_index), each product in FP64.
__global__ __launch_bounds__(kBlock) void k_mx_scale(int n, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                     const double *__restrict__ sc, float *__restrict__ v32)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    const double sl = sc[l];
    for (int k = ptr[l]; k < ptr[l + 1]; ++k)
        v32[k] = (float)(val[k] * sl * sc[idx[k]]);
}

// Gradient of a loss with respect to the stored values, given the adjoint
// solution lam (A lam = dL/dx) and the solution x: dL/dA_ij = -lam_i x_j.
// CSR (line = row i): -lam_l x_idx; CSC (line = column j): -lam_idx x_l;
// symmetric CSR (upper, one stored value stands for A_ij and A_ji):
// -(lam_l x_idx + lam_idx x_l), and -lam_l x_l on the diagonal.  Written in
// the caller's entry order (out[perm[k]]).  One thread per line.
__global__ __launch_bounds__(kBlock) void k_pattern_grad(int fmt, int n, const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ idx,
                                                         const double *__restrict__ lam,
                                                         const double *__restrict__ x,
                                                         const int32_t *__restrict__ perm, double *__restrict__ out)
{
#pragma clang fp contract(off)
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    const double ll = lam[l], xl = x[l];
    for (int k = ptr[l]; k < ptr[l + 1]; ++k) {
        const int j = idx[k];
        double g;
        if (fmt == kCsr) {
            g = -(ll * x[j]);
        } else if (fmt == kCsc) {
            g = -(lam[j] * xl);
        } else if (j == l) {
            g = -(ll * xl);
        } else {
            const double t1 = ll * x[j], t2 = lam[j] * xl; // two rounded products, then one rounded sum
            g = -(t1 + t2);
        }
        out[perm ? perm[k] : k] = g;
    }
}

// Parked sums of a scatter product: the handle's buffer, or the caller's
// scratch (IterCtx::part, products launched with a static scratch array).
inline double *parked_buf(const DevMatrix &m, const IterCtx &c)
{
    return c.part != nullptr ? c.part : m.part;
}

template <int W, class VT, class PT>
void csr_launch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_csr<W, 4, VT, PT>), dim3(m.csr_blocks), dim3(kBlock), 0, s, m.n,
                       m.csr_rows_per_block, m.ptr, m.idx, val, x, y, sig, c.st);
}

template <int SU, int E, class VT, class PT>
void scatter_launch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                    hipStream_t s)
{
    const size_t Ent = (size_t)m.lds_entries, R = (size_t)m.lds_lines;
    const size_t lds = Ent * 8 + R * 8 + (R + 1) * 4 + 2 * Ent * 2;
    hipLaunchKernelGGL((k_scatter_sums<SU, E, VT, PT>), dim3(m.scatter_wgs), dim3(kBlock), lds, s, m.ptr,
                       m.idx, val, x, y, parked_buf(m, c), sig, m.blocks, m.nblocks, m.slot_target, m.seg, m.tl,
                       m.lds_entries, m.lds_lines, c.st);
    if (m.ncolors > 1 && !c.defer_rows)
        hipLaunchKernelGGL(k_scatter_gather, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.n, m.rs_ptr,
                           m.rs_idx, m.has_c0, parked_buf(m, c), y, c.st);
}

inline const double *sym_slice_vals(const DevMatrix &m, const double *) { return m.ss_val; }
inline const float *sym_slice_vals(const DevMatrix &m, const float *) { return m.ss_val32; }

template <int SU, class VT, class PT>
void scatter_slices_launch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                           hipStream_t s)
{
    if (m.matrix_cached)
        hipLaunchKernelGGL((k_scatter_slices<SU, false, VT, PT>), dim3(m.scatter_wgs), dim3(kBlock), 0, s, m.ss_idx,
                           sym_slice_vals(m, val), m.ss_blk, x, y, parked_buf(m, c), sig, m.blocks, m.nblocks, m.slot_target,
                           m.seg, m.tl, c.st);
    else
        hipLaunchKernelGGL((k_scatter_slices<SU, true, VT, PT>), dim3(m.scatter_wgs), dim3(kBlock), 0, s, m.ss_idx,
                           sym_slice_vals(m, val), m.ss_blk, x, y, parked_buf(m, c), sig, m.blocks, m.nblocks, m.slot_target,
                           m.seg, m.tl, c.st);
    if (m.ncolors > 1 && !c.defer_rows)
        hipLaunchKernelGGL(k_scatter_gather, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.n, m.rs_ptr,
                           m.rs_idx, m.has_c0, parked_buf(m, c), y, c.st);
}

inline FusedDir fused_dir_of(const IterCtx &c)
{
    FusedDir fd;
    fd.pold = c.pold;
    fd.r = c.r;
    fd.pnew = c.pnew;
    fd.x = c.x;
    fd.rho_part = c.rho_part;
    fd.n_rho = c.n_rho;
    return fd;
}

template <int SU, class VT, class PT>
void compact_launch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                    hipStream_t s)
{
    if constexpr (sizeof(PT) == 8) {
        if (c.fused) { // two kernels per iteration (the row pass stays with the r update)
            if (m.matrix_cached)
                hipLaunchKernelGGL((k_scatter_compact<SU, false, VT, PT, true>), dim3(m.scatter_wgs),
                                   dim3(kCompactThreads), 0, s, m.ss_idx, sym_slice_vals(m, val), m.cblocks, m.nblocks,
                                   m.slot_target, m.seg, m.cp_rank, m.cp_dest, x, y, parked_buf(m, c), sig, c.st,
                                   fused_dir_of(c));
            else
                hipLaunchKernelGGL((k_scatter_compact<SU, true, VT, PT, true>), dim3(m.scatter_wgs),
                                   dim3(kCompactThreads), 0, s, m.ss_idx, sym_slice_vals(m, val), m.cblocks, m.nblocks,
                                   m.slot_target, m.seg, m.cp_rank, m.cp_dest, x, y, parked_buf(m, c), sig, c.st,
                                   fused_dir_of(c));
            return;
        }
    }
    if (m.matrix_cached)
        hipLaunchKernelGGL((k_scatter_compact<SU, false, VT, PT>), dim3(m.scatter_wgs), dim3(kCompactThreads), 0, s,
                           m.ss_idx,
                           sym_slice_vals(m, val), m.cblocks, m.nblocks, m.slot_target, m.seg, m.cp_rank, m.cp_dest, x, y, parked_buf(m, c),
                           sig, c.st);
    else
        hipLaunchKernelGGL((k_scatter_compact<SU, true, VT, PT>), dim3(m.scatter_wgs), dim3(kCompactThreads), 0, s,
                           m.ss_idx,
                           sym_slice_vals(m, val), m.cblocks, m.nblocks, m.slot_target, m.seg, m.cp_rank, m.cp_dest, x, y, parked_buf(m, c),
                           sig, c.st);
    if (m.parked > 0 && !c.defer_rows)
        hipLaunchKernelGGL(k_scatter_gather, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.n, m.rs_ptr,
                           m.rs_idx, nullptr, parked_buf(m, c), y, c.st);
}

template <class VT, class PT>
void compact_dispatch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                      hipStream_t s)
{
    if (m.max_slots <= 2 * kCompactThreads)
        compact_launch<2>(m, val, x, y, sig, c, s);
    else if (m.max_slots <= 4 * kCompactThreads)
        compact_launch<4>(m, val, x, y, sig, c, s);
    else
        compact_launch<10>(m, val, x, y, sig, c, s); // <= lines + entries = 9 x 512
}

template <int E, class VT, class PT>
void scatter_dispatch_su(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                         hipStream_t s)
{
    // write slots held in registers: SU per thread must cover the largest block
    if (m.sym_slices) {
        if (m.max_slots <= 2 * kBlock)
            scatter_slices_launch<2>(m, val, x, y, sig, c, s);
        else if (m.max_slots <= 4 * kBlock)
            scatter_slices_launch<4>(m, val, x, y, sig, c, s);
        else if (m.max_slots <= 6 * kBlock)
            scatter_slices_launch<6>(m, val, x, y, sig, c, s);
        else
            scatter_slices_launch<9>(m, val, x, y, sig, c, s);
        return;
    }
    if (m.max_slots <= 2 * kBlock)
        scatter_launch<2, E>(m, val, x, y, sig, c, s);
    else if (m.max_slots <= 4 * kBlock)
        scatter_launch<4, E>(m, val, x, y, sig, c, s);
    else if (m.max_slots <= 6 * kBlock)
        scatter_launch<6, E>(m, val, x, y, sig, c, s);
    else
        scatter_launch<9, E>(m, val, x, y, sig, c, s);
}

template <class VT, class PT>
void scatter_dispatch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig, const IterCtx &c,
                      hipStream_t s)
{
    // entries held in registers: E per thread must cover the largest block
    if (m.lds_entries <= 4 * kBlock)
        scatter_dispatch_su<4>(m, val, x, y, sig, c, s);
    else
        scatter_dispatch_su<kMaxScatterEntries / kBlock>(m, val, x, y, sig, c, s);
}

inline const double *panel_vals(const DevMatrix &m, const double *) { return m.pn_val; }
inline const float *panel_vals(const DevMatrix &m, const float *) { return m.pn_val32; }
inline const double *slice_vals(const DevMatrix &m, const double *) { return m.sl_val; }
inline const float *slice_vals(const DevMatrix &m, const float *) { return m.sl_val32; }

template <bool PANEL, int S, bool NT, class VT, class PT>
void slices_launch_nt(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig_part, const IterCtx &c,
                      hipStream_t s)
{
    if constexpr (!PANEL && sizeof(PT) == 8) {
        if (c.fused) { // two kernels per iteration
            if (m.sl_d16 != nullptr)
                hipLaunchKernelGGL((k_spmv_slices<false, S, NT, VT, PT, int16_t, true>), dim3(m.csr_blocks),
                                   dim3(kBlock), 0, s, m.sl_lines, m.nslices, m.sl_off, m.sl_d16, val, x, y, nullptr,
                                   nullptr, 0, sig_part, c.st, fused_dir_of(c));
            else
                hipLaunchKernelGGL((k_spmv_slices<false, S, NT, VT, PT, int32_t, true>), dim3(m.csr_blocks),
                                   dim3(kBlock), 0, s, m.sl_lines, m.nslices, m.sl_off, m.sl_col, val, x, y, nullptr,
                                   nullptr, 0, sig_part, c.st, fused_dir_of(c));
            return;
        }
    }
    if (m.sl_d16 != nullptr)
        hipLaunchKernelGGL((k_spmv_slices<PANEL, S, NT, VT, PT, int16_t>), dim3(m.csr_blocks), dim3(kBlock), 0, s,
                           m.sl_lines, m.nslices, m.sl_off, m.sl_d16, val, x, y,
                           PANEL ? m.pn_slot_target : nullptr, PANEL ? parked_buf(m, c) : nullptr,
                           PANEL ? m.pn_first_parked : 0, sig_part, c.st);
    else
        hipLaunchKernelGGL((k_spmv_slices<PANEL, S, NT, VT, PT, int32_t>), dim3(m.csr_blocks), dim3(kBlock), 0, s,
                           m.sl_lines, m.nslices, m.sl_off, m.sl_col, val, x, y,
                           PANEL ? m.pn_slot_target : nullptr, PANEL ? parked_buf(m, c) : nullptr,
                           PANEL ? m.pn_first_parked : 0, sig_part, c.st);
}

template <bool PANEL, int S, class VT, class PT>
void slices_launch(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig_part, const IterCtx &c,
                   hipStream_t s)
{
    if (m.matrix_cached)
        slices_launch_nt<PANEL, S, false>(m, val, x, y, sig_part, c, s);
    else
        slices_launch_nt<PANEL, S, true>(m, val, x, y, sig_part, c, s);
}

template <class VT, class PT>
void spmv_any(const DevMatrix &m, const VT *val, const PT *x, double *y, double *sig_part, const IterCtx &c,
              hipStream_t s)
{
    if (m.n == 0)
        return;
    if (m.slices) {
        // two slices per wave at a time once the waves average 1.5 or more
        // (160^3 CSR: FP64 132.8 -> 128.5 us per product; the FP32 product of
        // mixed precision gains too, the mixed solve 72.5 -> 71.4 ms)
        static const bool two_knob = [] { // experiments: CGMI_SLICE_TWO=0, one slice at a time
            const char *e = std::getenv("CGMI_SLICE_TWO");
            return !(e && std::strcmp(e, "0") == 0);
        }();
        const bool two = two_knob && 2 * (int64_t)m.nslices >= (int64_t)3 * kWaves * m.csr_blocks;
        if (m.panel && two)
            slices_launch<true, 2>(m, slice_vals(m, val), x, y, sig_part, c, s);
        else if (m.panel)
            slices_launch<true, 1>(m, slice_vals(m, val), x, y, sig_part, c, s);
        else if (two)
            slices_launch<false, 2>(m, slice_vals(m, val), x, y, sig_part, c, s);
        else
            slices_launch<false, 1>(m, slice_vals(m, val), x, y, sig_part, c, s);
    } else if (m.panel && m.nblocks > 0) {
        hipLaunchKernelGGL((k_panel_rows<VT, PT>), dim3(m.scatter_wgs), dim3(kBlock), 0, s, m.nblocks,
                           m.pn_chunk_slot, m.pn_slot_ptr, m.pn_slot_target, m.pn_col, panel_vals(m, val), x, y,
                           parked_buf(m, c), m.pn_first_parked, sig_part, c.st);
    }
    if (m.panel) {
        if (m.pn_gather && !c.defer_rows)
            hipLaunchKernelGGL(k_panel_gather, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.n,
                               m.has_c0, parked_buf(m, c), y, c.st);
        return;
    }
    if (m.slices)
        return;
    if (m.format == kCsr && m.csr_stream) {
        hipLaunchKernelGGL((k_spmv_csr_rows<VT, PT>), dim3(m.csr_blocks), dim3(kBlock), 0, s, m.csr_nrb, m.csr_rbe,
                           m.ptr, m.idx, val, x, y, sig_part, c.st);
    } else if (m.format == kCsr) {
        switch (m.lanes) {
        case 4: csr_launch<4>(m, val, x, y, sig_part, c, s); break;
        case 8: csr_launch<8>(m, val, x, y, sig_part, c, s); break;
        case 16: csr_launch<16>(m, val, x, y, sig_part, c, s); break;
        case 32: csr_launch<32>(m, val, x, y, sig_part, c, s); break;
        default: csr_launch<64>(m, val, x, y, sig_part, c, s); break;
        }
    } else if (m.compact) {
        compact_dispatch(m, val, x, y, sig_part, c, s); // symmetric CSR, compact blocks
    } else {
        scatter_dispatch(m, val, x, y, sig_part, c, s); // symmetric CSR, coloured (CSC runs on panels)
    }
}

} // namespace

void launch_spmv(const DevMatrix &m, const double *x, double *y, double *sig_part, const IterCtx &c, hipStream_t s)
{
    spmv_any(m, m.val, x, y, sig_part, c, s);
}

void launch_spmv32(const DevMatrix &m, const float *x, double *y, double *sig_part, const IterCtx &c, hipStream_t s)
{
    spmv_any(m, m.val32, x, y, sig_part, c, s);
}

// Elements per thread loaded up front by the vector kernels: the smallest
// power of two covering the chunk, at most kPre.
static int prefetch_depth(int chunk)
{
    int kp = 1;
    while (kp < kPre && kp * kBlock < chunk)
        kp *= 2;
    return kp;
}

void launch_update_r(const DevMatrix &m, double *r, const double *q, DevState *st, const double *sig_part,
                     double *rho_part, hipStream_t s, bool rows_deferred, bool fused)
{
    static_assert(kMaxSliceWgs <= 4 * kPartPerThread * kBlock, "slice partials fit four times the registers");
    // slices: up to kMaxSliceWgs dot partials (one slice per wavefront); the
    // r update then holds up to 32 of them per thread
    const int nsig = m.spmv_blocks();
    // partials per thread: the smallest power of two that covers nsig (each
    // is a load, also past nsig: they are read unguarded, at a clamped index)
    int ppt = 1;
    while (ppt * kBlock < nsig)
        ppt *= 2;
    RowPass g;
    g.rs_ptr = m.rs_ptr;
    g.rs_idx = m.rs_idx;
    g.has_c0 = m.has_c0;
    g.part = m.part; // iterations use the handle's own buffer
    const int mode = rows_deferred && m.row_pass() ? (m.panel ? 2 : m.compact ? 3 : 1) : 0;
    const dim3 grid(m.vec_blocks), blk(kBlock);
    const int kp = prefetch_depth(m.vec_chunk);
#define CGMI_UPDATE_R_KP(G, P, F, K)                                                                         \
    hipLaunchKernelGGL((k_update_r<G, P, F, K>), grid, blk, 0, s, m.n, m.vec_chunk, r, q, st, sig_part, nsig,   \
                       rho_part, g)
#define CGMI_UPDATE_R(G, P, F)                                                                               \
    do {                                                                                                     \
        switch (kp) {                                                                                        \
        case 1: CGMI_UPDATE_R_KP(G, P, F, 1); break;                                                         \
        case 2: CGMI_UPDATE_R_KP(G, P, F, 2); break;                                                         \
        case 4: CGMI_UPDATE_R_KP(G, P, F, 4); break;                                                         \
        default: CGMI_UPDATE_R_KP(G, P, F, kPre); break;                                                     \
        }                                                                                                    \
    } while (0)
#define CGMI_UPDATE_R_PPT(G, F)                                                                              \
    do {                                                                                                     \
        switch (ppt) {                                                                                       \
        case 1: CGMI_UPDATE_R(G, 1, F); break;                                                               \
        case 2: CGMI_UPDATE_R(G, 2, F); break;                                                               \
        case 4: CGMI_UPDATE_R(G, 4, F); break;                                                               \
        case 8: CGMI_UPDATE_R(G, 8, F); break;                                                               \
        case 16: CGMI_UPDATE_R(G, 16, F); break;                                                             \
        default: CGMI_UPDATE_R(G, 32, F); break;                                                             \
        }                                                                                                    \
    } while (0)
    if (fused && mode == 3) // two kernels per iteration: compact blocks or CSR slices
        CGMI_UPDATE_R_PPT(3, true);
    else if (fused)
        CGMI_UPDATE_R_PPT(0, true);
    else if (mode == 3)
        CGMI_UPDATE_R_PPT(3, false);
    else if (mode == 2)
        CGMI_UPDATE_R_PPT(2, false);
    else if (mode == 1)
        CGMI_UPDATE_R_PPT(1, false);
    else
        CGMI_UPDATE_R_PPT(0, false);
#undef CGMI_UPDATE_R_PPT
#undef CGMI_UPDATE_R
#undef CGMI_UPDATE_R_KP
}

// x/p update with PPT partials per thread: the smallest power of two that
// covers the vector kernels' workgroups
template <class PT>
void update_xp_launch(const DevMatrix &m, double *x, PT *p, const double *r, DevState *st, const double *rho_part,
                      hipStream_t s)
{
    static_assert(kMaxVecBlocks <= 8 * kBlock, "vector partials fit eight per thread");
    const dim3 grid(m.vec_blocks), blk(kBlock);
    const int kp = prefetch_depth(m.vec_chunk);
#define CGMI_UPDATE_XP_KP(P, K)                                                                              \
    hipLaunchKernelGGL((k_update_xp<PT, P, K>), grid, blk, 0, s, m.n, m.vec_chunk, x, p, r, st, rho_part, m.vec_blocks)
#define CGMI_UPDATE_XP(P)                                                                                    \
    do {                                                                                                     \
        switch (kp) {                                                                                        \
        case 1: CGMI_UPDATE_XP_KP(P, 1); break;                                                              \
        case 2: CGMI_UPDATE_XP_KP(P, 2); break;                                                              \
        case 4: CGMI_UPDATE_XP_KP(P, 4); break;                                                              \
        default: CGMI_UPDATE_XP_KP(P, kPre); break;                                                          \
        }                                                                                                    \
    } while (0)
    if (m.vec_blocks <= kBlock)
        CGMI_UPDATE_XP(1);
    else if (m.vec_blocks <= 2 * kBlock)
        CGMI_UPDATE_XP(2);
    else if (m.vec_blocks <= 4 * kBlock)
        CGMI_UPDATE_XP(4);
    else
        CGMI_UPDATE_XP(8);
#undef CGMI_UPDATE_XP
#undef CGMI_UPDATE_XP_KP
}

void launch_update_xp(const DevMatrix &m, double *x, double *p, const double *r, DevState *st,
                      const double *rho_part, hipStream_t s)
{
    update_xp_launch(m, x, p, r, st, rho_part, s);
}

void launch_update_xp32(const DevMatrix &m, double *x, float *p, const double *r, DevState *st,
                        const double *rho_part, hipStream_t s)
{
    update_xp_launch(m, x, p, r, st, rho_part, s);
}

void launch_mx_init(const DevMatrix &m, const double *r_out, double *rh, float *p, double *c, double *rho_part,
                    double *bb_part, hipStream_t s, bool keep_p)
{
    hipLaunchKernelGGL(k_mx_init, dim3(m.vec_blocks), dim3(kBlock), 0, s, m.n, m.vec_chunk, r_out, m.dscale, rh,
                       p, c, rho_part, bb_part, keep_p ? 1 : 0);
}

void launch_mx_apply(const DevMatrix &m, double *x, const double *c, hipStream_t s)
{
    if (m.n > 0)
        hipLaunchKernelGGL(k_mx_apply, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.n, x, m.dscale, c);
}

void launch_outer_norm(const DevMatrix &m, DevState *st, const double *rho_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_outer_norm, dim3(1), dim3(kBlock), 0, s, st, rho_part, m.vec_blocks);
}

void launch_check(const DevMatrix &m, DevState *st, const double *rho_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, st);
}

void launch_init_vec(const DevMatrix &m, const double *b, const double *x0, const double *q, double *r, double *p,
                     double *xw, double *rho_part, double *bb_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_vec, dim3(m.vec_blocks), dim3(kBlock), 0, s, m.n, m.vec_chunk, b, x0, q, r, p, xw,
                       rho_part, bb_part);
}

void launch_init_state(const DevMatrix &m, DevState *st, const double *bb_part, const double *rho_part, double tol,
                       int32_t maxit, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(kBlock), 0, s, st, bb_part, rho_part, m.vec_blocks, tol, maxit);
}

void launch_true_residual(const DevMatrix &m, const double *b, const double *q, double *part, DevState *st,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_resid_part, dim3(m.vec_blocks), dim3(kBlock), 0, s, m.n, m.vec_chunk, b, q, part);
    hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(kBlock), 0, s, st, part, m.vec_blocks);
}

void launch_fill(int n, double *x, double v, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, x, v);
}

void launch_permute(int64_t nnz, const double *src, const int32_t *perm, double *dst, hipStream_t s)
{
    if (nnz > 0)
        hipLaunchKernelGGL(k_permute<double>, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nnz,
                           src, perm, dst);
}

void launch_permute(int64_t nnz, const float *src, const int32_t *perm, float *dst, hipStream_t s)
{
    if (nnz > 0)
        hipLaunchKernelGGL(k_permute<float>, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nnz,
                           src, perm, dst);
}

void launch_set_values(int64_t nnz, const double *src, const int32_t *perm, double *val, hipStream_t s)
{
    if (nnz > 0)
        hipLaunchKernelGGL(k_gather_values, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nnz,
                           src, perm, val);
}

void launch_mx_rescale(const DevMatrix &m, double *sc, float *v32, int32_t *bad, hipStream_t s)
{
    if (m.n <= 0)
        return;
    const dim3 g((m.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_mx_diag, g, dim3(kBlock), 0, s, m.n, m.ptr, m.idx, m.val, sc, bad);
    hipLaunchKernelGGL(k_mx_scale, g, dim3(kBlock), 0, s, m.n, m.ptr, m.idx, m.val, sc, v32);
}

void launch_pattern_grad(const DevMatrix &m, const double *lam, const double *x, const int32_t *perm, double *out,
                         hipStream_t s)
{
    if (m.n > 0)
        hipLaunchKernelGGL(k_pattern_grad, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.format, m.n,
                           m.ptr, m.idx, lam, x, perm, out);
}

} // namespace cgmi

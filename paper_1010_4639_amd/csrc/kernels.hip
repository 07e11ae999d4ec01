// HIP kernels for gfx950 (CDNA4, wave64): sparse products over CSR, symmetric
// CSR and CSC, and the fused vector / reduction steps of conjugate gradient.
//
// All kernels use 256-thread workgroups.  Every reduction is a fixed tree
// (butterfly inside a wavefront, waves summed in index order, partials summed
// by a fixed per-thread stride), so results are bitwise reproducible.  No
// floating-point atomics anywhere; the only cross-workgroup communication is
// through per-workgroup partials read by a later kernel.
#include "kernels.h"

#include <cmath>

namespace cgmi {

namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kXcds = 8; // MI355X: workgroups are dealt round-robin to 8 XCDs, each with its own L2

// Workgroup id -> logical chunk, so that each XCD works on one contiguous
// range of chunks (neighbouring rows share x and y lines in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    const int per = nblk / kXcds, rem = nblk % kXcds;
    const int x = bid % kXcds, i = bid / kXcds;
    return x * per + min(x, rem) + i;
}

template <int W>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, W);
    return v; // butterfly: every lane of the group holds the same bits
}

// Sum over the workgroup; every thread returns the same bits.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = red[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w)
        t += red[w];
    return t;
}

// Sum of m per-workgroup partials, identical in every workgroup.
__device__ __forceinline__ double reduce_partials(const double *__restrict__ part, int m, double *red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += kBlock)
        s += part[i];
    return block_sum(s, red);
}

// Start of an iteration (before its product): stop when the current residual
// meets the tolerance or maxit products are done.  Every workgroup takes the
// same decision from the same bits; only workgroup 0 records it.
__device__ bool iter_gate(DevState *st, const double *__restrict__ rho_part, int n_rho, double *red)
{
    if (st->status != kRun)
        return false;
    const double rho = reduce_partials(rho_part, n_rho, red);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const int k = st->k;
    if (sqrt(rho) <= st->tol_nb) {
        if (lead) {
            st->rho = rho;
            st->iters = k;
            st->status = kConverged;
        }
        return false;
    }
    if (k >= st->maxit) {
        if (lead) {
            st->rho = rho;
            st->iters = k;
            st->status = kMaxit;
        }
        return false;
    }
    if (lead)
        st->rho = rho;
    return true;
}

// ------------------------------------------------------------------ CSR
// W lanes per row (4..64), U rows per lane group in flight, rows of the
// workgroup's contiguous range visited in passes of (256 / W) * U rows.
// Index / value streams use non-temporal loads (read once); x is gathered
// through the cache.  Fused epilogue: partial of x'y.
template <int W, int U>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int n, int rows_per_block, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     double *__restrict__ sig_part, DevState *st,
                                                     const double *__restrict__ rho_part, int n_rho)
{
    __shared__ double red[kWaves];
    if (st != nullptr && !iter_gate(st, rho_part, n_rho, red))
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
                v[u] = ok ? __builtin_nontemporal_load(val + k) : 0.0;
            }
            if (!any)
                break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xv = c[u] >= 0 ? x[c[u]] : 0.0;
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
            sig = fma(x[row], yv, sig);
        }
    }
    sig = block_sum(sig, red);
    if (threadIdx.x == 0)
        sig_part[blk] = sig;
}

// --------------------------------------------------- colour-phase scatter
// One workgroup per scatter block (see plan.h).  Stage 1: lane groups walk
// the block's lines; every product bound for another row is parked in LDS at
// its entry's local index (symmetric CSR also gathers its own row, incl. the
// diagonal, in registers).  Stage 2: one thread per write slot sums that
// slot's products in the fixed order of the plan and stores (first writer) or
// adds to (later colour) y; the last writer of a row adds p_i y_i to the dot.
template <bool SYM, int W>
__global__ __launch_bounds__(kBlock) void k_spmv_scatter(
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx, const double *__restrict__ val,
    const double *__restrict__ x, double *__restrict__ y, double *__restrict__ sig_part,
    const ScatterBlock *__restrict__ blocks, const int32_t *__restrict__ phase_blocks,
    const int32_t *__restrict__ slot_target, const uint8_t *__restrict__ slot_flag,
    const uint16_t *__restrict__ seg, const uint16_t *__restrict__ tl, int lds_entries, DevState *st,
    const double *__restrict__ rho_part, int n_rho, int gate)
{
    extern __shared__ double lds[];
    __shared__ double red[kWaves];
    if (st != nullptr) {
        if (gate) {
            if (!iter_gate(st, rho_part, n_rho, red))
                return;
        } else if (st->status != kRun) {
            return;
        }
    }
    const ScatterBlock bk = blocks[phase_blocks[xcd_remap(blockIdx.x, gridDim.x)]];
    double *sp = lds;
    double *gs = lds + lds_entries;
    constexpr int NG = kBlock / W;
    const int g = threadIdx.x / W, lane = threadIdx.x % W;
    for (int l = bk.line0 + g; l < bk.line1; l += NG) {
        const int s = max(ptr[l], bk.k0), e = min(ptr[l + 1], bk.k1);
        const double xl = x[l];
        double ga = 0.0;
        for (int k = s + lane; k < e; k += W) {
            const int j = __builtin_nontemporal_load(idx + k);
            const double v = __builtin_nontemporal_load(val + k);
            if (SYM) {
                ga = fma(v, x[j], ga);
                if (j != l)
                    sp[k - bk.k0] = v * xl;
            } else {
                sp[k - bk.k0] = v * xl;
            }
        }
        if (SYM) {
            ga = group_sum<W>(ga);
            if (lane == 0)
                gs[l - bk.line0] = ga;
        }
    }
    __syncthreads();
    const int nown = SYM ? bk.line1 - bk.line0 : 0;
    const uint16_t *sg = seg + bk.slot0 + bk.id;
    const uint16_t *tt = tl + bk.tl0;
    const int32_t *tg = slot_target + bk.slot0;
    const uint8_t *fl = slot_flag + bk.slot0;
    double sig = 0.0;
    for (int s = threadIdx.x; s < bk.nslots; s += kBlock) {
        double a = s < nown ? gs[s] : 0.0;
        const int t0 = sg[s], t1 = sg[s + 1];
        for (int t = t0; t < t1; ++t)
            a += sp[tt[t]];
        const int row = tg[s];
        const unsigned f = fl[s];
        const double yv = (f & kSlotFirst) ? a : y[row] + a;
        y[row] = yv;
        if (f & kSlotLast)
            sig = fma(x[row], yv, sig);
    }
    sig = block_sum(sig, red);
    if (threadIdx.x == 0)
        sig_part[bk.id] = sig;
}

// ------------------------------------------------------ vector kernels
__global__ __launch_bounds__(kBlock) void k_update_r(int n, int chunk, double *__restrict__ r,
                                                     const double *__restrict__ q, DevState *st,
                                                     const double *__restrict__ sig_part, int n_sig,
                                                     double *__restrict__ rho_part)
{
    __shared__ double red[kWaves];
    if (st->status != kRun)
        return;
    const double sigma = reduce_partials(sig_part, n_sig, red);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) {
            st->iters = st->k;
            st->sigma = sigma;
            st->status = kBreakdown;
        }
        return;
    }
    const double alpha = st->rho / sigma;
    if (lead) {
        st->alpha = alpha;
        st->sigma = sigma;
        st->k = st->k + 1;
    }
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    double acc = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0)
        rho_part[blk] = acc;
}

__global__ __launch_bounds__(kBlock) void k_update_xp(int n, int chunk, double *__restrict__ x,
                                                      double *__restrict__ p, const double *__restrict__ r,
                                                      const DevState *st, const double *__restrict__ rho_part,
                                                      int n_rho)
{
    __shared__ double red[kWaves];
    if (st->status != kRun)
        return;
    const double rho_new = reduce_partials(rho_part, n_rho, red);
    const double alpha = st->alpha;
    const double beta = rho_new / st->rho;
    const bool conv = sqrt(rho_new) <= st->tol_nb; // last step: x only
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = blk * chunk, i1 = min(n, i0 + chunk);
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double pi = p[i];
        x[i] = fma(alpha, pi, x[i]);
        if (!conv)
            p[i] = fma(beta, pi, r[i]);
    }
}

__global__ __launch_bounds__(kBlock) void k_check(DevState *st, const double *__restrict__ rho_part, int n_rho)
{
    __shared__ double red[kWaves];
    iter_gate(st, rho_part, n_rho, red);
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

template <int W>
void csr_launch(const DevMatrix &m, const double *x, double *y, double *sig, const IterCtx &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_csr<W, 4>), dim3(m.csr_blocks), dim3(kBlock), 0, s, m.n, m.csr_rows_per_block,
                       m.ptr, m.idx, m.val, x, y, sig, c.st, c.rho_part, c.n_rho);
}

template <bool SYM, int W>
void scatter_launch(const DevMatrix &m, const double *x, double *y, double *sig, const IterCtx &c, hipStream_t s)
{
    const size_t lds = (size_t)(m.lds_entries + m.lds_lines) * sizeof(double);
    for (int col = 0; col < m.ncolors; ++col) {
        const int nb = m.color_off[col + 1] - m.color_off[col];
        hipLaunchKernelGGL((k_spmv_scatter<SYM, W>), dim3(nb), dim3(kBlock), lds, s, m.ptr, m.idx, m.val, x, y,
                           sig, m.blocks, m.phase_blocks + m.color_off[col], m.slot_target, m.slot_flag, m.seg,
                           m.tl, m.lds_entries, c.st, c.rho_part, c.n_rho, col == 0 ? 1 : 0);
    }
}

template <bool SYM>
void scatter_dispatch(const DevMatrix &m, const double *x, double *y, double *sig, const IterCtx &c, hipStream_t s)
{
    switch (m.lanes) {
    case 4: scatter_launch<SYM, 4>(m, x, y, sig, c, s); break;
    case 8: scatter_launch<SYM, 8>(m, x, y, sig, c, s); break;
    case 16: scatter_launch<SYM, 16>(m, x, y, sig, c, s); break;
    case 32: scatter_launch<SYM, 32>(m, x, y, sig, c, s); break;
    default: scatter_launch<SYM, 64>(m, x, y, sig, c, s); break;
    }
}

} // namespace

void launch_spmv(const DevMatrix &m, const double *x, double *y, double *sig_part, const IterCtx &c, hipStream_t s)
{
    if (m.n == 0)
        return;
    if (m.format == kCsr) {
        switch (m.lanes) {
        case 4: csr_launch<4>(m, x, y, sig_part, c, s); break;
        case 8: csr_launch<8>(m, x, y, sig_part, c, s); break;
        case 16: csr_launch<16>(m, x, y, sig_part, c, s); break;
        case 32: csr_launch<32>(m, x, y, sig_part, c, s); break;
        default: csr_launch<64>(m, x, y, sig_part, c, s); break;
        }
    } else if (m.format == kSymCsr) {
        scatter_dispatch<true>(m, x, y, sig_part, c, s);
    } else {
        scatter_dispatch<false>(m, x, y, sig_part, c, s);
    }
}

void launch_update_r(const DevMatrix &m, double *r, const double *q, DevState *st, const double *sig_part,
                     double *rho_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_update_r, dim3(m.vec_blocks), dim3(kBlock), 0, s, m.n, m.vec_chunk, r, q, st, sig_part,
                       m.spmv_blocks(), rho_part);
}

void launch_update_xp(const DevMatrix &m, double *x, double *p, const double *r, const DevState *st,
                      const double *rho_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_update_xp, dim3(m.vec_blocks), dim3(kBlock), 0, s, m.n, m.vec_chunk, x, p, r, st,
                       rho_part, m.vec_blocks);
}

void launch_check(const DevMatrix &m, DevState *st, const double *rho_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, st, rho_part, m.vec_blocks);
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

} // namespace cgmi

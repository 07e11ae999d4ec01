// Batched conjugate gradient: many independent SPD systems of uneven size,
// each with R right-hand sides, advanced in lockstep by one sequence of
// kernels (captured in a HIP graph), every (system, right-hand side) pair --
// an "instance" -- with its own alpha, beta, residual and stopping test.
//
// Layout.  The systems are one block-diagonal CSR matrix (rows of system s
// are [sys_off[s], sys_off[s+1]), its columns stay inside that range).  The
// R right-hand sides are interleaved: element (i, r) of a vector sits at
// i*R + r, so a gathered column brings all R values in one 8R-byte access and
// the matrix is read once for all R products.  Rows are cut into row blocks
// that never span two systems; each workgroup owns a contiguous range of one
// system's row blocks, so every dot-product partial belongs to exactly one
// system and a system's scalars are sums over its own workgroups only.
//
// Per iteration: k_bspmm (Q = A P, partials of p'q per instance), k_bupdate_r
// (alpha, r -= alpha q, partials of r'r), k_bupdate_xp (beta, x += alpha p,
// p = r + beta p; the system's lead workgroup publishes r'r and the stop
// decision), as in the single-system solver.  Instances that stopped are
// skipped; a system whose instances have all stopped costs only early
// returns.  k_bcheck counts the running instances after each graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/cgmi.h"
#include "devutil.h"
#include "kernels.h"
#include "plan.h"

using namespace cgmi;
using namespace cgmi::dev;

namespace {

struct Inst {
    int32_t status, k, maxit, iters;
    int32_t conv_next, pad0, pad1, pad2;
    double tol_nb, nb, rho, alpha, sigma, rho_next, res_true, pad3;
};

struct WgDesc {
    int32_t sys, lead;   // system; 1 for the system's first workgroup
    int32_t rb0, rb1;    // row blocks [rb0, rb1)
    int32_t i0, i1;      // rows [i0, i1)
    int32_t wg0, wg1;    // workgroups of the system (its partials)
};


__device__ __forceinline__ bool inst_gate(Inst *I, bool lead)
{
    if (I->status != kRun)
        return false;
    const int k = I->k;
    if (I->conv_next) {
        if (lead) {
            I->rho = I->rho_next;
            I->iters = k;
            I->status = kConverged;
        }
        return false;
    }
    if (k >= I->maxit) {
        if (lead) {
            I->rho = I->rho_next;
            I->iters = k;
            I->status = kMaxit;
        }
        return false;
    }
    if (lead)
        I->rho = I->rho_next;
    return true;
}

// Q = A P for the R interleaved right-hand sides (row blocks of <= 256*EPT
// entries staged in LDS, one thread sums each row left to right).
// Q = A P for the R interleaved right-hand sides, W lanes per row (the
// second schedule the autotuner can pick): each lane accumulates R partial
// sums over the entries lane, lane + W, ... of its row, with U rows in flight
// per lane group, and the W lanes combine them by a butterfly (fixed order);
// the R values of a gathered row of P come in 16-byte loads.  No LDS, so
// occupancy is set by registers alone.
template <int R, int W, int U>
__global__ __launch_bounds__(kBlock) void k_bspmm_lanes(const WgDesc *__restrict__ wgs,
                                                        const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ P, double *__restrict__ Q,
                                                        double *__restrict__ sig_part, Inst *inst)
{
    static_assert(R <= W, "one storing lane per right-hand side");
    __shared__ double red[kWaves];
    __shared__ int act_s[R];
    constexpr int NG = kBlock / W;
    const WgDesc Wd = wgs[blockIdx.x];
    const int t = threadIdx.x;
    bool any = true;
    if (inst != nullptr) {
        if (t < R)
            act_s[t] = inst_gate(&inst[Wd.sys * R + t], Wd.lead != 0) ? 1 : 0;
        __syncthreads();
        any = false;
#pragma unroll
        for (int r = 0; r < R; ++r)
            any |= act_s[r] != 0;
    }
    const int g = t / W, lane = t % W;
    double sg = 0.0; // lane r < R: partial of p'q for right-hand side r
    if (any) {
        for (int base = Wd.i0 + g; base < Wd.i1; base += NG * U) {
            int rs[U], re[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = base + u * NG;
                const bool ok = r < Wd.i1;
                rs[u] = ok ? __builtin_nontemporal_load(ptr + r) : 0;
                re[u] = ok ? __builtin_nontemporal_load(ptr + r + 1) : 0;
            }
            double acc[U][R];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[u][r] = 0.0;
            for (int off = lane;; off += W) {
                bool anyk = false;
                int c[U];
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = rs[u] + off;
                    const bool ok = k < re[u];
                    anyk |= ok;
                    c[u] = ok ? __builtin_nontemporal_load(col + k) : -1;
                    v[u] = ok ? __builtin_nontemporal_load(val + k) : 0.0;
                }
                if (!anyk)
                    break;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (c[u] < 0)
                        continue;
                    if constexpr (R % 2 == 0) {
                        const double2 *p2 = reinterpret_cast<const double2 *>(P + (size_t)c[u] * R);
#pragma unroll
                        for (int h2 = 0; h2 < R / 2; ++h2) {
                            const double2 pv = p2[h2];
                            acc[u][2 * h2] = fma(v[u], pv.x, acc[u][2 * h2]);
                            acc[u][2 * h2 + 1] = fma(v[u], pv.y, acc[u][2 * h2 + 1]);
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            acc[u][r] = fma(v[u], P[(size_t)c[u] * R + r], acc[u][r]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int row = base + u * NG;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double q = group_sum<W>(acc[u][r]);
                    if (lane == r && row < Wd.i1) {
                        Q[(size_t)row * R + r] = q;
                        sg = fma(P[(size_t)row * R + r], q, sg);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sr = block_sum(lane == r ? sg : 0.0, red);
        if (t == 0)
            sig_part[blockIdx.x * R + r] = sr;
    }
}

template <int R, int EPT>
__global__ __launch_bounds__(kBlock) void k_bspmm(const WgDesc *__restrict__ wgs, const int32_t *__restrict__ rb_row,
                                                  const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                  const double *__restrict__ val, const double *__restrict__ P,
                                                  double *__restrict__ Q, double *__restrict__ sig_part, Inst *inst)
{
    constexpr int E = kBlock * EPT;
    __shared__ double prod[E * R];
    __shared__ int32_t lptr[kStreamRows + 1];
    __shared__ double red[kWaves];
    __shared__ int act_s[R];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x;
    bool any = true;
    if (inst != nullptr) {
        if (t < R)
            act_s[t] = inst_gate(&inst[W.sys * R + t], W.lead != 0) ? 1 : 0;
        __syncthreads();
        any = false;
#pragma unroll
        for (int r = 0; r < R; ++r)
            any |= act_s[r] != 0;
    }
    double sig[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        sig[r] = 0.0;
    if (any) {
        for (int b = W.rb0; b < W.rb1; ++b) {
            const int r0 = rb_row[b], r1 = rb_row[b + 1];
            const int nr = r1 - r0;
            const int e0 = ptr[r0], e1 = ptr[r1];
            if (e1 - e0 > E) { // one long row: workgroup tree per right-hand side
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double a = 0.0;
                    for (int e = e0 + t; e < e1; e += kBlock)
                        a = fma(val[e], P[(size_t)col[e] * R + r], a);
                    a = block_sum(a, red);
                    if (t == 0) {
                        Q[(size_t)r0 * R + r] = a;
                        sig[r] = fma(P[(size_t)r0 * R + r], a, sig[r]);
                    }
                }
                continue;
            }
            int c[EPT];
            double v[EPT];
#pragma unroll
            for (int m = 0; m < EPT; ++m) {
                const int e = e0 + t + m * kBlock;
                const bool ok = e < e1;
                c[m] = ok ? __builtin_nontemporal_load(col + e) : -1;
                v[m] = ok ? __builtin_nontemporal_load(val + e) : 0.0;
            }
            if (t < nr)
                lptr[t + 1] = ptr[r0 + t + 1] - e0;
            if (t == 0)
                lptr[0] = 0;
            // products stored by right-hand side (plane r holds entry e at r*E + e):
            // consecutive threads write consecutive words, and a row's sum reads
            // one contiguous run per plane
#pragma unroll
            for (int m = 0; m < EPT; ++m)
                if (c[m] >= 0) {
                    if constexpr (R % 2 == 0) {
                        const double2 *p2 = reinterpret_cast<const double2 *>(P + (size_t)c[m] * R);
#pragma unroll
                        for (int h2 = 0; h2 < R / 2; ++h2) {
                            const double2 pv = p2[h2];
                            prod[(2 * h2) * E + t + m * kBlock] = v[m] * pv.x;
                            prod[(2 * h2 + 1) * E + t + m * kBlock] = v[m] * pv.y;
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            prod[r * E + t + m * kBlock] = v[m] * P[(size_t)c[m] * R + r];
                    }
                }
            __syncthreads();
            if (t < nr) {
                const int k0 = lptr[t], k1 = lptr[t + 1];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double a = 0.0;
                    for (int k = k0; k < k1; ++k)
                        a += prod[r * E + k];
                    Q[(size_t)(r0 + t) * R + r] = a;
                    sig[r] = fma(P[(size_t)(r0 + t) * R + r], a, sig[r]);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sr = block_sum(sig[r], red);
        if (t == 0)
            sig_part[blockIdx.x * R + r] = sr;
    }
}

// Two-entry vectors for the paired loads of the slices.
template <class T>
struct Pair2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

// Column of a slice entry: as stored (int32_t, -1 = padding) or as the
// 16-bit offset from its row (int16_t, kPad16 = padding).
__device__ __forceinline__ int bcol_of(int32_t raw, int) { return raw; }
__device__ __forceinline__ int bcol_of(int16_t raw, int row) { return raw == kPad16 ? -1 : row + raw; }

// Q = A P for the R interleaved right-hand sides over the sliced layout (the
// third schedule): each system's rows in slices of 64, lane l of a wave owns
// row 64 s + l, and a slice stores its rows' entries pairwise, k-th pair
// first (entries 2j, 2j + 1 of lane l at off + 128 j + 2 l, the last entry of
// an odd width at off + 64 (w - 1) + l; padding: column -1, or kPad16 for
// CT = int16_t, columns stored as offsets from the row when every one is
// within 32767).  The lanes of one load gather neighbouring rows of P for a
// stencil-like matrix, each 8R bytes, so the gathers coalesce.  A row is
// summed left to right from rounded products, the order of the LDS schedule
// (same bits).  Waves of a workgroup take its slices in turn.
template <int R, int U, class CT>
__global__ __launch_bounds__(kBlock) void k_bspmm_slices(const WgDesc *__restrict__ wgs,
                                                         const int32_t *__restrict__ sl_row,
                                                         const int32_t *__restrict__ sl_off,
                                                         const CT *__restrict__ col,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ P, double *__restrict__ Q,
                                                         double *__restrict__ sig_part, Inst *inst)
{
#pragma clang fp contract(off)
    __shared__ double red[kWaves];
    __shared__ int act_s[R];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x;
    bool any = true;
    if (inst != nullptr) {
        if (t < R)
            act_s[t] = inst_gate(&inst[W.sys * R + t], W.lead != 0) ? 1 : 0;
        __syncthreads();
        any = false;
#pragma unroll
        for (int r = 0; r < R; ++r)
            any |= act_s[r] != 0;
    }
    double sig[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        sig[r] = 0.0;
    const int lane = t & 63;
    if (any) {
        for (int sl = W.rb0 + (t >> 6); sl < W.rb1; sl += kWaves) {
            const int e0 = sl_off[sl], L = (sl_off[sl + 1] - e0) / 64;
            const int row = sl_row[sl] + lane;
            double a[R];
#pragma unroll
            for (int r = 0; r < R; ++r)
                a[r] = 0.0;
            for (int k0 = 0; k0 < L; k0 += U) {
                static_assert(U % 2 == 0, "entries come in pairs");
                int c[U];
                double v[U], pv[U][R];
                // one 2-wide load per pair, unconditional: the single last
                // entry of an odd width through the aligned pair holding it
                // (the lane's parity picks the half), past the width positions
                // 0 and 1 (discarded); then the entries are selected
                typename Pair2<CT>::type craw[U / 2];
                typename Pair2<double>::type vraw[U / 2];
#pragma unroll
                for (int u = 0; u < U; u += 2) {
                    const int k = k0 + u;
                    const int e = k + 1 < L ? e0 + (k >> 1) * 128 + 2 * lane : k < L ? e0 + k * 64 + (lane & ~1) : 0;
                    craw[u >> 1] = __builtin_nontemporal_load(reinterpret_cast<const typename Pair2<CT>::type *>(col + e));
                    vraw[u >> 1] =
                        __builtin_nontemporal_load(reinterpret_cast<const typename Pair2<double>::type *>(val + e));
                }
#pragma unroll
                for (int u = 0; u < U; u += 2) {
                    const int k = k0 + u;
                    const bool pair = k + 1 < L, hi = !pair && (lane & 1);
                    c[u] = k < L ? bcol_of(hi ? craw[u >> 1].y : craw[u >> 1].x, row) : -1;
                    c[u + 1] = pair ? bcol_of(craw[u >> 1].y, row) : -1;
                    v[u] = hi ? vraw[u >> 1].y : vraw[u >> 1].x;
                    v[u + 1] = vraw[u >> 1].y;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if constexpr (R % 2 == 0) {
                        const double2 *p2 = reinterpret_cast<const double2 *>(P + (size_t)max(c[u], 0) * R);
#pragma unroll
                        for (int h2 = 0; h2 < R / 2; ++h2) {
                            // unguarded load (row clamped to 0), then a select:
                            // a guarded load would wait inside its branch
                            const double2 q2 = p2[h2];
                            pv[u][2 * h2] = c[u] >= 0 ? q2.x : 0.0;
                            pv[u][2 * h2 + 1] = c[u] >= 0 ? q2.y : 0.0;
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                        {
                            const double q = P[(size_t)max(c[u], 0) * R + r];
                            pv[u][r] = c[u] >= 0 ? q : 0.0;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (c[u] >= 0)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            a[r] = a[r] + v[u] * pv[u][r];
            }
            if (row < W.i1) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    Q[(size_t)row * R + r] = a[r];
                    sig[r] = fma(P[(size_t)row * R + r], a[r], sig[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sr = block_sum(sig[r], red);
        if (t == 0)
            sig_part[blockIdx.x * R + r] = sr;
    }
}

// Per instance r of this workgroup's system: sum of the system's partials
// (fixed order), by thread r.
template <int R>
__device__ __forceinline__ double sys_sum(const double *__restrict__ part, const WgDesc &W, int r)
{
    double s = 0.0;
    for (int w = W.wg0; w < W.wg1; ++w)
        s += part[w * R + r];
    return s;
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_bupdate_r(const WgDesc *__restrict__ wgs, double *__restrict__ Rv,
                                                      const double *__restrict__ Q, Inst *inst,
                                                      const double *__restrict__ sig_part,
                                                      double *__restrict__ rho_part)
{
    __shared__ double red[kWaves];
    __shared__ double sh_alpha[R];
    __shared__ int sh_act[R];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x;
    if (t < R) {
        Inst *I = &inst[W.sys * R + t];
        int a = I->status == kRun;
        double al = 0.0;
        if (a) {
            const double sg = sys_sum<R>(sig_part, W, t);
            if (!(sg > 0.0) || !isfinite(sg)) {
                if (W.lead) {
                    I->iters = I->k;
                    I->sigma = sg;
                    I->status = kBreakdown;
                }
                a = 0;
            } else {
                al = I->rho / sg;
                if (W.lead) {
                    I->alpha = al;
                    I->sigma = sg;
                    I->k = I->k + 1;
                }
            }
        }
        sh_alpha[t] = al;
        sh_act[t] = a;
    }
    __syncthreads();
    const int r = t % R; // the stride is a multiple of R: a thread keeps its instance
    const bool act = sh_act[r] != 0;
    const double al = sh_alpha[r];
    double acc = 0.0;
    if (act) {
        const size_t j1 = (size_t)W.i1 * R;
        for (size_t j = (size_t)W.i0 * R + t; j < j1; j += kBlock) {
            const double rv = fma(-al, Q[j], Rv[j]);
            Rv[j] = rv;
            acc = fma(rv, rv, acc);
        }
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const double s = block_sum(r == rr ? acc : 0.0, red);
        if (t == 0)
            rho_part[blockIdx.x * R + rr] = s;
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_bupdate_xp(const WgDesc *__restrict__ wgs, double *__restrict__ X,
                                                       double *__restrict__ P, const double *__restrict__ Rv,
                                                       Inst *inst, const double *__restrict__ rho_part)
{
    __shared__ double sh_alpha[R], sh_beta[R];
    __shared__ int sh_act[R], sh_conv[R];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x;
    if (t < R) {
        Inst *I = &inst[W.sys * R + t];
        const int a = I->status == kRun;
        double be = 0.0;
        int conv = 0;
        if (a) {
            const double rn = sys_sum<R>(rho_part, W, t);
            be = rn / I->rho;
            conv = sqrt(rn) <= I->tol_nb;
            if (W.lead) {
                I->rho_next = rn;
                I->conv_next = conv;
            }
        }
        sh_alpha[t] = a ? I->alpha : 0.0;
        sh_beta[t] = be;
        sh_act[t] = a;
        sh_conv[t] = conv;
    }
    __syncthreads();
    const int r = t % R;
    if (!sh_act[r])
        return;
    const double al = sh_alpha[r], be = sh_beta[r];
    const bool conv = sh_conv[r] != 0;
    const size_t j1 = (size_t)W.i1 * R;
    for (size_t j = (size_t)W.i0 * R + t; j < j1; j += kBlock) {
        const double pj = P[j];
        X[j] = fma(al, pj, X[j]);
        if (!conv)
            P[j] = fma(be, pj, Rv[j]);
    }
}

// After each graph launch: apply the pending stop decisions and count the
// instances still running (one workgroup).
__global__ __launch_bounds__(kBlock) void k_bcheck(Inst *inst, int ninst, double *running)
{
    __shared__ double red[kWaves];
    double c = 0.0;
    for (int i = threadIdx.x; i < ninst; i += kBlock) {
        Inst *I = &inst[i];
        if (I->status != kRun)
            continue;
        if (I->conv_next) {
            I->rho = I->rho_next;
            I->iters = I->k;
            I->status = kConverged;
        } else if (I->k >= I->maxit) {
            I->rho = I->rho_next;
            I->iters = I->k;
            I->status = kMaxit;
        } else {
            c += 1.0;
        }
    }
    c = block_sum(c, red);
    if (threadIdx.x == 0)
        running[0] = c;
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_binit_vec(const WgDesc *__restrict__ wgs, const double *__restrict__ B,
                                                      const double *__restrict__ X0, const double *__restrict__ Q,
                                                      double *__restrict__ Rv, double *__restrict__ P,
                                                      double *__restrict__ Xw, double *__restrict__ rho_part,
                                                      double *__restrict__ bb_part)
{
    __shared__ double red[kWaves];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x, r = t % R;
    double ar = 0.0, ab = 0.0;
    const size_t j1 = (size_t)W.i1 * R;
    for (size_t j = (size_t)W.i0 * R + t; j < j1; j += kBlock) {
        const double bj = B[j];
        const double rv = bj - Q[j];
        Rv[j] = rv;
        P[j] = rv;
        Xw[j] = X0[j];
        ar = fma(rv, rv, ar);
        ab = fma(bj, bj, ab);
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const double sr = block_sum(r == rr ? ar : 0.0, red);
        const double sb = block_sum(r == rr ? ab : 0.0, red);
        if (t == 0) {
            rho_part[blockIdx.x * R + rr] = sr;
            bb_part[blockIdx.x * R + rr] = sb;
        }
    }
}

// One thread per instance: ||b||, r0'r0, status, tolerance.
template <int R>
__global__ __launch_bounds__(kBlock) void k_binit_state(const WgDesc *__restrict__ wgs,
                                                        const int32_t *__restrict__ sys_wg0, Inst *inst, int ninst,
                                                        const double *__restrict__ rho_part,
                                                        const double *__restrict__ bb_part, double tol, int maxit)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= ninst)
        return;
    const int s = i / R, r = i % R;
    const WgDesc W = wgs[sys_wg0[s]];
    const double nb = sqrt(sys_sum<R>(bb_part, W, r));
    const double rho = sys_sum<R>(rho_part, W, r);
    Inst *I = &inst[i];
    I->k = 0;
    I->iters = 0;
    I->maxit = maxit;
    I->nb = nb;
    I->rho = rho;
    I->alpha = 0.0;
    I->sigma = 0.0;
    I->res_true = 0.0;
    I->tol_nb = tol * nb;
    I->rho_next = rho;
    I->conv_next = sqrt(rho) <= tol * nb ? 1 : 0;
    I->status = !isfinite(nb) ? kNonfinite : (nb == 0.0 ? kZeroRhs : kRun);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_bresid(const WgDesc *__restrict__ wgs, const double *__restrict__ B,
                                                   const double *__restrict__ Q, double *__restrict__ part)
{
    __shared__ double red[kWaves];
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x, r = t % R;
    double a = 0.0;
    const size_t j1 = (size_t)W.i1 * R;
    for (size_t j = (size_t)W.i0 * R + t; j < j1; j += kBlock) {
        const double d = B[j] - Q[j];
        a = fma(d, d, a);
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        const double s = block_sum(r == rr ? a : 0.0, red);
        if (t == 0)
            part[blockIdx.x * R + rr] = s;
    }
}

// Copy out: x of the instance (unless b had a non-finite entry: untouched;
// b == 0: zero), and the true relative residual per instance.
template <int R>
__global__ __launch_bounds__(kBlock) void k_bfinish(const WgDesc *__restrict__ wgs, const int32_t *__restrict__ sys_wg0,
                                                    Inst *inst, const double *__restrict__ part,
                                                    const double *__restrict__ Xw, double *__restrict__ X)
{
    const WgDesc W = wgs[blockIdx.x];
    const int t = threadIdx.x, r = t % R;
    const Inst *I = &inst[W.sys * R + r];
    const int st = I->status;
    const size_t j1 = (size_t)W.i1 * R;
    for (size_t j = (size_t)W.i0 * R + t; j < j1; j += kBlock) {
        if (st == kNonfinite)
            continue;
        X[j] = st == kZeroRhs ? 0.0 : Xw[j];
    }
    if (W.lead && t < R) {
        Inst *Ir = &inst[W.sys * R + t];
        const double s = sys_sum<R>(part, W, t);
        Ir->res_true = Ir->nb > 0.0 ? sqrt(s) / Ir->nb : 0.0;
    }
    (void)sys_wg0;
}

} // namespace

// ------------------------------------------------------------------ host
struct cg_batch {
    int nsys = 0, R = 1;
    int64_t N = 0, nnz = 0;
    std::vector<int64_t> sys_off;
    std::vector<int32_t> hptr, hidx; // host copy of the structure (re-planning by the autotuner)
    // plan: row blocks of 256 * ept entries; lanes = 0 runs the products on
    // them through LDS, lanes = 8 / 16 uses that many lanes per row instead,
    // lanes = 1 runs one lane per row over the sliced layout (the workgroups
    // then own runs of slices instead of row blocks)
    int ept = 4, G = 0, nrb = 0, wg_target = 2048, lanes = 0;
    // sliced layout (built once, on first use): per system, slices of 64 rows
    std::vector<int32_t> hsl_row, hsl_sys0; // first row of each slice; first slice of each system (+ end)
    int32_t *sl_row = nullptr, *sl_off = nullptr, *sl_col = nullptr;
    int16_t *sl_d16 = nullptr; // columns as 16-bit offsets from the row (every one within 32767), else null
    double *sl_val = nullptr;
    // device
    std::vector<void *> allocs, plan_allocs;
    int32_t *ptr = nullptr, *idx = nullptr, *rb_row = nullptr, *sys_wg0 = nullptr;
    double *val = nullptr;
    WgDesc *wgs = nullptr;
    Inst *inst = nullptr;
    double *P = nullptr, *Rv = nullptr, *Q = nullptr, *Xw = nullptr;
    double *sig = nullptr, *rho = nullptr, *bb = nullptr, *running = nullptr;
    double *host_run = nullptr; // pinned [2]
    Inst *host_inst = nullptr;  // pinned [ninst]
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t stream = nullptr, capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int batch = 16, graph_batch = 0;
    std::string err;
};

namespace {

int bfail(cg_batch *h, hipError_t e, const char *what)
{
    h->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CG_ERR_NOMEM : CG_ERR_HIP;
}

template <class T>
int balloc(cg_batch *h, std::vector<void *> &list, T **out, size_t count)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess)
        return bfail(h, e, "hipMalloc");
    list.push_back(p);
    *out = static_cast<T *>(p);
    return CG_OK;
}

template <class T>
int bupload(cg_batch *h, std::vector<void *> &list, T **out, const T *src, size_t count)
{
    int st = balloc(h, list, out, count);
    if (st != CG_OK)
        return st;
    if (count) {
        hipError_t e = hipMemcpy(*out, src, count * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return bfail(h, e, "hipMemcpy");
    }
    return CG_OK;
}

void free_list(std::vector<void *> &l)
{
    for (void *p : l)
        (void)hipFree(p);
    l.clear();
}

void drop_graph(cg_batch *h)
{
    if (h->gexec)
        (void)hipGraphExecDestroy(h->gexec);
    if (h->graph)
        (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->graph_batch = 0;
}

// Row blocks (<= 256*ept entries, <= 256 rows, never across systems) and the
// workgroup split: system s gets max(1, round(wg_target * nnz_s / nnz))
// workgroups (at most one per row block), each a contiguous run of its row
// blocks.  Returns the partial-array size needed (G * R).
int build_plan(cg_batch *h, int ept, int wg_target)
{
    const int E = kBlock * ept;
    std::vector<int32_t> rb;
    std::vector<int32_t> sys_rb0(h->nsys + 1, 0);
    const int32_t *ptr = h->hptr.data();
    for (int s = 0; s < h->nsys; ++s) {
        sys_rb0[s] = (int32_t)rb.size();
        const int64_t a = h->sys_off[s], b = h->sys_off[s + 1];
        int64_t r0 = a;
        rb.push_back((int32_t)a);
        for (int64_t r = a; r < b; ++r) {
            const int64_t len = (int64_t)ptr[r + 1] - ptr[r];
            if (r > r0 && ((int64_t)ptr[r + 1] - ptr[r0] > E || r - r0 >= kStreamRows || len > E)) {
                rb.push_back((int32_t)r);
                r0 = r;
            }
            if (len > E) {
                rb.push_back((int32_t)(r + 1));
                r0 = r + 1;
            }
        }
        if (rb.back() == b) // the system ended on a long row
            rb.pop_back();
    }
    sys_rb0[h->nsys] = (int32_t)rb.size();
    rb.push_back((int32_t)h->N);
    std::vector<WgDesc> w;
    std::vector<int32_t> wg0(h->nsys);
    for (int s = 0; s < h->nsys; ++s) {
        const int nrbs = sys_rb0[s + 1] - sys_rb0[s];
        const int64_t nnzs = (int64_t)ptr[h->sys_off[s + 1]] - ptr[h->sys_off[s]];
        int g = (int)std::llround((double)wg_target * (double)nnzs / (double)std::max<int64_t>(h->nnz, 1));
        g = std::max(1, std::min(g, nrbs));
        wg0[s] = (int32_t)w.size();
        for (int k = 0; k < g; ++k) {
            WgDesc d{};
            d.sys = s;
            d.lead = k == 0;
            d.rb0 = sys_rb0[s] + (int)((int64_t)k * nrbs / g);
            d.rb1 = sys_rb0[s] + (int)((int64_t)(k + 1) * nrbs / g);
            d.i0 = rb[d.rb0];
            d.i1 = rb[d.rb1];
            w.push_back(d);
        }
    }
    for (auto &d : w) {
        d.wg0 = wg0[d.sys];
        d.wg1 = d.sys + 1 < h->nsys ? wg0[d.sys + 1] : (int32_t)w.size();
    }
    drop_graph(h);
    free_list(h->plan_allocs);
    int st;
    const size_t np = w.size() * (size_t)h->R;
    if ((st = bupload(h, h->plan_allocs, &h->rb_row, rb.data(), rb.size())) != CG_OK ||
        (st = bupload(h, h->plan_allocs, &h->wgs, w.data(), w.size())) != CG_OK ||
        (st = bupload(h, h->plan_allocs, &h->sys_wg0, wg0.data(), wg0.size())) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->sig, np)) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->rho, np)) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->bb, np)) != CG_OK)
        return st;
    h->G = (int)w.size();
    h->nrb = (int)rb.size() - 1;
    h->ept = ept;
    h->wg_target = wg_target;
    return CG_OK;
}

// The sliced layout of the block-diagonal matrix, once: each system's rows
// in slices of 64 (the last one of a system may be short), entries paired as
// in k_bspmm_slices (slice_position), padded with column -1 / value 0.
int ensure_slices(cg_batch *h)
{
    if (h->sl_col || h->sl_d16)
        return CG_OK;
    const int32_t *ptr = h->hptr.data(), *idx = h->hidx.data();
    std::vector<int32_t> row0, off(1, 0), sys0(h->nsys + 1, 0);
    for (int s = 0; s < h->nsys; ++s) {
        sys0[s] = (int32_t)row0.size();
        const int64_t a = h->sys_off[s], b = h->sys_off[s + 1];
        for (int64_t r = a; r < b; r += 64) {
            int64_t L = 0;
            for (int64_t i = r; i < std::min(b, r + 64); ++i)
                L = std::max<int64_t>(L, (int64_t)ptr[i + 1] - ptr[i]);
            if ((int64_t)off.back() + 64 * L > INT32_MAX) {
                h->err = "sliced layout too large for 32-bit positions";
                return CG_ERR_UNSUPPORTED;
            }
            row0.push_back((int32_t)r);
            off.push_back(off.back() + (int32_t)(64 * L));
        }
    }
    sys0[h->nsys] = (int32_t)row0.size();
    const size_t npos = (size_t)off.back();
    std::vector<int32_t> col(npos, -1), src(npos, -1);
    std::vector<int16_t> d16(npos, kPad16);
    bool c16 = true; // every column within 32767 of its row (experiments: CGMI_COL16=0, never)
    if (const char *e = std::getenv("CGMI_COL16"))
        c16 = std::strcmp(e, "0") != 0;
    for (int s = 0; s < h->nsys; ++s) {
        const int64_t b = h->sys_off[s + 1];
        for (int32_t q = sys0[s]; q < sys0[s + 1]; ++q) {
            const int64_t w = (off[q + 1] - off[q]) / 64;
            for (int64_t i = row0[q]; i < std::min<int64_t>(b, (int64_t)row0[q] + 64); ++i)
                for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
                    const int64_t e = off[q] + slice_position(k - ptr[i], i - row0[q], w);
                    col[e] = idx[k];
                    src[e] = (int32_t)k;
                    const int64_t d = (int64_t)idx[k] - i;
                    c16 = c16 && d >= -32767 && d <= 32767;
                    d16[e] = (int16_t)d;
                }
        }
    }
    // values: gathered on the device from the CSR copy through src
    std::vector<void *> tmp;
    int32_t *dsrc = nullptr;
    int st;
    if ((st = bupload(h, h->allocs, &h->sl_row, row0.data(), row0.size())) != CG_OK ||
        (st = bupload(h, h->allocs, &h->sl_off, off.data(), off.size())) != CG_OK ||
        (c16 ? (st = bupload(h, h->allocs, &h->sl_d16, d16.data(), d16.size()))
             : (st = bupload(h, h->allocs, &h->sl_col, col.data(), col.size()))) != CG_OK ||
        (st = balloc(h, h->allocs, &h->sl_val, npos)) != CG_OK || (st = bupload(h, tmp, &dsrc, src.data(), npos)) != CG_OK) {
        free_list(tmp);
        return st;
    }
    launch_permute((int64_t)npos, h->val, dsrc, h->sl_val, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    free_list(tmp);
    if (e != hipSuccess)
        return bfail(h, e, "sliced values");
    h->hsl_row.swap(row0);
    h->hsl_sys0.swap(sys0);
    return CG_OK;
}

// Workgroup split over the slices: system s gets max(1, round(wg_target *
// nnz_s / nnz)) workgroups (at most one per slice), each a contiguous run of
// its slices.
int build_plan_slices(cg_batch *h, int wg_target)
{
    int st = ensure_slices(h);
    if (st != CG_OK)
        return st;
    const int32_t *ptr = h->hptr.data();
    std::vector<WgDesc> w;
    std::vector<int32_t> wg0(h->nsys);
    for (int s = 0; s < h->nsys; ++s) {
        const int q0 = h->hsl_sys0[s], nq = h->hsl_sys0[s + 1] - q0;
        const int64_t nnzs = (int64_t)ptr[h->sys_off[s + 1]] - ptr[h->sys_off[s]];
        int g = (int)std::llround((double)wg_target * (double)nnzs / (double)std::max<int64_t>(h->nnz, 1));
        g = std::max(1, std::min(g, nq));
        wg0[s] = (int32_t)w.size();
        for (int k = 0; k < g; ++k) {
            WgDesc d{};
            d.sys = s;
            d.lead = k == 0;
            d.rb0 = q0 + (int)((int64_t)k * nq / g);
            d.rb1 = q0 + (int)((int64_t)(k + 1) * nq / g);
            d.i0 = h->hsl_row[d.rb0];
            d.i1 = d.rb1 < q0 + nq ? h->hsl_row[d.rb1] : (int32_t)h->sys_off[s + 1];
            w.push_back(d);
        }
    }
    for (auto &d : w) {
        d.wg0 = wg0[d.sys];
        d.wg1 = d.sys + 1 < h->nsys ? wg0[d.sys + 1] : (int32_t)w.size();
    }
    drop_graph(h);
    free_list(h->plan_allocs);
    const size_t np = w.size() * (size_t)h->R;
    if ((st = bupload(h, h->plan_allocs, &h->wgs, w.data(), w.size())) != CG_OK ||
        (st = bupload(h, h->plan_allocs, &h->sys_wg0, wg0.data(), wg0.size())) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->sig, np)) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->rho, np)) != CG_OK ||
        (st = balloc(h, h->plan_allocs, &h->bb, np)) != CG_OK)
        return st;
    h->rb_row = nullptr;
    h->G = (int)w.size();
    h->nrb = 0;
    h->wg_target = wg_target;
    h->lanes = 1;
    return CG_OK;
}

template <int R, int EPT>
void spmm_r(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    hipLaunchKernelGGL((k_bspmm<R, EPT>), dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->rb_row, h->ptr, h->idx, h->val,
                       P, Q, h->sig, inst);
}

template <int R>
void spmm_e(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    // LDS holds 256 * EPT * R products (<= 32 KB)
    if (h->ept == 1)
        spmm_r<R, 1>(h, P, Q, inst, s);
    else if (h->ept == 2)
        spmm_r<R, 2>(h, P, Q, inst, s);
    else
        spmm_r<R, 4>(h, P, Q, inst, s);
}

template <int R>
void spmm_lanes(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    constexpr int U = R == 4 ? 1 : 2; // rows in flight per lane group (registers: 8 waves per SIMD)
    if (h->lanes == 8)
        hipLaunchKernelGGL((k_bspmm_lanes<R, 8, U>), dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->ptr, h->idx, h->val,
                           P, Q, h->sig, inst);
    else
        hipLaunchKernelGGL((k_bspmm_lanes<R, 16, U>), dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->ptr, h->idx,
                           h->val, P, Q, h->sig, inst);
}

template <int R>
void spmm_slices(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    constexpr int U = 8; // positions per round
    if (h->sl_d16)
        hipLaunchKernelGGL((k_bspmm_slices<R, U, int16_t>), dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->sl_row,
                           h->sl_off, h->sl_d16, h->sl_val, P, Q, h->sig, inst);
    else
        hipLaunchKernelGGL((k_bspmm_slices<R, U, int32_t>), dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->sl_row,
                           h->sl_off, h->sl_col, h->sl_val, P, Q, h->sig, inst);
}

// the product of the current plan and schedule
template <int R>
void spmm_any(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    if (h->lanes == 1)
        spmm_slices<R>(h, P, Q, inst, s);
    else if (h->lanes)
        spmm_lanes<R>(h, P, Q, inst, s);
    else
        spmm_e<R>(h, P, Q, inst, s);
}

void spmm(cg_batch *h, const double *P, double *Q, Inst *inst, hipStream_t s)
{
    if (h->lanes == 1) {
        if (h->R == 1)
            spmm_slices<1>(h, P, Q, inst, s);
        else if (h->R == 2)
            spmm_slices<2>(h, P, Q, inst, s);
        else
            spmm_slices<4>(h, P, Q, inst, s);
        return;
    }
    if (h->lanes) {
        if (h->R == 1)
            spmm_lanes<1>(h, P, Q, inst, s);
        else if (h->R == 2)
            spmm_lanes<2>(h, P, Q, inst, s);
        else
            spmm_lanes<4>(h, P, Q, inst, s);
        return;
    }
    if (h->R == 1)
        spmm_e<1>(h, P, Q, inst, s);
    else if (h->R == 2)
        spmm_e<2>(h, P, Q, inst, s);
    else
        spmm_e<4>(h, P, Q, inst, s);
}

template <int R>
void iteration_r(cg_batch *h, hipStream_t s)
{
    spmm_any<R>(h, h->P, h->Q, h->inst, s);
    hipLaunchKernelGGL(k_bupdate_r<R>, dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->Rv, h->Q, h->inst, h->sig, h->rho);
    hipLaunchKernelGGL(k_bupdate_xp<R>, dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->Xw, h->P, h->Rv, h->inst, h->rho);
}

void iteration(cg_batch *h, hipStream_t s)
{
    if (h->R == 1)
        iteration_r<1>(h, s);
    else if (h->R == 2)
        iteration_r<2>(h, s);
    else
        iteration_r<4>(h, s);
}

template <int R>
void init_r(cg_batch *h, const double *B, const double *X0, double tol, int maxit, hipStream_t s)
{
    const int ninst = h->nsys * R;
    spmm_any<R>(h, X0, h->Q, nullptr, s);
    hipLaunchKernelGGL(k_binit_vec<R>, dim3(h->G), dim3(kBlock), 0, s, h->wgs, B, X0, h->Q, h->Rv, h->P, h->Xw,
                       h->rho, h->bb);
    hipLaunchKernelGGL(k_binit_state<R>, dim3((ninst + kBlock - 1) / kBlock), dim3(kBlock), 0, s, h->wgs,
                       h->sys_wg0, h->inst, ninst, h->rho, h->bb, tol, maxit);
}

template <int R>
void finish_r(cg_batch *h, const double *B, double *X, hipStream_t s)
{
    spmm_any<R>(h, h->Xw, h->Q, nullptr, s);
    hipLaunchKernelGGL(k_bresid<R>, dim3(h->G), dim3(kBlock), 0, s, h->wgs, B, h->Q, h->bb);
    hipLaunchKernelGGL(k_bfinish<R>, dim3(h->G), dim3(kBlock), 0, s, h->wgs, h->sys_wg0, h->inst, h->bb, h->Xw, X);
}

int build_graph(cg_batch *h)
{
    if (h->gexec && h->graph_batch == h->batch)
        return CG_OK;
    drop_graph(h);
    hipError_t e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return bfail(h, e, "hipStreamBeginCapture");
    for (int i = 0; i < h->batch; ++i)
        iteration(h, h->capture);
    hipLaunchKernelGGL(k_bcheck, dim3(1), dim3(kBlock), 0, h->capture, h->inst, h->nsys * h->R, h->running);
    if ((e = hipStreamEndCapture(h->capture, &h->graph)) != hipSuccess)
        return bfail(h, e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bfail(h, e, "hipGraphInstantiate");
    h->graph_batch = h->batch;
    return CG_OK;
}

void release(cg_batch *h)
{
    drop_graph(h);
    for (auto &e : h->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (h->host_run)
        (void)hipHostFree(h->host_run);
    if (h->host_inst)
        (void)hipHostFree(h->host_inst);
    free_list(h->plan_allocs);
    free_list(h->allocs);
    if (h->capture)
        (void)hipStreamDestroy(h->capture);
}

thread_local std::string g_berr;

} // namespace

extern "C" {

int cg_batch_create(cg_batch **out, int32_t nsys, const int64_t *sys_off, const int32_t *ptr, const int32_t *idx,
                    const double *vals, int32_t nrhs, int index_base)
{
    if (!out) {
        g_berr = "out is NULL";
        return CG_ERR_ARG;
    }
    *out = nullptr;
    std::unique_ptr<cg_batch> h;
    try {
        h.reset(new cg_batch());
        if (nsys < 1 || !sys_off || (nrhs != 1 && nrhs != 2 && nrhs != 4) || (index_base != 0 && index_base != 1)) {
            g_berr = "need nsys >= 1, sys_off, nrhs in {1, 2, 4}, index_base 0 or 1";
            return CG_ERR_ARG;
        }
        if (sys_off[0] != 0) {
            g_berr = "sys_off[0] must be 0";
            return CG_ERR_STRUCTURE;
        }
        for (int s = 0; s < nsys; ++s)
            if (sys_off[s + 1] <= sys_off[s]) {
                g_berr = "every system needs at least one row (sys_off increasing)";
                return CG_ERR_STRUCTURE;
            }
        const int64_t N = sys_off[nsys];
        std::vector<int32_t> p0, i0;
        std::string err;
        int st = validate_and_normalise(kCsr, N, ptr, idx, vals, index_base, 0, p0, i0, err);
        if (st != CG_OK) {
            g_berr = err;
            return st;
        }
        // block-diagonal: the columns of a row stay inside its system
        for (int s = 0; s < nsys; ++s)
            for (int64_t r = sys_off[s]; r < sys_off[s + 1]; ++r)
                for (int64_t k = p0[r]; k < p0[r + 1]; ++k)
                    if (i0[k] < sys_off[s] || i0[k] >= sys_off[s + 1]) {
                        g_berr = "row " + std::to_string(r) + " couples to another system";
                        return CG_ERR_STRUCTURE;
                    }
        if (N > 0 && p0[N] > 0 && !vals) {
            g_berr = "vals is NULL";
            return CG_ERR_ARG;
        }
        h->nsys = nsys;
        h->R = nrhs;
        h->N = N;
        h->nnz = p0[N];
        h->sys_off.assign(sys_off, sys_off + nsys + 1);
        const size_t nv = (size_t)N * nrhs;
        if ((st = bupload(h.get(), h->allocs, &h->ptr, p0.data(), p0.size())) != CG_OK ||
            (st = bupload(h.get(), h->allocs, &h->idx, i0.data(), i0.size())) != CG_OK ||
            (st = bupload(h.get(), h->allocs, &h->val, vals, i0.size())) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->inst, (size_t)nsys * nrhs)) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->P, nv)) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->Rv, nv)) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->Q, nv)) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->Xw, nv)) != CG_OK ||
            (st = balloc(h.get(), h->allocs, &h->running, 1)) != CG_OK) {
            g_berr = h->err;
            release(h.get());
            return st;
        }
        h->hptr.swap(p0);
        h->hidx.swap(i0);
        hipError_t e = hipHostMalloc((void **)&h->host_run, 2 * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&h->host_inst, (size_t)nsys * nrhs * sizeof(Inst), hipHostMallocDefault);
        for (auto &ev : h->ev)
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            st = bfail(h.get(), e, "host resources");
            g_berr = h->err;
            release(h.get());
            return st;
        }
        if ((st = build_plan(h.get(), 4, 2048)) != CG_OK) {
            g_berr = h->err;
            release(h.get());
            return st;
        }
        // schedule override (tests, experiments): CGMI_BATCH_LANES=8 or 16
        // (lanes per row), 1 (the sliced layout)
        if (const char *ev = std::getenv("CGMI_BATCH_LANES")) {
            const int l = std::atoi(ev);
            if (l == 1)
                st = build_plan_slices(h.get(), 4096);
            else
                h->lanes = (l == 8 || l == 16) ? l : 0;
            if (st != CG_OK) {
                g_berr = h->err;
                release(h.get());
                return st;
            }
        }
    } catch (const std::bad_alloc &) {
        g_berr = "host allocation failed";
        if (h)
            release(h.get());
        return CG_ERR_NOMEM;
    }
    g_berr.clear();
    *out = h.release();
    return CG_OK;
}

int cg_batch_set_stream(cg_batch *h, void *hip_stream)
{
    if (!h)
        return CG_ERR_ARG;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return CG_OK;
}

int cg_batch_spmm(cg_batch *h, const double *X, double *Y)
{
    if (!h || !X || !Y || X == Y)
        return CG_ERR_ARG;
    spmm(h, X, Y, nullptr, h->stream);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CG_OK : bfail(h, e, "launch");
}

int cg_batch_autotune(cg_batch *h, int32_t *entries_per_block, int32_t *lanes_per_row, int32_t *workgroups,
                      float *best_us)
{
    if (!h)
        return CG_ERR_ARG;
    // candidates: schedule (row blocks of 256 / 512 / 1024 entries through
    // LDS, or 8 / 16 lanes per row) x workgroup budget; each timed on 10
    // products of a fixed vector after one warm-up
    struct Cand {
        int ept, lanes; // lanes = 1: the sliced layout (ept unused)
    };
    const Cand cands[6] = {{1, 0}, {2, 0}, {4, 0}, {4, 8}, {4, 16}, {0, 1}};
    const int wgt_all[3] = {1024, 2048, 4096};
    const size_t nv = (size_t)h->N * h->R;
    double *X = nullptr, *Y = nullptr;
    hipError_t e = hipMalloc(&X, nv * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(&Y, nv * sizeof(double));
    if (e == hipSuccess)
        e = hipMemsetAsync(X, 0, nv * sizeof(double), h->stream);
    if (e != hipSuccess) {
        (void)hipFree(X);
        return bfail(h, e, "autotune buffers");
    }
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    float best = 1e30f;
    int best_e = h->ept, best_l = h->lanes, best_w = h->wg_target, st = CG_OK;
    for (const Cand &cd : cands) {
        for (int wgt : wgt_all) {
            if ((st = cd.lanes == 1 ? build_plan_slices(h, 2 * wgt) : build_plan(h, cd.ept, wgt)) != CG_OK)
                break;
            h->lanes = cd.lanes;
            spmm(h, X, Y, nullptr, h->stream);
            (void)hipEventRecord(a, h->stream);
            for (int i = 0; i < 10; ++i)
                spmm(h, X, Y, nullptr, h->stream);
            (void)hipEventRecord(b, h->stream);
            (void)hipEventSynchronize(b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) {
                best = ms;
                best_e = cd.ept;
                best_l = cd.lanes;
                best_w = cd.lanes == 1 ? 2 * wgt : wgt;
            }
        }
        if (st != CG_OK)
            break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(X);
    (void)hipFree(Y);
    if (st == CG_OK)
        st = best_l == 1 ? build_plan_slices(h, best_w) : build_plan(h, best_e, best_w);
    h->lanes = best_l;
    if (entries_per_block)
        *entries_per_block = best_l == 1 ? 0 : kBlock * h->ept;
    if (lanes_per_row)
        *lanes_per_row = h->lanes;
    if (workgroups)
        *workgroups = h->G;
    if (best_us)
        *best_us = best * 1e3f / 10.f;
    return st;
}

int cg_batch_solve(cg_batch *h, const double *B, double *X, double tol, int32_t maxit, int32_t *iters,
                   int32_t *status, cg_info *info)
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
    if (!h || !B || !X || B == X || !(tol >= 0.0) || maxit < 0)
        return done(CG_ERR_ARG);
    hipStream_t s = h->stream;
    int st = build_graph(h);
    if (st != CG_OK)
        return done(st);
    if (h->R == 1)
        init_r<1>(h, B, X, tol, maxit, s);
    else if (h->R == 2)
        init_r<2>(h, B, X, tol, maxit, s);
    else
        init_r<4>(h, B, X, tol, maxit, s);
    hipError_t e;
    auto launch = [&](int slot) -> hipError_t {
        hipError_t r = hipGraphLaunch(h->gexec, s);
        if (r == hipSuccess)
            r = hipMemcpyAsync(&h->host_run[slot], h->running, sizeof(double), hipMemcpyDeviceToHost, s);
        if (r == hipSuccess)
            r = hipEventRecord(h->ev[slot], s);
        return r;
    };
    if ((e = launch(0)) != hipSuccess)
        return done(bfail(h, e, "hipGraphLaunch"));
    for (int i = 0;; ++i) {
        if ((e = launch((i + 1) & 1)) != hipSuccess)
            return done(bfail(h, e, "hipGraphLaunch"));
        if ((e = hipEventSynchronize(h->ev[i & 1])) != hipSuccess)
            return done(bfail(h, e, "hipEventSynchronize"));
        if (h->host_run[i & 1] == 0.0)
            break;
    }
    if (h->R == 1)
        finish_r<1>(h, B, X, s);
    else if (h->R == 2)
        finish_r<2>(h, B, X, s);
    else
        finish_r<4>(h, B, X, s);
    const int ninst = h->nsys * h->R;
    if ((e = hipMemcpyAsync(h->host_inst, h->inst, (size_t)ninst * sizeof(Inst), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(bfail(h, e, "state readback"));
    int worst = CG_OK, maxits = 0;
    double worst_rel = 0.0, worst_true = 0.0;
    for (int i = 0; i < ninst; ++i) {
        const Inst &I = h->host_inst[i];
        int code;
        switch (I.status) {
        case kConverged:
        case kZeroRhs: code = CG_OK; break;
        case kMaxit: code = CG_NOT_CONVERGED; break;
        case kBreakdown: code = CG_ERR_BREAKDOWN; break;
        case kNonfinite: code = CG_ERR_NONFINITE; break;
        default: code = CG_ERR_HIP; break;
        }
        if (iters)
            iters[i] = I.iters;
        if (status)
            status[i] = code;
        if (code < 0 ? (worst >= 0 || code < worst) : (worst >= 0 && code > worst))
            worst = code;
        maxits = std::max(maxits, I.iters);
        if (I.nb > 0.0)
            worst_rel = std::max(worst_rel, std::sqrt(I.rho) / I.nb);
        worst_true = std::max(worst_true, I.res_true);
    }
    info->iters = maxits;
    info->relres = worst_rel;
    info->relres_true = worst_true;
    return done(worst);
}

void cg_batch_destroy(cg_batch *h)
{
    if (!h)
        return;
    (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
}

const char *cg_batch_last_error(const cg_batch *h)
{
    return h ? h->err.c_str() : g_berr.c_str();
}

} // extern "C"

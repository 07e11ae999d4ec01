// Device helpers shared by the kernel files: XCD-aware workgroup order and
// deterministic (fixed-tree) reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace cgmi {
namespace dev {

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

// x[c] for c >= 0, else 0.  FP32 x: the load is unguarded (index clamped to
// 0; x holds at least one element) and the value selected, since a guarded
// load takes its conversion to FP64 into the branch and waits there,
// serialising the gathers of a round.  FP64 x: a guarded load (nothing to
// convert; the unguarded form costs address registers and occupancy).
template <class PT>
__device__ __forceinline__ PT gather0(const PT *__restrict__ x, int c)
{
    if constexpr (sizeof(PT) == 4) {
        const PT v = x[c < 0 ? 0 : c];
        return c >= 0 ? v : PT(0);
    } else {
        return c >= 0 ? x[c] : PT(0);
    }
}

template <int W>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, W);
    return v; // butterfly: every lane of the group holds the same bits
}

// Sum over a workgroup of TB threads (red: TB / 64 entries); every thread
// returns the same bits.  Waves are added in index order, so waves whose
// threads all hold +0.0 leave the bits of the sum over the others unchanged.
template <int TB>
__device__ __forceinline__ double block_sum_n(double v, double *red)
{
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = red[0];
#pragma unroll
    for (int w = 1; w < TB / 64; ++w)
        t += red[w];
    return t;
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

// Partials (m <= N * kBlock) in two steps, so that their loads can be
// issued before a kernel's own loads and summed while those are in flight:
// partials_load, then partials_sum, which adds them in the order of
// reduce_partials (same bits).
constexpr int kPartPerThread = (kMaxSpmvBlocks + kBlock - 1) / kBlock;
static_assert(kMaxVecBlocks <= kMaxSpmvBlocks, "vector partials fit the same registers");

template <int N>
__device__ __forceinline__ void partials_load(const double *__restrict__ part, int m, double (&pv)[N])
{
    // unguarded loads (index clamped to m - 1, m >= 1) and a select: a
    // guarded load would take the first add of the sum into its branch and
    // wait there before the next load is issued
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int i = threadIdx.x + j * kBlock;
        const double v = part[min(i, m - 1)];
        pv[j] = i < m ? v : 0.0;
    }
}

template <int N>
__device__ __forceinline__ double partials_sum(const double (&pv)[N], int m, double *red)
{
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j)
        if ((int)threadIdx.x + j * kBlock < m)
            s += pv[j];
    return block_sum(s, red);
}

// Sum of m per-workgroup partials, identical in every workgroup.
__device__ __forceinline__ double reduce_partials(const double *__restrict__ part, int m, double *red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += kBlock)
        s += part[i];
    return block_sum(s, red);
}

} // namespace dev
} // namespace cgmi

// Finite-element operator of the solve: linear (P1) tetrahedra with one
// coefficient nu_e (reluctivity) per element,
//
//     A(nu) = sum_e nu_e K_e,   K_e[a][b] = |T_e| grad(phi_a) . grad(phi_b),
//
// restricted to the unknowns (vertices on the Dirichlet boundary carry no
// row).  This is the kind of matrix the paper solves (abstract, section I:
// finite-element discretisations of Maxwell's equations for electrical
// machines; section III: the SPD system A x = b).  Two device operations make
// the solve differentiable in nu:
//   * assembly  vals = A(nu) on the operator's full-CSR pattern;
//   * gradient  dL/dnu_e = -lam_e' K_e x_e, for the solution x and the
//     adjoint lam = A^-1 dL/dx, both from the same CG.
//
// Layout (device): per element the dof of its 4 vertices (int32 x 4) and the
// 10 distinct entries of K_e stored by entry (entry p of every element
// contiguous, so element kernels read them coalesced); per stored entry of A
// the list of element contributions (element << 4 | entry), in ascending
// element order, so every assembled value is summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/cgmi.h"
#include "plan.h"

using cgmi::kBlock;

namespace {

// index of the distinct entry (a, b), a <= b, of a symmetric 4x4 matrix
__host__ __device__ constexpr int pair_index(int a, int b)
{
    return a <= b ? a * 4 - a * (a - 1) / 2 + (b - a) : b * 4 - b * (b - 1) / 2 + (a - b);
}

struct Vec3 {
    double x, y, z;
};

__device__ __forceinline__ Vec3 sub(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Vec3 cross(Vec3 a, Vec3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dotp(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// K_e from the vertices.  With edges e_r = P_r - P_0 (r = 1..3) the
// barycentric gradients are grad(phi_r) = c_r / det, c_1 = e_2 x e_3,
// c_2 = e_3 x e_1, c_3 = e_1 x e_2, det = e_1 . c_1, and
// grad(phi_0) = -(sum of the others); |T| = |det| / 6, hence
// K[a][b] = c_a . c_b / (6 |det|).  A degenerate or non-finite element
// raises *bad.
__global__ __launch_bounds__(kBlock) void k_fem_khat(int64_t nelem, const double *__restrict__ coords,
                                                     const int32_t *__restrict__ tets, double *__restrict__ khat,
                                                     int32_t *__restrict__ bad)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nelem)
        return;
    Vec3 P[4];
    for (int a = 0; a < 4; ++a) {
        const int64_t v = tets[4 * e + a];
        P[a] = {coords[3 * v], coords[3 * v + 1], coords[3 * v + 2]};
    }
    const Vec3 e1 = sub(P[1], P[0]), e2 = sub(P[2], P[0]), e3 = sub(P[3], P[0]);
    Vec3 c[4];
    c[1] = cross(e2, e3);
    c[2] = cross(e3, e1);
    c[3] = cross(e1, e2);
    c[0] = {-(c[1].x + c[2].x + c[3].x), -(c[1].y + c[2].y + c[3].y), -(c[1].z + c[2].z + c[3].z)};
    const double det = dotp(e1, c[1]);
    const double w = 1.0 / (6.0 * fabs(det));
    if (!(fabs(det) > 0.0) || !isfinite(w))
        *bad = 1;
    for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b)
            khat[(int64_t)pair_index(a, b) * nelem + e] = dotp(c[a], c[b]) * w;
}

// vals[k] = sum over the contributions of entry k of nu_e K_e[p], in list order.
__global__ __launch_bounds__(kBlock) void k_fem_assemble(int64_t nnz, int64_t nelem,
                                                         const int32_t *__restrict__ cptr,
                                                         const int32_t *__restrict__ cq,
                                                         const double *__restrict__ khat,
                                                         const double *__restrict__ nu, double *__restrict__ vals)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnz)
        return;
    double s = 0.0;
    for (int c = cptr[k]; c < cptr[k + 1]; ++c) {
        const int32_t q = cq[c];
        const int64_t e = q >> 4;
        s += nu[e] * khat[(int64_t)(q & 15) * nelem + e];
    }
    vals[k] = s;
}

// grad_e = -lam_e' K_e x_e (vertex values 0 on the Dirichlet boundary).
__global__ __launch_bounds__(kBlock) void k_fem_nu_grad(int64_t nelem, const int4 *__restrict__ edof,
                                                        const double *__restrict__ khat,
                                                        const double *__restrict__ lam,
                                                        const double *__restrict__ x, double *__restrict__ grad)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nelem)
        return;
    const int4 d4 = edof[e];
    const int d[4] = {d4.x, d4.y, d4.z, d4.w};
    double l[4], v[4];
    for (int a = 0; a < 4; ++a) {
        l[a] = d[a] >= 0 ? lam[d[a]] : 0.0;
        v[a] = d[a] >= 0 ? x[d[a]] : 0.0;
    }
    double s = 0.0;
    for (int a = 0; a < 4; ++a) {
        s += khat[(int64_t)pair_index(a, a) * nelem + e] * (l[a] * v[a]);
        for (int b = a + 1; b < 4; ++b)
            s += khat[(int64_t)pair_index(a, b) * nelem + e] * (l[a] * v[b] + l[b] * v[a]);
    }
    grad[e] = -s;
}

} // namespace

struct cg_fem {
    int64_t npts = 0, nelem = 0, n = 0, nnz = 0, ncontrib = 0;
    std::vector<int32_t> rowptr, col; // host copy of the pattern
    int32_t *edof = nullptr;
    double *khat = nullptr;
    int32_t *cptr = nullptr, *cq = nullptr;
    std::vector<void *> allocs;
    hipStream_t stream = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_fem_err;

int fem_hip_fail(cg_fem *f, hipError_t e, const char *what)
{
    f->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CG_ERR_NOMEM : CG_ERR_HIP;
}

template <class T>
int fem_alloc(cg_fem *f, T **out, size_t count)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess)
        return fem_hip_fail(f, e, "hipMalloc");
    f->allocs.push_back(p);
    *out = static_cast<T *>(p);
    return CG_OK;
}

template <class T>
int fem_upload(cg_fem *f, T **out, const T *src, size_t count)
{
    int st = fem_alloc(f, out, count);
    if (st == CG_OK && count) {
        hipError_t e = hipMemcpy(*out, src, count * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return fem_hip_fail(f, e, "hipMemcpy");
    }
    return st;
}

void fem_release(cg_fem *f)
{
    for (void *p : f->allocs)
        (void)hipFree(p);
    f->allocs.clear();
}

// Host planning: element dofs, the pattern (pairs of unknowns sharing an
// element, columns sorted) and the contribution lists.
int fem_plan(cg_fem *f, const double *coords, const int32_t *tets, const int32_t *dof, std::vector<int32_t> &edof,
             std::vector<int32_t> &cptr, std::vector<int32_t> &cq)
{
    const int64_t npts = f->npts, nelem = f->nelem, n = f->n;
    for (int64_t i = 0; i < 3 * npts; ++i)
        if (!std::isfinite(coords[i])) {
            f->err = "coordinate " + std::to_string(i) + " is not finite";
            return CG_ERR_NONFINITE;
        }
    for (int64_t i = 0; i < npts; ++i)
        if (dof[i] < -1 || dof[i] >= n) {
            f->err = "dof[" + std::to_string(i) + "] outside [-1, n)";
            return CG_ERR_ARG;
        }
    edof.resize((size_t)(4 * nelem));
    for (int64_t i = 0; i < 4 * nelem; ++i) {
        if (tets[i] < 0 || tets[i] >= npts) {
            f->err = "tets[" + std::to_string(i) + "] outside [0, npts)";
            return CG_ERR_ARG;
        }
        edof[i] = dof[tets[i]];
    }
    // candidate columns per row (with repeats), then sorted and made unique
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t e = 0; e < nelem; ++e) {
        int live = 0;
        for (int a = 0; a < 4; ++a)
            live += edof[4 * e + a] >= 0;
        for (int a = 0; a < 4; ++a)
            if (edof[4 * e + a] >= 0)
                cnt[edof[4 * e + a] + 1] += live;
    }
    for (int64_t i = 0; i < n; ++i)
        cnt[i + 1] += cnt[i];
    std::vector<int32_t> cand((size_t)cnt[n]);
    {
        std::vector<int64_t> next(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < nelem; ++e)
            for (int a = 0; a < 4; ++a) {
                const int32_t i = edof[4 * e + a];
                if (i < 0)
                    continue;
                for (int b = 0; b < 4; ++b)
                    if (edof[4 * e + b] >= 0)
                        cand[next[i]++] = edof[4 * e + b];
            }
    }
    f->rowptr.assign((size_t)n + 1, 0);
    f->col.clear();
    f->col.reserve((size_t)cnt[n] / 4 + 1);
    for (int64_t i = 0; i < n; ++i) {
        auto b = cand.begin() + cnt[i], e = cand.begin() + cnt[i + 1];
        std::sort(b, e);
        const auto u = std::unique(b, e);
        if ((int64_t)f->col.size() + (u - b) >= (int64_t)INT32_MAX) {
            f->err = "pattern has 2^31 or more entries";
            return CG_ERR_ARG;
        }
        f->col.insert(f->col.end(), b, u);
        f->rowptr[i + 1] = (int32_t)f->col.size();
    }
    std::vector<int32_t>().swap(cand);
    f->nnz = (int64_t)f->col.size();
    // contributions: entry k of (dof_a, dof_b) receives pair (a, b) of e
    const int64_t ncontrib_max = cnt[n];
    if (ncontrib_max >= (int64_t)INT32_MAX) {
        f->err = "too many element contributions for int32 lists";
        return CG_ERR_ARG;
    }
    std::vector<int32_t> kpos((size_t)ncontrib_max);
    cptr.assign((size_t)f->nnz + 1, 0);
    int64_t m = 0;
    for (int64_t e = 0; e < nelem; ++e)
        for (int a = 0; a < 4; ++a) {
            const int32_t i = edof[4 * e + a];
            if (i < 0)
                continue;
            const int32_t *rb = f->col.data() + f->rowptr[i], *re = f->col.data() + f->rowptr[i + 1];
            for (int b = 0; b < 4; ++b) {
                const int32_t j = edof[4 * e + b];
                if (j < 0)
                    continue;
                const int32_t k = (int32_t)(std::lower_bound(rb, re, j) - f->col.data());
                kpos[m++] = k;
                cptr[k + 1]++;
            }
        }
    for (int64_t k = 0; k < f->nnz; ++k)
        cptr[k + 1] += cptr[k];
    cq.resize((size_t)m);
    {
        std::vector<int32_t> next(cptr.begin(), cptr.end() - 1);
        int64_t t = 0;
        for (int64_t e = 0; e < nelem; ++e)
            for (int a = 0; a < 4; ++a) {
                if (edof[4 * e + a] < 0)
                    continue;
                for (int b = 0; b < 4; ++b)
                    if (edof[4 * e + b] >= 0)
                        cq[next[kpos[t++]]++] = (int32_t)(e << 4 | pair_index(a, b));
            }
    }
    f->ncontrib = m;
    return CG_OK;
}

} // namespace

extern "C" {

int cg_fem_create(cg_fem **out, int64_t npts, const double *coords, int64_t nelem, const int32_t *tets,
                  const int32_t *dof, int64_t n)
{
    if (!out) {
        g_fem_err = "out is NULL";
        return CG_ERR_ARG;
    }
    *out = nullptr;
    if (npts < 0 || nelem < 0 || n < 0 || n >= (int64_t)INT32_MAX || npts >= (int64_t)INT32_MAX ||
        nelem >= ((int64_t)1 << 27) || (npts > 0 && (!coords || !dof)) || (nelem > 0 && !tets)) {
        g_fem_err = "need 0 <= n, npts < 2^31, 0 <= nelem < 2^27 and non-NULL arrays";
        return CG_ERR_ARG;
    }
    std::unique_ptr<cg_fem> f;
    int st;
    try {
        f.reset(new cg_fem());
        f->npts = npts;
        f->nelem = nelem;
        f->n = n;
        std::vector<int32_t> edof, cptr, cq;
        st = fem_plan(f.get(), coords, tets, dof, edof, cptr, cq);
        if (st == CG_OK && nelem > 0) {
            double *dco = nullptr;
            int32_t *dtet = nullptr, *bad = nullptr;
            if ((st = fem_upload(f.get(), &f->edof, edof.data(), edof.size())) == CG_OK &&
                (st = fem_alloc(f.get(), &f->khat, (size_t)(10 * nelem))) == CG_OK &&
                (st = fem_upload(f.get(), &f->cptr, cptr.data(), cptr.size())) == CG_OK &&
                (st = fem_upload(f.get(), &f->cq, cq.data(), cq.size())) == CG_OK &&
                (st = fem_upload(f.get(), &dco, coords, (size_t)(3 * npts))) == CG_OK &&
                (st = fem_upload(f.get(), &dtet, tets, (size_t)(4 * nelem))) == CG_OK &&
                (st = fem_alloc(f.get(), &bad, 1)) == CG_OK) {
                int32_t hbad = 0;
                hipError_t e = hipMemcpy(bad, &hbad, sizeof(hbad), hipMemcpyHostToDevice);
                if (e == hipSuccess) {
                    hipLaunchKernelGGL(k_fem_khat, dim3((unsigned)((nelem + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                                       nullptr, nelem, dco, dtet, f->khat, bad);
                    e = hipGetLastError();
                }
                if (e == hipSuccess)
                    e = hipMemcpy(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost);
                if (e != hipSuccess) {
                    st = fem_hip_fail(f.get(), e, "element matrices");
                } else if (hbad) {
                    f->err = "an element has zero or non-finite volume";
                    st = CG_ERR_ARG;
                }
                // the coordinates and point ids are not needed after this
                for (void *p : {(void *)dco, (void *)dtet, (void *)bad}) {
                    f->allocs.erase(std::remove(f->allocs.begin(), f->allocs.end(), p), f->allocs.end());
                    (void)hipFree(p);
                }
            }
        }
    } catch (const std::bad_alloc &) {
        f->err = "host allocation failed";
        st = CG_ERR_NOMEM;
    }
    if (st != CG_OK) {
        g_fem_err = f->err;
        fem_release(f.get());
        return st;
    }
    g_fem_err.clear();
    *out = f.release();
    return CG_OK;
}

int cg_fem_set_stream(cg_fem *f, void *hip_stream)
{
    if (!f)
        return CG_ERR_ARG;
    f->stream = static_cast<hipStream_t>(hip_stream);
    return CG_OK;
}

int cg_fem_pattern(const cg_fem *f, int64_t *nnz, int32_t *rowptr, int32_t *col)
{
    if (!f)
        return CG_ERR_ARG;
    if (nnz)
        *nnz = f->nnz;
    if (rowptr)
        std::memcpy(rowptr, f->rowptr.data(), f->rowptr.size() * sizeof(int32_t));
    if (col && f->nnz)
        std::memcpy(col, f->col.data(), (size_t)f->nnz * sizeof(int32_t));
    return CG_OK;
}

int cg_fem_assemble(cg_fem *f, const double *nu, double *vals)
{
    if (!f)
        return CG_ERR_ARG;
    if (f->nnz == 0)
        return CG_OK;
    if (!vals || (f->nelem > 0 && !nu)) {
        f->err = "nu / vals NULL";
        return CG_ERR_ARG;
    }
    hipLaunchKernelGGL(k_fem_assemble, dim3((unsigned)((f->nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, f->stream,
                       f->nnz, f->nelem, f->cptr, f->cq, f->khat, nu, vals);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CG_OK : fem_hip_fail(f, e, "k_fem_assemble");
}

int cg_fem_nu_grad(cg_fem *f, const double *lam, const double *x, double *grad)
{
    if (!f)
        return CG_ERR_ARG;
    if (f->nelem == 0)
        return CG_OK;
    if (!grad || (f->n > 0 && (!lam || !x))) {
        f->err = "lam / x / grad NULL";
        return CG_ERR_ARG;
    }
    hipLaunchKernelGGL(k_fem_nu_grad, dim3((unsigned)((f->nelem + kBlock - 1) / kBlock)), dim3(kBlock), 0, f->stream,
                       f->nelem, reinterpret_cast<const int4 *>(f->edof), f->khat, lam, x, grad);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CG_OK : fem_hip_fail(f, e, "k_fem_nu_grad");
}

void cg_fem_destroy(cg_fem *f)
{
    if (!f)
        return;
    (void)hipStreamSynchronize(f->stream);
    fem_release(f);
    delete f;
}

const char *cg_fem_last_error(const cg_fem *f)
{
    return f ? f->err.c_str() : g_fem_err.c_str();
}

} // extern "C"

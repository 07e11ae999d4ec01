/*
 * CPU oracle for the conjugate-gradient / SpMV path -- TEST INFRASTRUCTURE.
 *
 * Plain, serial, obviously-correct FP64 code that the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code,
 * header or constant with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so every
 * product and sum is rounded exactly as written, left to right from +0.0).
 *
 * What it follows (Rodrigues et al., "Parallel Sparse Matrix Solver on the GPU
 * Applied to Simulation of Electrical Machines"):
 *   - section III, CG algorithm: alpha = r'r / p'Ap, x += alpha p, convergence
 *     test, r -= alpha Ap, beta = r_k'r_k / r_{k-1}'r_{k-1}, p = r + beta p;
 *   - section III, SpMV text: the "trivial" CSR product (one row -> one sum),
 *     and the symmetric storage A = L + D + U with U' = L, where the stored
 *     triangle plus its transpose (read column-wise) gives y = Ax;
 *   - section III, problem size text: symmetric sparse FP64 matrices stored in
 *     full or symmetric CSR; section I: Ax = b with A SPD.
 * Readings taken where the paper is silent (the convergence criterion is the
 * relative recursive residual ||r||_2 <= tol ||b||_2 tested after the r
 * update; r0 = b - A x0; the loop bound is maxit; the single SpMV per
 * iteration is reused for the r update; non-positive p'Ap is a breakdown) are
 * listed with the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* status codes: the same meaning as the GPU library's (independently defined) */
#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_STRUCTURE (-2)
#define ORC_ERR_BREAKDOWN (-3)
#define ORC_ERR_NONFINITE (-4)
#define ORC_ERR_NOMEM (-5)

#define ORC_FMT_CSR 0
#define ORC_FMT_SYM_CSR 1 /* upper triangle incl. diagonal, stored by rows */
#define ORC_FMT_CSC 2

#define ORC_CHECK_SYMMETRY 1u

typedef struct {
    int32_t iters;
    int32_t status;
    double relres;      /* sqrt(r'r) / ||b|| of the recursive residual */
    double relres_true; /* ||b - A x|| / ||b||, one extra product */
    double ms_loop;     /* wall time of the iteration loop only */
} orc_info;

/* ---------------------------------------------------------------- SpMV */

/* CSR: y_i = sum_k val[k] x[col[k]] over row i, k ascending (the paper's
 * "trivial" kernel: one row, one running sum). */
void orc_spmv_csr(int64_t n, const int32_t *ptr, const int32_t *col,
                  const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* CSC: y = sum_j x_j A(:, j), columns ascending, entries ascending. */
void orc_spmv_csc(int64_t n, const int32_t *ptr, const int32_t *row,
                  const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = ptr[j]; k < ptr[j + 1]; ++k)
            y[row[k]] += val[k] * x[j];
}

/* Symmetric CSR (stored triangle T = D + U, by rows): y = T x + U' x.
 * Row i gathers its own entries; every off-diagonal entry (i, j) also adds
 * its mirror a_ji x_i to y_j. */
void orc_spmv_symcsr(int64_t n, const int32_t *ptr, const int32_t *col,
                     const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            int64_t j = col[k];
            y[i] += val[k] * x[j];
            if (j != i)
                y[j] += val[k] * x[i];
        }
}

void orc_spmv(int fmt, int64_t n, const int32_t *ptr, const int32_t *idx,
              const double *val, const double *x, double *y)
{
    if (fmt == ORC_FMT_CSR)
        orc_spmv_csr(n, ptr, idx, val, x, y);
    else if (fmt == ORC_FMT_CSC)
        orc_spmv_csc(n, ptr, idx, val, x, y);
    else
        orc_spmv_symcsr(n, ptr, idx, val, x, y);
}

/* ------------------------------------------------------------- vectors */

/* The scalar products r'r and p'Ap of the algorithm are taken as their exact
 * values rounded to FP64: the paper leaves the summation order to a library
 * routine, and a left-to-right FP64 loop over n ~ 1e4-1e6 terms is itself a
 * source of error (up to n u sum|a_i b_i|) that moves CG's stopping step.
 * Evaluation: Dot2 of Ogita, Rump and Oishi ("Accurate sum and dot product",
 * SIAM J. Sci. Comput. 26(6), 2005): every product split exactly as
 * p + pe (pe = fma(a, b, -p)), every addition split exactly as t + e (TwoSum),
 * the error terms summed apart and added once at the end.  The result is as
 * accurate as if computed in twice the working precision, then rounded. */
double orc_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p = a[i] * b[i];
        const double pe = fma(a[i], b[i], -p);
        const double t = s + p;
        const double z = t - s;
        const double e = (s - (t - z)) + (p - z);
        s = t;
        c += e + pe;
    }
    return s + c;
}

/* The literal left-to-right loop, kept to measure how much an unspecified
 * summation order moves the iteration (dot_mode 1 of orc_cg). */
double orc_dot_plain(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

/* Pairwise (recursive halving) summation of the products: the two halves
 * [0, h) and [h, n), h = n / 2, summed apart and added; runs of at most 8
 * terms left to right.  The order of blocked and tree reductions on parallel
 * hardware; error <= gamma(ceil(log2 n) + 8) sum |a_i b_i|.  Kept, like the
 * plain loop, to measure how far an unspecified summation order moves the
 * iteration (dot_mode 2 of orc_cg). */
double orc_dot_pairwise(int64_t n, const double *a, const double *b)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += a[i] * b[i];
        return s;
    }
    const int64_t h = n / 2;
    return orc_dot_pairwise(h, a, b) + orc_dot_pairwise(n - h, a + h, b + h);
}

/* Left-to-right accumulation with a fused multiply-add per term (one
 * rounding per term): the scalar product of FMA hardware.  Error <= gamma_n
 * sum |a_i b_i| like the plain loop (dot_mode 3 of orc_cg). */
double orc_dot_fused(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s = fma(a[i], b[i], s);
    return s;
}

/* --------------------------------------------------------- conversions */

/* Stable counting-sort transpose: (ptr, idx, val) by lines -> by the other
 * index.  Used both for CSR -> CSC and for CSC -> CSR. */
int orc_transpose(int64_t n, const int32_t *ptr, const int32_t *idx, const double *val,
                  int32_t *tptr, int32_t *tidx, double *tval)
{
    int64_t nnz = ptr[n];
    for (int64_t i = 0; i <= n; ++i)
        tptr[i] = 0;
    for (int64_t k = 0; k < nnz; ++k)
        tptr[idx[k] + 1]++;
    for (int64_t i = 0; i < n; ++i)
        tptr[i + 1] += tptr[i];
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!next)
        return ORC_ERR_NOMEM;
    for (int64_t i = 0; i < n; ++i)
        next[i] = tptr[i];
    for (int64_t l = 0; l < n; ++l)
        for (int64_t k = ptr[l]; k < ptr[l + 1]; ++k) {
            int32_t dst = next[idx[k]]++;
            tidx[dst] = (int32_t)l;
            tval[dst] = val[k];
        }
    free(next);
    return ORC_OK;
}

/* Keep the entries with col >= row (the upper triangle incl. diagonal).
 * Returns the new nnz; out arrays must hold ptr[n] entries. */
int64_t orc_csr_upper(int64_t n, const int32_t *ptr, const int32_t *col, const double *val,
                      int32_t *uptr, int32_t *ucol, double *uval)
{
    int64_t m = 0;
    uptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] >= i) {
                ucol[m] = col[k];
                uval[m] = val[k];
                ++m;
            }
        uptr[i + 1] = (int32_t)m;
    }
    return m;
}

/* Symmetric CSR (upper) -> full CSR: row i is the mirrored lower part
 * (entries (k, i) with k < i, k ascending) followed by its stored row. */
int64_t orc_sym_expand(int64_t n, const int32_t *uptr, const int32_t *ucol, const double *uval,
                       int32_t *ptr, int32_t *col, double *val)
{
    /* the lower part of row i = column i of the stored upper triangle */
    int64_t nnz_u = uptr[n];
    int32_t *tptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *tidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz_u > 0 ? nnz_u : 1));
    double *tval = (double *)malloc(sizeof(double) * (size_t)(nnz_u > 0 ? nnz_u : 1));
    if (!tptr || !tidx || !tval) {
        free(tptr); free(tidx); free(tval);
        return -1;
    }
    orc_transpose(n, uptr, ucol, uval, tptr, tidx, tval);
    int64_t m = 0;
    ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = tptr[i]; k < tptr[i + 1]; ++k)
            if (tidx[k] < i) {
                col[m] = tidx[k];
                val[m] = tval[k];
                ++m;
            }
        for (int64_t k = uptr[i]; k < uptr[i + 1]; ++k) {
            col[m] = ucol[k];
            val[m] = uval[k];
            ++m;
        }
        ptr[i + 1] = (int32_t)m;
    }
    free(tptr); free(tidx); free(tval);
    return m;
}

/* ---------------------------------------------------------- validation */

/* Structure checks on 0- or 1-based input, mirroring the library's rules:
 * ptr[0] == base, ptr non-decreasing, indices in range and strictly
 * increasing within a line, symmetric CSR holds only j >= i and every row
 * starts with its diagonal, values finite; optionally exact symmetry. */
int orc_validate(int fmt, int64_t n, const int32_t *ptr, const int32_t *idx,
                 const double *val, int base, uint32_t flags)
{
    if (fmt < 0 || fmt > 2 || n < 0 || (base != 0 && base != 1))
        return ORC_ERR_ARG;
    if (n == 0)
        return ORC_OK;
    if (!ptr)
        return ORC_ERR_ARG;
    if (ptr[0] != base)
        return ORC_ERR_STRUCTURE;
    for (int64_t i = 0; i < n; ++i)
        if (ptr[i + 1] < ptr[i])
            return ORC_ERR_STRUCTURE;
    int64_t nnz = (int64_t)ptr[n] - base;
    if (nnz > 0 && (!idx || !val))
        return ORC_ERR_ARG;
    for (int64_t l = 0; l < n; ++l) {
        int64_t b = ptr[l] - base, e = ptr[l + 1] - base;
        for (int64_t k = b; k < e; ++k) {
            int64_t j = (int64_t)idx[k] - base;
            if (j < 0 || j >= n)
                return ORC_ERR_STRUCTURE;
            if (k > b && idx[k] <= idx[k - 1])
                return ORC_ERR_STRUCTURE;
            /* symmetric CSR: the row starts with its diagonal; with strictly
             * increasing indices that also rules out any entry j < i */
            if (fmt == ORC_FMT_SYM_CSR && k == b && j != l)
                return ORC_ERR_STRUCTURE;
        }
        if (fmt == ORC_FMT_SYM_CSR && e == b)
            return ORC_ERR_STRUCTURE;
    }
    for (int64_t k = 0; k < nnz; ++k)
        if (!isfinite(val[k]))
            return ORC_ERR_NONFINITE;
    if ((flags & ORC_CHECK_SYMMETRY) && fmt != ORC_FMT_SYM_CSR) {
        /* A == A' exactly: compare with the transpose entry by entry */
        int32_t *p0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t *i0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        int32_t *tp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t *ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        double *tv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        int st = ORC_OK;
        if (!p0 || !i0 || !tp || !ti || !tv) {
            st = ORC_ERR_NOMEM;
        } else {
            for (int64_t i = 0; i <= n; ++i)
                p0[i] = ptr[i] - base;
            for (int64_t k = 0; k < nnz; ++k)
                i0[k] = idx[k] - base;
            orc_transpose(n, p0, i0, val, tp, ti, tv);
            for (int64_t i = 0; i <= n && st == ORC_OK; ++i)
                if (tp[i] != p0[i])
                    st = ORC_ERR_STRUCTURE;
            for (int64_t k = 0; k < nnz && st == ORC_OK; ++k)
                if (ti[k] != i0[k] || tv[k] != val[k])
                    st = ORC_ERR_STRUCTURE;
        }
        free(p0); free(i0); free(tp); free(ti); free(tv);
        return st;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ CG */

static double now_ms(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/*
 * Conjugate gradient on a 0-based matrix in the given format.
 *   x      in: x0, out: the last iterate (untouched on ORC_ERR_ARG / NONFINITE)
 *   hist_* optional (NULL = off): alpha_k, beta_k and ||r_k|| per iteration
 *          (hist_cap entries), and x after iterations x_first,
 *          x_first + x_stride, ... into x_hist (x_cap snapshots of n values).
 *   dot_mode 0: scalar products by orc_dot (exact value, rounded once);
 *            1: the plain left-to-right loop; 2: pairwise summation;
 *            3: fused multiply-add throughout -- scalar products accumulated
 *               left to right with one rounding per term, x += alpha p,
 *               r -= alpha q and p = r + beta p each one fused operation
 *               (what FMA hardware and its BLAS do).
 * With the environment variable ORC_PROGRESS set to k > 0, one line with the
 * iteration count and the recursive relative residual goes to stderr every
 * k iterations (output only; a long run on a large system shows it is alive).
 */
int orc_cg(int fmt, int64_t n, const int32_t *ptr, const int32_t *idx, const double *val,
           const double *b, double *x, double tol, int32_t maxit, orc_info *info,
           double *alpha_hist, double *beta_hist, double *res_hist, int32_t hist_cap,
           double *x_hist, int32_t x_stride, int32_t x_cap, int32_t x_first, int dot_mode)
{
    double (*dot)(int64_t, const double *, const double *) =
        dot_mode == 1 ? orc_dot_plain : dot_mode == 2 ? orc_dot_pairwise : dot_mode == 3 ? orc_dot_fused : orc_dot;
    const int fused = dot_mode == 3;
    orc_info loc;
    if (!info)
        info = &loc;
    memset(info, 0, sizeof(*info));
    if (n < 0 || maxit < 0 || !(tol >= 0.0)) {
        info->status = ORC_ERR_ARG;
        return ORC_ERR_ARG;
    }
    if (n == 0) {
        info->status = ORC_OK;
        return ORC_OK;
    }
    double nb = sqrt(dot(n, b, b));
    if (!isfinite(nb)) {
        info->status = ORC_ERR_NONFINITE;
        return ORC_ERR_NONFINITE;
    }
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = 0.0;
        info->status = ORC_OK;
        return ORC_OK;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        info->status = ORC_ERR_NOMEM;
        return ORC_ERR_NOMEM;
    }
    const char *pe = getenv("ORC_PROGRESS");
    const long progress = pe ? strtol(pe, NULL, 10) : 0;
    double t0 = now_ms();
    /* init: r0 = b - A x0, p0 = r0 */
    orc_spmv(fmt, n, ptr, idx, val, x, q);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        p[i] = r[i];
    }
    double rho = dot(n, r, r);
    int status = ORC_NOT_CONVERGED;
    int32_t k = 0;
    if (sqrt(rho) <= tol * nb) {
        status = ORC_OK;
    } else {
        for (k = 1; k <= maxit; ++k) {
            /* alpha = r'r / p'Ap with the iteration's single product q = Ap */
            orc_spmv(fmt, n, ptr, idx, val, p, q);
            double sigma = dot(n, p, q);
            if (!(sigma > 0.0) || !isfinite(sigma)) {
                status = ORC_ERR_BREAKDOWN;
                --k;
                break;
            }
            double alpha = rho / sigma;
            if (fused) {
                for (int64_t i = 0; i < n; ++i) {
                    x[i] = fma(alpha, p[i], x[i]);
                    r[i] = fma(-alpha, q[i], r[i]);
                }
            } else {
                for (int64_t i = 0; i < n; ++i)
                    x[i] = x[i] + alpha * p[i];
                for (int64_t i = 0; i < n; ++i)
                    r[i] = r[i] - alpha * q[i];
            }
            double rho_new = dot(n, r, r);
            double beta = rho_new / rho;
            if (alpha_hist && k <= hist_cap) {
                alpha_hist[k - 1] = alpha;
                beta_hist[k - 1] = beta;
                res_hist[k - 1] = sqrt(rho_new);
            }
            if (x_hist && x_stride > 0 && k >= x_first && (k - x_first) % x_stride == 0 &&
                (k - x_first) / x_stride < x_cap)
                memcpy(x_hist + (size_t)((k - x_first) / x_stride) * (size_t)n, x, sizeof(double) * (size_t)n);
            rho = rho_new;
            if (progress > 0 && k % progress == 0) {
                fprintf(stderr, "[oracle cg] n=%lld iteration %d relres %.3e %.0f ms\n", (long long)n, k,
                        sqrt(rho) / nb, now_ms() - t0);
                fflush(stderr);
            }
            if (sqrt(rho) <= tol * nb) {
                status = ORC_OK;
                break;
            }
            if (fused) {
                for (int64_t i = 0; i < n; ++i)
                    p[i] = fma(beta, p[i], r[i]);
            } else {
                for (int64_t i = 0; i < n; ++i)
                    p[i] = r[i] + beta * p[i];
            }
        }
        if (k > maxit)
            k = maxit;
    }
    info->ms_loop = now_ms() - t0;
    info->iters = k;
    info->status = status;
    info->relres = sqrt(rho) / nb;
    /* true residual ||b - A x|| / ||b|| */
    orc_spmv(fmt, n, ptr, idx, val, x, q);
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - q[i];
    info->relres_true = sqrt(dot(n, r, r)) / nb;
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------- timing mode */

/*
 * TIMING MODE ONLY -- not the correctness reference (orc_cg is).  The CSR
 * iteration of orc_cg with every loop split into static, contiguous chunks
 * over the OpenMP threads (OMP_NUM_THREADS, default all host cores), so that
 * the CPU baseline is the same algorithm on the whole host rather than one
 * core.  The row sums are the serial ones (one row, one running sum); each
 * thread forms the exactly rounded scalar product of its chunk as a Dot2 pair
 * (sum, error), and the pairs are combined in thread order with TwoSum, so
 * r'r and p'Ap keep the exactness of orc_dot up to the final rounding of the
 * combined pair.  Only CSR: the symmetric and CSC products scatter into other
 * rows and have no race-free static split.  *threads receives the count used.
 */
#ifdef _OPENMP
#include <omp.h>
#endif

static double omp_dot2(int64_t n, const double *a, const double *b, double *ps, double *pc, int nt)
{
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t i0 = n * t / nt, i1 = n * (t + 1) / nt;
        double hi = 0.0, lo = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
            const double prod = a[i] * b[i];
            const double prod_err = fma(a[i], b[i], -prod);
            const double sum = hi + prod;
            const double bv = sum - hi;
            const double sum_err = (hi - (sum - bv)) + (prod - bv);
            hi = sum;
            lo += sum_err + prod_err;
        }
        ps[t] = hi;
        pc[t] = lo;
    }
    double hi = 0.0, lo = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double sum = hi + ps[t];
        const double bv = sum - hi;
        lo += ((hi - (sum - bv)) + (ps[t] - bv)) + pc[t];
        hi = sum;
    }
    return hi + lo;
}

int orc_cg_csr_omp(int64_t n, const int32_t *ptr, const int32_t *col, const double *val, const double *b,
                   double *x, double tol, int32_t maxit, orc_info *info, int32_t *threads)
{
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    if (threads)
        *threads = nt;
    memset(info, 0, sizeof(*info));
    if (n <= 0 || maxit < 0 || !(tol >= 0.0)) {
        info->status = n == 0 ? ORC_OK : ORC_ERR_ARG;
        return info->status;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *ps = (double *)malloc(sizeof(double) * (size_t)nt);
    double *pc = (double *)malloc(sizeof(double) * (size_t)nt);
    if (!r || !p || !q || !ps || !pc) {
        free(r); free(p); free(q); free(ps); free(pc);
        info->status = ORC_ERR_NOMEM;
        return ORC_ERR_NOMEM;
    }
    const double nb = sqrt(omp_dot2(n, b, b, ps, pc, nt));
    double t0 = now_ms();
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0.0;
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
            ax += val[e] * x[col[e]];
        r[i] = b[i] - ax;
        p[i] = r[i];
    }
    double rho = omp_dot2(n, r, r, ps, pc, nt);
    int status = ORC_NOT_CONVERGED;
    int32_t k = 0;
    if (sqrt(rho) <= tol * nb) {
        status = ORC_OK;
    } else {
        for (k = 1; k <= maxit; ++k) {
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
                    s += val[e] * p[col[e]];
                q[i] = s;
            }
            const double sigma = omp_dot2(n, p, q, ps, pc, nt);
            if (!(sigma > 0.0) || !isfinite(sigma)) {
                status = ORC_ERR_BREAKDOWN;
                --k;
                break;
            }
            const double alpha = rho / sigma;
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int64_t i = 0; i < n; ++i) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
            const double rho_new = omp_dot2(n, r, r, ps, pc, nt);
            const double beta = rho_new / rho;
            rho = rho_new;
            if (sqrt(rho) <= tol * nb) {
                status = ORC_OK;
                break;
            }
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * p[i];
        }
        if (k > maxit)
            k = maxit;
    }
    info->ms_loop = now_ms() - t0;
    info->iters = k;
    info->status = status;
    info->relres = nb > 0.0 ? sqrt(rho) / nb : 0.0;
    free(r); free(p); free(q); free(ps); free(pc);
    return status;
}

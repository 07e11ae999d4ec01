// Device-side declarations shared by the kernels and the C-ABI driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.h"

namespace cgmi {

// Iteration state kept in device memory.  Every kernel reads it at entry,
// and every field is written by one thread only (block 0, thread 0), so
// kernel boundaries are the synchronisation.  One field is written while
// other blocks of the same kernel may still read it: `status`, set by the
// stop decision of iter_gate and by k_update_r on breakdown.  That is safe
// because every block takes the same decision from fields that kernel does
// not write (conv_next, k, maxit, and the same p'Ap partials): a block that
// still reads kRun reaches the same stop and returns without writing
// anything, exactly as a block that already reads the new status does.  A
// gate whose decision could differ between blocks would need the status
// written in a later kernel instead.
enum DevStatus : int32_t {
    kRun = 0,        // iterating
    kConverged = 1,  // ||r|| <= tol ||b||
    kMaxit = 2,      // maxit products done
    kBreakdown = 3,  // p'Ap <= 0 or non-finite
    kNonfinite = 4,  // ||b|| not finite
    kZeroRhs = 5     // b == 0: x = 0
};

struct DevState {
    int32_t status;
    int32_t k;       // products Ap completed inside the loop
    int32_t maxit;
    int32_t iters;   // final count (set when the loop stops)
    double tol_nb;   // tol * ||b||
    double nb;       // ||b||
    double rho;      // r'r of the current residual
    double alpha;    // step of the current iteration
    double sigma;    // p'Ap of the current iteration
    double res_true; // ||b - A x|| / ||b|| (filled after the loop)
    double rho_next; // r'r after the latest r update (published for the next iteration's gate)
    int32_t conv_next; // sqrt(rho_next) <= tol_nb
    int32_t pad;
};

// Device image of a planned matrix.
struct DevMatrix {
    int format = 0;
    int n = 0;
    int lanes = 16;
    const int32_t *ptr = nullptr;
    const int32_t *idx = nullptr;
    const double *val = nullptr;
    const float *val32 = nullptr;  // mixed precision: values of D^-1/2 A D^-1/2 in FP32
    const double *dscale = nullptr; // mixed precision: D^-1/2
    // CSR
    int csr_blocks = 0, csr_rows_per_block = 0;
    bool csr_stream = false;
    int csr_nrb = 0;
    const int32_t *csr_rb = nullptr;
    const int2 *csr_rbe = nullptr;       // per row-block boundary: {first row, first entry}
    bool slices = false;                 // sliced layout of CSR rows / CSC panel slots (plan.h)
    int sl_lines = 0, nslices = 0;
    const int32_t *sl_off = nullptr, *sl_col = nullptr, *sl_src = nullptr;
    const int16_t *sl_d16 = nullptr;     // banded: 16-bit column offsets from the line's row instead of sl_col
    double *sl_val = nullptr;            // values at the slice positions (0 at padding)
    float *sl_val32 = nullptr;           // mixed precision: val32 at the slice positions
    // scatter
    int nblocks = 0, ncolors = 0, lds_entries = 0, lds_lines = 0, max_slots = 0;
    std::vector<int32_t> color_off;      // host copy: blocks per colour
    std::vector<int32_t> color_slot_off; // host copy: slots per colour (device arrays in colour order)
    int scatter_wgs = 0;                 // workgroups of k_scatter_sums (= dot partials)
    const ScatterBlock *blocks = nullptr; // in colour order; slot0 / id refer to the colour-ordered arrays
    double *part = nullptr;              // parked slot sums (colours >= 1); CSC panels: by row
    const int32_t *rs_ptr = nullptr;     // per row: its parked slots [rs_ptr[i], rs_ptr[i+1]) of rs_idx
    const int32_t *rs_idx = nullptr;     //   slot indices, ascending colour (symmetric CSR); null (compact
                                         //   blocks): the parked sums themselves are stored by row
    const uint8_t *has_c0 = nullptr;     // per row: written by a colour-0 block; CSC panels: bit 1 = part_i
    const int32_t *slot_target = nullptr;
    const uint8_t *slot_flag = nullptr;
    const uint16_t *seg = nullptr;
    const uint16_t *tl = nullptr;          // sliced blocks: local positions
    // symmetric CSR, sliced blocks (plan.h)
    bool sym_slices = false;
    const int2 *ss_blk = nullptr;          // per device block: {first position, entries per line}
    const int32_t *ss_idx = nullptr, *ss_src = nullptr;
    double *ss_val = nullptr;              // values at the positions (0 at padding)
    float *ss_val32 = nullptr;             // mixed precision: val32 at the positions
    int64_t ss_positions = 0;
    // symmetric CSR, compact blocks (plan.h): positions in ss_idx / ss_val,
    // slots in slot_target / seg, contributions in tl, parked sums in part
    // with per-row lists rs_ptr / rs_idx (has_c0 unused: every row is stored
    // by the block that owns its line)
    bool compact = false;                 // (its rows renumbered in block order: vperm / vinv)
    const CompactBlock *cblocks = nullptr;
    const int32_t *vperm = nullptr;       // [n] device row k = caller's row vperm[k]
    const int32_t *vinv = nullptr;        // [n] caller's row i = device row vinv[i]
    const uint16_t *cp_rank = nullptr;    // [8 n] LDS place of each entry's mirror product
    const int32_t *cp_dest = nullptr;     // [parked] place of each parked sum in the by-row array
    int64_t parked = 0;
    // CSC column panels (nblocks = chunks, scatter_wgs = their workgroups)
    bool panel = false;
    bool pn_gather = false;               // some row has parked sums or no writer
    const int32_t *pn_chunk_slot = nullptr, *pn_slot_ptr = nullptr, *pn_slot_target = nullptr;
    const int32_t *pn_col = nullptr, *pn_src = nullptr;
    double *pn_val = nullptr;             // values in panel order (from val through pn_src)
    float *pn_val32 = nullptr;            // mixed precision: val32 in panel order
    int pn_first_parked = 0;
    // sliced kernels: ordinary (cache-allocating) loads of the matrix streams
    // when the product's bytes fit the Infinity Cache, non-temporal otherwise
    bool matrix_cached = false;
    // vectors
    int vec_blocks = 0, vec_chunk = 0;
    int spmv_blocks() const { return format == kCsr || slices ? csr_blocks : scatter_wgs; }
    // the product ends with a row pass (parked slot sums, rows with no writer)
    int64_t part_doubles = 0;             // entries of `part` (0: no parked sums)
    bool row_pass() const
    {
        return panel ? pn_gather : compact ? parked > 0 : (format == kSymCsr && ncolors > 1);
    }
};

// Iteration context: null st = plain product (no gating, p'q partials still
// written to sig_part).
struct IterCtx {
    DevState *st = nullptr;
    const double *rho_part = nullptr;
    int n_rho = 0;
    // leave the row pass of a scatter product to the r update (y then holds
    // only the colour-0 rows; the iteration's q is never read elsewhere)
    bool defer_rows = false;
    // parked sums of a scatter product in this buffer instead of the
    // handle's (at least DevMatrix::part_doubles entries)
    double *part = nullptr;
    // Two kernels per CG iteration (small systems): the product forms the
    // search direction p = r + beta p_prev itself -- for every gathered
    // column and for its own rows, which it stores in pnew -- and applies
    // x += alpha p_prev to its own rows; beta and the stop decision come from
    // the r update's partials (rho_part), which it reduces like the x/p
    // update does.  Same arithmetic, same bits as three kernels.
    bool fused = false;
    const double *pold = nullptr, *r = nullptr;
    double *pnew = nullptr, *x = nullptr;
};

// y = A x; writes spmv_blocks() partials of x'y into sig_part.
void launch_spmv(const DevMatrix &m, const double *x, double *y, double *sig_part, const IterCtx &ctx,
                 hipStream_t s);
// y = A32 x with the FP32 copy of the scaled values (FP64 arithmetic).
void launch_spmv32(const DevMatrix &m, const float *x, double *y, double *sig_part, const IterCtx &c,
                   hipStream_t s);
// r -= alpha q with alpha = rho / sum(sig_part); rho_part <- partials of r'r.
// rows_deferred: q came from a product launched with defer_rows, so each
// q_i is finished here from the parked slot sums first.
void launch_update_r(const DevMatrix &m, double *r, const double *q, DevState *st, const double *sig_part,
                     double *rho_part, hipStream_t s, bool rows_deferred = false, bool fused = false);
// x += alpha p; p = r + beta p (unless converged) with beta = sum(rho_part) / rho.
void launch_update_xp(const DevMatrix &m, double *x, double *p, const double *r, DevState *st,
                      const double *rho_part, hipStream_t s);
// mixed precision: the same update with p stored in FP32
void launch_update_xp32(const DevMatrix &m, double *x, float *p, const double *r, DevState *st,
                        const double *rho_part, hipStream_t s);
// mixed precision: rh = D^-1/2 r_out, p = fl32(rh) (unless keep_p: the
// direction of the previous inner solve carries over), c = 0, partials of rh'rh
void launch_mx_init(const DevMatrix &m, const double *r_out, double *rh, float *p, double *c, double *rho_part,
                    double *bb_part, hipStream_t s, bool keep_p);
// mixed precision: x += D^-1/2 c
void launch_mx_apply(const DevMatrix &m, double *x, const double *c, hipStream_t s);
// st->rho = sum(rho_part), st->res_true = sqrt(st->rho) / st->nb (one workgroup)
void launch_outer_norm(const DevMatrix &m, DevState *st, const double *rho_part, hipStream_t s);
// convergence / maxit test of the current residual (one workgroup).
void launch_check(const DevMatrix &m, DevState *st, const double *rho_part, hipStream_t s);
// r = b - q, p = r, xw = x0; partials of r'r and b'b.
void launch_init_vec(const DevMatrix &m, const double *b, const double *x0, const double *q, double *r, double *p,
                     double *xw, double *rho_part, double *bb_part, hipStream_t s);
void launch_init_state(const DevMatrix &m, DevState *st, const double *bb_part, const double *rho_part, double tol,
                       int32_t maxit, hipStream_t s);
// res_true = ||b - q|| / ||b|| into st (two launches)
void launch_true_residual(const DevMatrix &m, const double *b, const double *q, double *part, DevState *st,
                          hipStream_t s);
void launch_fill(int n, double *x, double v, hipStream_t s);
// dst[k] = src[perm[k]] for k < nnz, 0 where perm[k] < 0 (values into the
// CSC panel order or the CSR slice positions)
void launch_permute(int64_t nnz, const double *src, const int32_t *perm, double *dst, hipStream_t s);
void launch_permute(int64_t nnz, const float *src, const int32_t *perm, float *dst, hipStream_t s);
// val[k] = src[perm ? perm[k] : k] for k < nnz
void launch_set_values(int64_t nnz, const double *src, const int32_t *perm, double *val, hipStream_t s);
// mixed precision: recompute D^-1/2 (into sc, the caller's row order) and the FP32 scaled values from
// m.val; *bad <- 1 on a bad diagonal
void launch_mx_rescale(const DevMatrix &m, double *sc, float *v32, int32_t *bad, hipStream_t s);
// out[perm ? perm[k] : k] = dL/d(stored value k) from the adjoint lam and the solution x
void launch_pattern_grad(const DevMatrix &m, const double *lam, const double *x, const int32_t *perm, double *out,
                         hipStream_t s);

} // namespace cgmi

/*
 * cgmi -- conjugate gradient for sparse symmetric positive-definite systems
 * on one MI355X (gfx950), FP64.
 *
 * The operation is the one of Rodrigues et al., "Parallel Sparse Matrix
 * Solver on the GPU Applied to Simulation of Electrical Machines":
 *   - section I: solve A x = b, A square, symmetric, positive definite and
 *     sparse, b known;
 *   - section III (algorithm): the conjugate-gradient iteration
 *       alpha = r'r / p'Ap ; x += alpha p ; stop if converged ;
 *       r -= alpha Ap ; beta = r_k'r_k / r_{k-1}'r_{k-1} ; p = r + beta p
 *     with the single product Ap of each iteration computed by a sparse
 *     matrix-vector product;
 *   - section III (storage): A held in full CSR, or -- exploiting symmetry,
 *     A = L + D + U with U' = L -- only one triangle plus the diagonal, the
 *     product then being the stored triangle read by rows plus the same
 *     arrays read by columns (the paper's "SCSR" and "SCSC" kernels); the
 *     abstract also names CSC storage.
 *
 * Readings where the paper is silent: convergence is ||r_k||_2 <= tol*||b||_2
 * on the recursively updated residual, tested after the r update; r0 is
 * b - A x0; the loop bound is maxit; p'Ap <= 0 (or non-finite) stops with
 * CG_ERR_BREAKDOWN; the iteration count is the number of products Ap made
 * inside the loop.
 *
 * Conventions for every call
 *   - indices are int32, values float64; index_base 0 or 1 (the paper's
 *     arrays are 1-based) is converted once at creation;
 *   - host pointers are read during the call only and never retained;
 *   - device pointers (b, x, y) point to n float64 values in device memory
 *     of the current HIP device (for example torch.Tensor.data_ptr() of a
 *     ROCm tensor) and must stay valid until the work on the handle's
 *     stream that uses them has finished;
 *   - functions return a cg_status; no exception crosses the boundary;
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef CGMI_H
#define CGMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cg_handle cg_handle; /* opaque, owned by the library */

/* storage formats */
enum {
    CG_FMT_CSR = 0,     /* full matrix by rows: ptr = rowptr[n+1], idx = column of each entry */
    CG_FMT_SYM_CSR = 1, /* symmetric: upper triangle incl. diagonal by rows (j >= i; each row
                           starts with its diagonal). The same arrays are the CSC of the lower
                           triangle L + D, i.e. the paper's symmetric storage. */
    CG_FMT_CSC = 2      /* full matrix by columns: ptr = colptr[n+1], idx = row of each entry */
};

/* status codes: 0 success, > 0 warning (x holds the last iterate), < 0 error */
typedef enum {
    CG_OK = 0,
    CG_NOT_CONVERGED = 1,  /* maxit products done without meeting tol */
    CG_ERR_ARG = -1,       /* bad argument (null pointer, bad enum, tol < 0, ...) */
    CG_ERR_STRUCTURE = -2, /* malformed sparse structure (see cg_create) */
    CG_ERR_BREAKDOWN = -3, /* p'Ap <= 0 or non-finite: A is not SPD (x = last iterate) */
    CG_ERR_NONFINITE = -4, /* NaN / Inf in the values or in b */
    CG_ERR_NOMEM = -5,     /* host or device allocation failed */
    CG_ERR_HIP = -6,       /* a HIP runtime call failed (detail in cg_last_error) */
    CG_ERR_UNSUPPORTED = -7 /* structure the scatter plan cannot colour (> 64 colours) */
} cg_status;

/* cg_create flags */
#define CG_CHECK_SYMMETRY 1u /* CSR / CSC: require A == A' exactly (pattern and bits) */
#define CG_MIXED 2u          /* also keep an FP32 copy of D^-1/2 A D^-1/2 (D = diag A, which must be
                                positive) for cg_solve_mixed */
#define CG_LOWER 4u          /* CG_FMT_SYM_CSR given as the paper stores it: the LOWER triangle incl.
                                diagonal by rows (j <= i, each row ends with its diagonal); converted
                                exactly to the upper layout at creation (same arrays as CSC of D + U) */

typedef struct {
    int32_t iters;      /* products Ap inside the loop (0 if the start already met tol) */
    int32_t status;     /* the cg_status also returned by cg_solve */
    double relres;      /* ||r_k||_2 / ||b||_2 of the recursive residual */
    double relres_true; /* ||b - A x||_2 / ||b||_2 of the returned x (one extra product) */
    double ms;          /* host wall time of the call, milliseconds */
    int32_t outer;      /* cg_solve_mixed: refinement steps (0 for cg_solve) */
    int32_t reserved;
} cg_info;

/* Plan summary (host-side description of how the product is executed). */
typedef struct {
    int64_t n;
    int64_t nnz;             /* stored entries */
    int32_t format;
    int32_t lanes_per_line;  /* lanes that share one row / column in the product */
    int32_t spmv_blocks;     /* workgroups (= dot-product partials) of one product */
    int32_t vec_blocks;      /* workgroups of the vector kernels */
    int32_t colors;          /* scatter formats: colour phases per product; CSR: 0 */
    int32_t scatter_blocks;  /* scatter formats: blocks of the plan (sizes of cg_analyze_export) */
    int32_t max_block_entries;
    int32_t slices;          /* 1 = sliced layout (CSR: 64-row slices; CSC: 64-slot slices;
                                symmetric CSR: blocks stored k-th entry first); 2 = CSR or CSC
                                slices whose columns are stored as 16-bit offsets from the row
                                the line adds to (every column within 32767 of it) */
    int32_t cached_loads;    /* 1 = the sliced product reads the matrix with ordinary loads, so that
                                it stays in the Infinity Cache between iterations (small enough);
                                0 = non-temporal loads */
    int32_t compact;         /* symmetric CSR: 1 = compact blocks grown on the graph of A (each block
                                stores its own rows, parks the rest); 0 = coloured line ranges, or,
                                with slices != 0, the triangle expanded into full-row slices (systems
                                whose vector kernels have at most 256 workgroups, n <= 65 536) */
    int64_t slots;           /* scatter formats: total (block, target) write slots */
    int64_t plan_bytes;      /* device bytes of the plan beyond ptr / idx / vals */
    int64_t parked;          /* scatter formats: slot sums parked and added by the row pass */
    int64_t device_bytes;    /* every device byte the handle holds (matrix, plan, work vectors) */
} cg_plan_stats;

/*
 * cg_create -- copy A to the device and plan its product.
 * The paper's problem (section I: A sparse, symmetric positive definite,
 * known) in the storage of section III: full CSR, or the symmetric storage
 * of one triangle plus the diagonal (given as the paper keeps it with
 * CG_LOWER, 1-based with index_base 1 -- section III reads its matrices from
 * files in full or symmetric CSR); CSC as the abstract names it.  The plan
 * replaces the paper's atomic updates of the transpose product (section III,
 * SCSC kernel) by an atomic-free one (compact blocks or coloured line ranges
 * for symmetric CSR, two-colour column panels for CSC).
 *   out         receives the handle (NULL on error; nothing is leaked)
 *   format      CG_FMT_*
 *   n           order of A (n >= 0; n == 0 is an empty system)
 *   ptr         host, n+1 int32: line pointers, ptr[0] == index_base,
 *               non-decreasing, ptr[n] - index_base = nnz < 2^31
 *   idx         host, nnz int32: index of each entry, in [base, base+n),
 *               strictly increasing within a line (sorted, no duplicates)
 *   vals        host, nnz float64, all finite
 *   index_base  0 or 1
 *   flags       0 or CG_CHECK_SYMMETRY | CG_MIXED | CG_LOWER
 * Errors: CG_ERR_ARG (also: CG_MIXED with a diagonal entry <= 0 or missing),
 * CG_ERR_STRUCTURE (rules above; for CG_FMT_SYM_CSR every
 * row must start with its diagonal), CG_ERR_NONFINITE, CG_ERR_NOMEM,
 * CG_ERR_HIP, CG_ERR_UNSUPPORTED.  Blocks the host (planning and upload).
 */
int cg_create(cg_handle **out, int format, int64_t n, const int32_t *ptr, const int32_t *idx,
              const double *vals, int index_base, uint32_t flags);

/* Stream for all later work of the handle (a hipStream_t; NULL = the null
 * stream).  Always stream-ordered with the caller's own work on it. */
int cg_set_stream(cg_handle *h, void *hip_stream);

/* Iterations captured per graph launch in cg_solve (default 32, 1..4096;
 * rounded up to even where two kernels run per iteration, small systems).
 * Only affects scheduling, never the result.  The inner solves of
 * cg_solve_mixed use at most 8 per launch. */
int cg_set_batch(cg_handle *h, int32_t iters_per_launch);

/*
 * cg_solve -- CG from x0 to ||r||_2 <= tol ||b||_2 or maxit products.
 * The iteration of section III (alpha = r'r / p'Ap, x += alpha p,
 * r -= alpha Ap, beta = r'r / r_old'r_old, p = r + beta p), with the one
 * product Ap per iteration of that section and every scalar kept on the
 * device -- the paper moves only the scalars between host and GPU; here the
 * host reads a status word once per launched group of iterations.
 *   b     device, n float64 (read only)
 *   x     device, n float64: in x0, out the solution / last iterate; a
 *         buffer distinct from b (CG_ERR_ARG otherwise).
 *         Untouched on CG_ERR_ARG and CG_ERR_NONFINITE; set to 0 when b == 0.
 *   tol   >= 0, relative to ||b||_2
 *   maxit >= 0
 *   info  may be NULL
 * Returns CG_OK, CG_NOT_CONVERGED, CG_ERR_BREAKDOWN, CG_ERR_NONFINITE,
 * CG_ERR_ARG or CG_ERR_HIP.  Blocks the host until the result is known; all
 * device work runs on the handle's stream.
 */
int cg_solve(cg_handle *h, const double *b, double *x, double tol, int32_t maxit, cg_info *info);

/*
 * cg_solve_mixed -- FP64 iterative refinement around FP32 inner CG solves.
 * The paper runs the same CG in single precision (section IV, Tesla C870)
 * and in double precision; here the product and the search directions of
 * the inner CG use FP32 storage (the FP32 copy of D^-1/2 A D^-1/2 made at
 * cg_create with CG_MIXED, FP32 p), while the residual b - A x (FP64
 * product), all dot products and the alpha / beta recurrences stay FP64:
 *   r = b - A x ; repeat { solve (D^-1/2 A D^-1/2) c = D^-1/2 r by CG to
 *   ||r_c|| <= inner_tol ||D^-1/2 r|| ; x += D^-1/2 c ; r = b - A x }
 *   until ||r|| <= tol ||b|| (the TRUE residual).  After an inner solve
 *   that converged, the next one starts from the replaced residual but keeps
 *   the search direction (residual replacement, as in reliable-update
 *   Krylov solvers), so the refinement steps do not restart the iteration.
 *   b, x, tol    as in cg_solve
 *   maxit        >= 0: inner iterations allowed in total
 *   inner_tol    in (0, 1); 1e-2 was fastest on the 160^3 FEM system
 *   max_outer    >= 1: refinement steps allowed
 * Returns CG_OK, CG_NOT_CONVERGED (maxit or max_outer reached, x = last
 * iterate), CG_ERR_BREAKDOWN (an inner solve broke down before any
 * progress), CG_ERR_NONFINITE, CG_ERR_ARG (also: handle created without
 * CG_MIXED) or CG_ERR_HIP.  info->iters counts inner iterations,
 * info->outer refinement steps, info->relres = info->relres_true.
 */
int cg_solve_mixed(cg_handle *h, const double *b, double *x, double tol, int32_t maxit, double inner_tol,
                   int32_t max_outer, cg_info *info);

/*
 * Batched solves: many independent SPD systems of uneven size, each with
 * nrhs right-hand sides, advanced together by one sequence of kernels
 * replayed from a HIP graph; every (system, right-hand side) pair has its own
 * CG scalars and stopping test (the iteration of section III, per pair).
 *   nsys      >= 1 systems
 *   sys_off   host, nsys+1 int64: rows of system s are [sys_off[s], sys_off[s+1])
 *             (sys_off[0] = 0, strictly increasing)
 *   ptr, idx, vals  host CSR of the block-diagonal matrix (global indices;
 *             every column of a row lies inside the row's system), rules of
 *             cg_create for CG_FMT_CSR
 *   nrhs      1, 2 or 4; vectors are interleaved: entry (i, r) at i*nrhs + r
 * Errors as cg_create, plus CG_ERR_STRUCTURE for a row coupling two systems.
 */
typedef struct cg_batch cg_batch;
int cg_batch_create(cg_batch **out, int32_t nsys, const int64_t *sys_off, const int32_t *ptr, const int32_t *idx,
                    const double *vals, int32_t nrhs, int index_base);
int cg_batch_set_stream(cg_batch *h, void *hip_stream);
/* Y = A X for all systems and right-hand sides (device, N*nrhs float64 each). */
int cg_batch_spmm(cg_batch *h, const double *X, double *Y);
/* Project-written autotuner: times the product for every schedule -- row
 * blocks of 256, 512 or 1024 entries summed through LDS, or 8 or 16 lanes
 * per row combined by butterflies, or one lane per row over 64-row slices of
 * each system (entries paired side by side; columns as 16-bit offsets from
 * the row when every one lies within 32767 of it) -- x workgroup budget (1024, 2048,
 * 4096; twice that for the slices), keeps the fastest plan and reports it
 * (outputs may be NULL; lanes_per_row = 0 means the LDS row-block schedule,
 * 1 the slices, whose entries_per_block is 0).  Uses the GPU. */
int cg_batch_autotune(cg_batch *h, int32_t *entries_per_block, int32_t *lanes_per_row, int32_t *workgroups,
                      float *best_us);
/* Solves all pairs from X (in: x0, out: solutions) to ||r|| <= tol ||b|| each.
 *   B, X      device, N*nrhs float64, interleaved
 *   iters, status  host, nsys*nrhs int32 each (pair s*nrhs + r), may be NULL:
 *             per-pair iteration count and cg_status
 *   info      aggregate: iters = max over pairs, status = worst pair status,
 *             relres / relres_true = max over pairs
 * Returns the worst status (CG_OK if every pair converged). */
int cg_batch_solve(cg_batch *h, const double *B, double *X, double tol, int32_t maxit, int32_t *iters,
                   int32_t *status, cg_info *info);
void cg_batch_destroy(cg_batch *h);
/* Detail of the last error on h; with h == NULL, of the calling thread's last
 * failed cg_batch_create.  Never NULL. */
const char *cg_batch_last_error(const cg_batch *h);

/* y = A x (device pointers, n float64 each, x and y must not overlap):
 * the sparse matrix-vector product of section III in the handle's storage
 * (CSR: one sum per row; symmetric: the stored triangle by rows plus its
 * mirror by columns; CSC: column scatter).  Asynchronous on the handle's
 * stream. */
int cg_spmv(cg_handle *h, const double *x, double *y);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as cg_spmv -- same kernels, same bits -- with its scratch (the
 * workgroups' dot partials and, for symmetric CSR and CSC, the parked sums
 * of the row pass) in a fixed 32 MiB array in device memory instead of the
 * handle's buffers.  Calls no hipMalloc / hipFree or other allocating
 * routine (the first call on a device looks the array's address up once).
 * Every call on one GPU shares that GPU's array, so calls whose products
 * overlap on one GPU (other streams, other threads, other handles) race; the
 * array keeps the last call's contents and needs no clearing (every value a
 * product reads it writes first).
 *   h     handle whose device is the current device
 *   x, y  device pointers, n float64 each, not overlapping
 * Errors: CG_ERR_ARG if h / x / y is NULL, x == y, the current device is not
 * the handle's, or the product needs more scratch than the array holds
 * (8 bytes per dot partial plus 8 per parked sum: n of them for CSC,
 * cg_plan_stats.parked for symmetric CSR; about 4M rows of CSC);
 * CG_ERR_HIP.  Asynchronous on the handle's stream.
 */
int cg_spmv_static(cg_handle *h, const double *x, double *y);

/*
 * Differentiating the solve.  For x = A^-1 b and a loss L(x), the adjoint
 * lam = A^-1 dL/dx (A symmetric, so a second cg_solve on the same handle)
 * gives dL/db = lam and dL/dA_ij = -lam_i x_j; nothing from the forward
 * iterations is kept.  (The paper's solver is section III's CG; these two
 * calls make it usable inside a gradient-based outer loop.)
 *
 * cg_set_values -- replace the values of the handle's matrix, structure
 * unchanged (no re-planning).
 *   vals  device, nnz float64, in the entry order of the arrays given to
 *         cg_create (also for CG_LOWER input); read before the call's work
 *         on the handle's stream ends
 * Enqueued on the handle's stream.  With CG_MIXED the FP32 scaled copy is
 * rebuilt too, and the call blocks until it is done: CG_ERR_ARG if a line
 * then lacks a positive, finite diagonal (the FP32 copy is then unusable until
 * the next successful call).  Values are not checked for finiteness.
 */
int cg_set_values(cg_handle *h, const double *vals);

/*
 * cg_pattern_grad -- dL/d(stored value) for every stored entry, given the
 * adjoint lam and the solution x (device, n float64 each):
 *   CSR, CSC:       grad[k] = -lam_i x_j for the entry (i, j)
 *   symmetric CSR:  the stored u_ij (i < j) stands for A_ij and A_ji, so
 *                   grad[k] = -(lam_i x_j + lam_j x_i); diagonal -lam_i x_i
 *   grad  device, nnz float64, written in the caller's entry order
 * Asynchronous on the handle's stream.
 */
int cg_pattern_grad(cg_handle *h, const double *lam, const double *x, double *grad);

/*
 * Finite-element operator with one coefficient per element: linear
 * tetrahedra, A(nu) = sum_e nu_e K_e with K_e[a][b] = |T_e| grad(phi_a) .
 * grad(phi_b) (the stiffness matrix of a magnetostatic / electrostatic model,
 * nu = reluctivity), rows and columns of Dirichlet vertices removed.  The
 * paper's systems are of this kind (abstract and section I: finite-element
 * models of Maxwell's equations; section III: the SPD matrix solved).
 *
 * cg_fem_create -- plan the operator.
 *   npts    points (>= 0); coords host, 3*npts float64 (x, y, z), finite
 *   nelem   elements (0 <= nelem < 2^27); tets host, 4*nelem int32 point ids
 *   dof     host, npts int32: the unknown of each point in [0, n), or -1 for
 *           a Dirichlet point (value 0, no row)
 *   n       unknowns (rows of A)
 * Builds on the host the full-CSR pattern of A (entry (i, j) iff an element
 * has unknowns i and j; columns sorted) and, per entry, the list of element
 * contributions in ascending element order; on the device the element
 * matrices K_e (10 distinct values each).  Errors: CG_ERR_ARG (sizes, ids,
 * an element of zero or non-finite volume, > 2^31 entries), CG_ERR_NONFINITE
 * (coordinates), CG_ERR_NOMEM, CG_ERR_HIP.  Blocks the host.
 */
typedef struct cg_fem cg_fem;
int cg_fem_create(cg_fem **out, int64_t npts, const double *coords, int64_t nelem, const int32_t *tets,
                  const int32_t *dof, int64_t n);
int cg_fem_set_stream(cg_fem *f, void *hip_stream);
/* The pattern: *nnz; rowptr host n+1 int32 and col host nnz int32 (each may
 * be NULL, e.g. to ask for nnz first).  0-based. */
int cg_fem_pattern(const cg_fem *f, int64_t *nnz, int32_t *rowptr, int32_t *col);
/* vals = A(nu) on the pattern (device: nu nelem float64, vals nnz float64);
 * each value summed over its contributions in the fixed list order.
 * Asynchronous on the operator's stream. */
int cg_fem_assemble(cg_fem *f, const double *nu, double *vals);
/* grad_e = dL/dnu_e = -lam_e' K_e x_e (device: lam, x n float64; grad nelem
 * float64); Dirichlet vertices contribute 0.  Asynchronous. */
int cg_fem_nu_grad(cg_fem *f, const double *lam, const double *x, double *grad);
void cg_fem_destroy(cg_fem *f);
/* Detail of the last error on f; with f == NULL, of the calling thread's last
 * failed cg_fem_create.  Never NULL. */
const char *cg_fem_last_error(const cg_fem *f);

/* Plan summary of a handle. */
int cg_get_stats(const cg_handle *h, cg_plan_stats *stats);

/* Frees every device and host resource of the handle (NULL is a no-op).
 * Waits for the handle's outstanding work first.  (Lifetime management has
 * no counterpart in the paper, whose program holds one matrix from file read
 * to solution -- section III.) */
void cg_destroy(cg_handle *h);

/* Static text for a status code. */
const char *cg_status_string(int status);

/* Detail of the last error on h; with h == NULL, of the calling thread's last
 * failed cg_create / cg_analyze.  Never NULL (empty string if none). */
const char *cg_last_error(const cg_handle *h);

/*
 * Host-only planning, no GPU needed: validate the structure exactly as
 * cg_create does and report the plan it would build.  vals may be NULL
 * (then the finiteness check is skipped).  Same errors as cg_create.
 */
int cg_analyze(int format, int64_t n, const int32_t *ptr, const int32_t *idx, const double *vals,
               int index_base, uint32_t flags, cg_plan_stats *stats);

/*
 * Host-only export of the scatter plan of CG_FMT_SYM_CSR / CG_FMT_CSC
 * (colour of every block, its line and entry range, and its write slots),
 * so the plan can be checked independently.  Arrays sized from cg_analyze:
 *   blk_color, blk_line0, blk_line1      [scatter_blocks]  int32
 *   blk_entry0, blk_entry1               [scatter_blocks]  int32 (0-based)
 *   blk_slot0                            [scatter_blocks+1] int64: slots of block b
 *                                        are [blk_slot0[b], blk_slot0[b+1])
 *   slot_target                          [slots] int32: row of y written
 *   slot_flags                           [slots] uint8: bit0 first writer of
 *                                        that row, bit1 last writer
 *   slot_count                           [slots] int32: products summed into it
 * Returns CG_ERR_ARG for CG_FMT_CSR and CG_FMT_CSC (see cg_analyze_panels)
 * and for a symmetric matrix planned in compact blocks (cg_analyze_compact).
 */
int cg_analyze_export(int format, int64_t n, const int32_t *ptr, const int32_t *idx, int index_base,
                      int32_t *blk_color, int32_t *blk_line0, int32_t *blk_line1, int32_t *blk_entry0,
                      int32_t *blk_entry1, int64_t *blk_slot0, int32_t *slot_target, uint8_t *slot_flags,
                      int32_t *slot_count);

/*
 * Host-only export of the compact-block plan of CG_FMT_SYM_CSR (chosen when
 * every stored row has at most 8 entries and, unless CGMI_SYM_EXPAND=0, the
 * system has more than 65 536 rows; cg_plan_stats.compact == 1).
 * Blocks are grown on the graph of A (breadth first from the lowest free
 * row, at most 512 rows each, fewer on small systems); a block stores y for its own rows and parks
 * its sums for the other rows its mirrored products reach (the transpose
 * half of the symmetric product, section III of the paper), so no two
 * blocks write one location.  Sizes from cg_analyze: n, scatter_blocks,
 * slots.
 *   block_of     [n] int32: block of each row
 *   blk_slot0    [scatter_blocks+1] int64: slots of block b are
 *                [blk_slot0[b], blk_slot0[b+1])
 *   blk_lines    [scatter_blocks] int32: its own rows = its first slots
 *   slot_target  [slots] int32: row of y each slot adds to
 *   slot_count   [slots] int32: mirrored products summed into the slot
 * Any output may be NULL.  Returns CG_ERR_ARG if the plan of these arrays is
 * not compact (other formats, or a row longer than 8 entries).  Same errors
 * as cg_analyze otherwise.
 */
int cg_analyze_compact(int64_t n, const int32_t *ptr, const int32_t *idx, int index_base, int32_t *block_of,
                       int64_t *blk_slot0, int32_t *blk_lines, int32_t *slot_target, int32_t *slot_count);

/*
 * Host-only export of the CSC plan ("column panels"), so it can be checked
 * independently.  The columns are cut into panels of `width` >= 2 bw + 1
 * columns (bw = the largest |i - j| of an entry), so panels k and k + 2 never
 * write the same row; even panels are colour 0, odd panels colour 1.  Inside
 * a panel the entries are ordered by row, then column; a slot is one (panel,
 * row) pair and its entries are contiguous.  Sizes from cg_analyze on
 * CG_FMT_CSC: nnz, slots, scatter_blocks (= chunks).
 *   width         *int64 panel width in columns
 *   entry_src     [nnz] int32: 0-based position in idx of each entry, panel order
 *   slot_target   [slots] int32: row written by the slot
 *   slot_ptr      [slots+1] int32: the slot's entries, panel order
 *   slot_panel    [slots] int32: panel of the slot
 *   chunk_slot    [chunks+1] int32: slots of each workgroup chunk
 *   first_parked  *int32: slots from here on are colour 1 (their sums are
 *                 parked, then added to y row by row)
 * Any output may be NULL.  Same errors as cg_analyze.
 */
int cg_analyze_panels(int64_t n, const int32_t *ptr, const int32_t *idx, int index_base, int64_t *width,
                      int32_t *entry_src, int32_t *slot_target, int32_t *slot_ptr, int32_t *slot_panel,
                      int32_t *chunk_slot, int32_t *first_parked);

#ifdef __cplusplus
}
#endif

#endif /* CGMI_H */

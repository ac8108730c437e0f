/*
 * mskm.h -- C ABI of the MI355X (gfx950) multiscale kernel solver.
 *
 * The library computes the monolithic kernel-based multiscale approximation of
 * Lot & Rieger, "Efficiently parallelizable kernel-based multi-scale algorithm"
 * (arXiv 2503.04914):
 *
 *   given nested (or arbitrary) point sets X_1, ..., X_L in R^d (d = 2, 3),
 *   support radii delta_1, ..., delta_L and samples f|X_l, find coefficients
 *   alpha^(l) such that the block-lower-triangular system T_L alpha = f of
 *   eq. (bigt) holds, with blocks
 *       B_{k,j}[i][n] = phi(||x_i^(k) - x_n^(j)|| / delta_j),   A_l = B_{l,l},
 *   phi = phi_{3,1}(r) = (1-r)_+^4 (4r+1) (Section 5). The solve follows the
 *   split D alpha = beta, T' beta = f of eq. (split): Jacobi sweeps on T'
 *   (Theorem jacobi) whose inner solves, like the final D alpha = beta, are
 *   per-level conjugate gradients on the SPD blocks A_l (Theorem cg), all
 *   levels in one launch. The approximant is
 *       f_L(y) = sum_l sum_n alpha_n^(l) phi(||y - x_n^(l)|| / delta_l)
 *   (eq. (fapproximation)).
 *
 * Conventions
 *   - Kernel scaling: unit peak, phi(||x-y||/delta). The paper's eq.
 *     (kernelscaling) carries an extra factor delta^-d; its coefficients are
 *     delta_l^d times the ones returned here. The approximant is identical.
 *   - Support: (i, n) is a structural nonzero iff d2 < delta_j*delta_j with
 *     d2 = dx*dx + dy*dy (+ dz*dz) evaluated left to right in FP64, each
 *     operation rounded separately (no fused multiply-add).
 *   - Indexing: "global input index" = position in the concatenated point
 *     array (level 0 first). Level l occupies [level_offsets[l],
 *     level_offsets[l+1]).
 *   - Multi-RHS vectors are row-major [N][nrhs] (point-major).
 *
 * Ownership and memory
 *   - The caller owns every buffer it passes and allocates every output.
 *   - Without MSKM_IO_DEVICE, array arguments are host pointers and calls
 *     return after the results are in host memory.
 *   - With MSKM_IO_DEVICE in the call's flags, f / alpha / query / out
 *     arguments are device pointers on the context's device (for instance
 *     torch tensors); work is issued on the context stream. Calls still wait
 *     for completion before returning (the solver reads convergence flags).
 *   - Handles are opaque; a context must not be used from two threads at once.
 *
 * Errors
 *   MSKM_OK (0) on success. Negative values: failure, outputs undefined.
 *   Positive values: warning, outputs written (MSKM_ENOCONV: tolerance not
 *   reached within the iteration caps; the report holds what was reached).
 *   mskm_last_error() returns a thread-local message for the last failure.
 */
#ifndef MSKM_H
#define MSKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSKM_ABI_VERSION 3

typedef int32_t mskm_status;
enum {
  MSKM_OK = 0,
  MSKM_ENOCONV = 1,   /* warning: tolerance not met, outputs written */
  MSKM_EINVAL = -1,   /* bad argument */
  MSKM_ENOMEM = -2,   /* device or host allocation failed */
  MSKM_EDEVICE = -3,  /* HIP runtime error */
  MSKM_ELIMIT = -4,   /* a size exceeds an index range (int32 columns etc.) */
  MSKM_ESTATE = -5    /* handle in the wrong state (e.g. no FP64 values) */
};

/* kernels */
enum { MSKM_WENDLAND_3_1 = 31 };

/* flags of mskm_hier_desc.flags */
enum {
  MSKM_POINTS_ON_DEVICE = 1 << 0, /* points is a device pointer */
  MSKM_STORE_FP64 = 1 << 1,       /* keep FP64 block values (plain path) */
  MSKM_STORE_FP32 = 1 << 2,       /* keep FP32 block values (mixed path); without
                                     STORE_FP64 also each value's FP32 rounding
                                     remainder, which the FP64 residual adds back */
  MSKM_PREFIX_NESTED = 1 << 3,    /* prefix-nested sets X_1 c X_2 c ... (Section 2):
                                     points holds only the largest level, and level
                                     l is its first level_offsets[l+1] -
                                     level_offsets[l] points */
  MSKM_SLICED_LOWER = 1 << 4      /* also keep a sliced copy of the strict lower
                                     blocks (64-row slices, one segment per coarser
                                     level, 16-bit column offsets; 6-10 more bytes
                                     per lower entry) for faster lower and full
                                     products and FP64 residuals; left out when a
                                     segment spans more than 65536 points */
};

/* flags of calls taking vectors */
enum { MSKM_IO_DEVICE = 1 << 0 };

typedef struct mskm_ctx mskm_ctx;
typedef struct mskm_hier mskm_hier;

/* ---------------------------------------------------------------- context */

/* Bind device `device` and the HIP stream `hip_stream` (a hipStream_t, or
 * NULL to let the library create its own). The context owns nothing the
 * caller passed. Fails with MSKM_EDEVICE if the device cannot be used. */
mskm_status mskm_create(int32_t device, void* hip_stream, mskm_ctx** out);
/* Frees the context, including the device and pinned blocks it keeps from
 * destroyed hierarchies (see mskm_hier_destroy). Hierarchies created on it
 * are destroyed first: they give their blocks back to it. */
mskm_status mskm_destroy(mskm_ctx* ctx);

/* Thread-local description of the last failure ("" if none). */
const char* mskm_last_error(void);

/* Library ABI version (MSKM_ABI_VERSION). */
int32_t mskm_abi_version(void);

/* -------------------------------------------------------------- hierarchy */

typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int32_t levels;               /* L >= 1 */
  const int64_t* level_offsets; /* host, [L+1], 0 = off[0] <= off[1] <= ... */
  const double* points;         /* AoS [N][dim], N = off[L]; host unless POINTS_ON_DEVICE.
                                   With PREFIX_NESTED: [P][dim], P = the largest level size */
  const double* delta;          /* host, [L], finite and > 0 */
  int32_t kernel;               /* MSKM_WENDLAND_3_1 */
  int32_t flags;                /* MSKM_POINTS_ON_DEVICE | MSKM_STORE_FP64 | MSKM_STORE_FP32 |
                                   MSKM_PREFIX_NESTED | MSKM_SLICED_LOWER;
                                   neither STORE flag means STORE_FP64 */
} mskm_hier_desc;

/* Cell lists per level, neighbour search for every level pair k >= j and
 * evaluation of all blocks B_{k,j} (Section 3) into device-resident CSR:
 * one CSR for the block diagonal D_L and one for the strict lower part
 * T_L - D_L. Points are copied; the caller may free them on return.
 * Returns once the last passes are queued on the context stream (later
 * calls on that stream run after them; mskm_hier_stats_get and
 * mskm_hier_destroy wait for them).
 * MSKM_ELIMIT if N >= 2^31 or a row would exceed 2^31 entries. */
mskm_status mskm_hier_create(mskm_ctx* ctx, const mskm_hier_desc* desc, mskm_hier** out);

/* One hierarchy object holding `count` independent hierarchies (groups), for
 * solving many uneven hierarchies in the same launches. All descriptors need
 * the same dim and storage flags; at most 4096 levels in total. Inputs and
 * outputs of later calls (f, alpha) are the groups' vectors concatenated in
 * descriptor order, each in its own input order. Internally the levels are
 * ordered depth-major, so the levels of one depth across all groups are
 * solved together; mskm_hier_level_info maps level indices to (group,
 * depth). mskm_export_* and mskm_apply work on batches; mskm_evaluate does
 * not (EINVAL). */
mskm_status mskm_hier_create_batch(mskm_ctx* ctx, const mskm_hier_desc* descs, int32_t count, mskm_hier** out);
/* Waits for the context stream, then frees the hierarchy. Its device blocks go
 * to the context's cache (up to 32 GiB) and serve later allocations of the
 * same size, so a hierarchy rebuilt with the same shape allocates nothing new;
 * the cache is emptied when an allocation would fail, and by mskm_destroy. */
mskm_status mskm_hier_destroy(mskm_hier* h);

typedef struct {
  int32_t dim, levels;
  int64_t n_total;
  int64_t nnz_diag;   /* structural nonzeros of D_L */
  int64_t nnz_lower;  /* structural nonzeros of T_L - D_L */
  int32_t has_fp64, has_fp32;
  int64_t device_bytes; /* device memory held by the hierarchy */
  double assemble_ms;   /* device time of the last assembly */
  int32_t ngroups;      /* independent hierarchies held (1 unless created as a batch) */
  int32_t sell_col16;   /* 1 when the sliced copy of D_L also holds 16-bit column offsets (variant 4064) */
  int64_t sell_entries; /* stored entries of the sliced copy of D_L, padding included */
  int32_t lower_sliced; /* 1 when the sliced copy of T_L - D_L exists (MSKM_SLICED_LOWER) */
  int64_t lower_sliced_entries; /* its stored entries, padding included */
} mskm_hier_stats;

/* The first call after creation waits for the assembly's last passes (it
 * reads assemble_ms from their events); later calls do not wait.
 * MSKM_EDEVICE when those events cannot be read. */
mskm_status mskm_hier_stats_get(const mskm_hier* h, mskm_hier_stats* out);

/* Cumulative level sizes in level order: level l holds off[l+1]-off[l]
 * points (host, [L+1]). For a single hierarchy these are the level offsets
 * it was created with. */
mskm_status mskm_hier_offsets(const mskm_hier* h, int64_t* off);

typedef struct {
  int32_t group;        /* hierarchy (descriptor index) the level belongs to */
  int32_t depth;        /* level index within its hierarchy (0 = coarsest) */
  int64_t n;            /* points */
  int64_t input_offset; /* first point in the concatenated input order */
  double delta;         /* support radius */
} mskm_level_info;

mskm_status mskm_hier_level_info(const mskm_hier* h, int32_t level, mskm_level_info* info);

/* Export block B_{row_level, col_level} (levels of one hierarchy, the column
 * level not finer than the row level; EINVAL otherwise) in
 * canonical CSR: rows in input order of level row_level, columns = input
 * index within level col_level, ascending. rowptr has N(row_level)+1
 * entries. Pass col == NULL to query the entry count into *nnz_out only.
 * val may be NULL; it receives FP64 values (or FP32 values widened when
 * only FP32 is stored). Host pointers. */
mskm_status mskm_export_block(mskm_ctx* ctx, const mskm_hier* h, int32_t row_level, int32_t col_level,
                              int64_t* rowptr, int32_t* col, double* val, int64_t* nnz_out);

/* Like mskm_export_block for the listed rows only: rows[0..nrows) are row
 * indices within level row_level (any order, repeats allowed); output row
 * r of the CSR is row rows[r]. rowptr has nrows+1 entries. Host pointers.
 * For spot checks of very large blocks. */
mskm_status mskm_export_rows(mskm_ctx* ctx, const mskm_hier* h, int32_t row_level, int32_t col_level,
                             const int64_t* rows, int64_t nrows, int64_t* rowptr, int32_t* col, double* val,
                             int64_t* nnz_out);

/* Internal (spatially sorted) order: perm[i] = global input index of
 * internal position i. Host pointer, [N]. */
mskm_status mskm_export_perm(mskm_ctx* ctx, const mskm_hier* h, int32_t* perm);

/* ------------------------------------------------------------------ apply */

enum {
  MSKM_OP_DIAG = 0,  /* y = D_L x      (block diagonal, eq. (matrix_decomposition)) */
  MSKM_OP_LOWER = 1, /* y = (T_L - D_L) x (strict lower blocks) */
  MSKM_OP_FULL = 2   /* y = T_L x      (eq. (bigt)) */
};
enum { MSKM_PREC_FP64 = 0, MSKM_PREC_FP32 = 1 };

/* y = op x with x, y [N][nrhs] in input order (FP64). prec selects which
 * stored values are applied (FP32: values and accumulation in FP32, x
 * rounded to FP32). */
mskm_status mskm_apply(mskm_ctx* ctx, const mskm_hier* h, int32_t op, int32_t prec, const double* x, int32_t nrhs,
                       double* y, int32_t flags);

/* y = op x on device vectors kept in the internal (cell-sorted) order of the
 * hierarchy (see mskm_export_perm), launched `repeats` (>= 1) times back to
 * back on the context stream. x, y: device arrays of N FP64 values for
 * MSKM_PREC_FP64 or N FP32 values for MSKM_PREC_FP32; y must not alias x.
 * avg_ms (nullable) receives the mean device time per launch from HIP events
 * recorded around the launches. Used for bandwidth measurement and by callers
 * that work in the internal order throughout. */
mskm_status mskm_apply_internal(mskm_ctx* ctx, const mskm_hier* h, int32_t op, int32_t prec, const void* x, void* y,
                                int32_t repeats, float* avg_ms);

/* Autotuner: times every CSR SpMV variant -- lanes per row 4, 8, 16, 32, 64,
 * each with per-entry loads, 16-byte loads, 16-byte non-temporal loads, and
 * with entry values recomputed in the kernel from the points (the stored
 * column structure, phi evaluated in the operator's precision) (variant
 * codes w, w + 1000, w + 2000, w + 3000), and for DIAG also the sliced
 * (SELL, 64-row slices, one row per lane) copy of the diagonal blocks, with
 * 16-bit column offsets from each slice's smallest column when every slice
 * spans at most 65536 rows (code 4064; 32-bit columns otherwise) or with
 * 32-bit columns (code 4032) -- for each operator (DIAG, LOWER, FULL) and
 * each stored precision on this hierarchy's own blocks (`repeats` >= 1
 * timed launches per variant) and keeps the fastest for later apply / solve
 * calls (the CG products use the DIAG choice). times_ms (nullable, host,
 * [3][2][22]) receives the mean
 * ms per launch of every [op][precision][variant] in that order (0 where a
 * precision is not stored or a variant does not apply).
 * The choice is also remembered by the context: hierarchies created later
 * on it with the same dimension, level count, point count and nonzero
 * counts start with the tuned widths. */
mskm_status mskm_autotune(mskm_ctx* ctx, mskm_hier* h, int32_t repeats, float* times_ms);

/* Mean device time (avg_ms, host) of the product kernel of the
 * preconditioned CG iteration (Theorem cg; q = A_l z with the dot partials
 * z.q, z.r and r.r the iteration needs) on level `level` alone, in the
 * diagonal variant chosen for prec and the vector precision of prec, launched
 * `repeats` (>= 1) times back to back between two HIP events on the context
 * stream: the launch shape of the solver's CG products, for bandwidth
 * measurement. Overwrites the hierarchy's solver workspace (no solve may be
 * in flight on it). */
mskm_status mskm_cg_product_time(mskm_ctx* ctx, mskm_hier* h, int32_t level, int32_t prec, int32_t repeats,
                                 float* avg_ms);

/* Mean device time (avg_ms, host) of the CG product of the many-right-hand-
 * side solve (Theorem cg applied to nrhs systems at once: Q = A_l P for an
 * N x nrhs block P, point-major, with the per-system partials p.q) on level
 * `level` alone, in the vector precision of prec (FP32 values and vectors,
 * or FP64), launched `repeats` (>= 1) times back to back between two HIP
 * events on the context stream: the launch shape of the solver's products.
 * nrhs in [2, 512] (MSKM_EINVAL otherwise). Allocates and frees its own P, Q
 * and partials (MSKM_ENOMEM when they do not fit). */
mskm_status mskm_mr_product_time(mskm_ctx* ctx, mskm_hier* h, int32_t level, int32_t prec, int32_t nrhs,
                                 int32_t repeats, float* avg_ms);

/* Pins the CG-product layout of the many-right-hand-side solve for nrhs
 * right-hand sides (a multiple of 64 in [64, 512]) in precision prec: chunk
 * = 64, 128, 256 or 512 right-hand sides per launch slice (dividing nrhs).
 * Without a pin the first solve with nrhs times the candidates on the
 * largest level and keeps the fastest. MSKM_EINVAL for other values. */
mskm_status mskm_set_mr_chunk(mskm_hier* h, int32_t nrhs, int32_t prec, int32_t chunk);

/* Current SpMV variant code for op (MSKM_OP_*) and prec (MSKM_PREC_*). */
mskm_status mskm_spmv_width(const mskm_hier* h, int32_t op, int32_t prec, int32_t* width);

/* Pins the SpMV variant of op / prec to `width`, one of the autotuner's
 * codes (4, 8, 16, 32, 64, plus 0, 1000, 2000 or 3000; 4064 or 4032 for DIAG), e.g. a choice saved from
 * an earlier autotune. Results do not depend on the variant beyond FP
 * summation order. MSKM_EINVAL for an unknown op, precision or code. */
mskm_status mskm_set_spmv_width(mskm_hier* h, int32_t op, int32_t prec, int32_t width);

/* ------------------------------------------------------------------ solve */

enum { MSKM_ALG_MONOLITHIC = 0, MSKM_ALG_SEQUENTIAL = 1 };
/* MSKM_PRECOND_BLOCK_JACOBI: CG on A_l preconditioned by the dense inverses
 * of A_l's diagonal blocks over the cells of the level's grid (cells of more
 * than 32 points cut into chunks); built at the first such solve and kept
 * with the hierarchy. MSKM_PRECOND_LEARNED: no preconditioner, the network's
 * prediction as each level's CG start (the same as MSKM_PRECOND_NONE with
 * warm_start = MSKM_START_LEARNED). MSKM_PRECOND_FLEX_LEARNED: the network
 * as a preconditioner applied at every iteration, z = M^-1 r + net(r) (M the
 * block-Jacobi matrix above, net(r) the network's prediction of A_l^-1 r from
 * r's stencils, see the learned warm start below), inside flexible CG
 * (Notay's FCG with one previous direction, which tolerates a preconditioner
 * that changes between iterations); sequential algorithm, one right-hand
 * side, zero start. Block-Jacobi PCG is its fallback: a level whose r.r has
 * not fallen by 4x over a window of 8 iterations drops the network for the
 * rest of its solve (counted in mskm_report.warm_fallbacks). All are build
 * extensions (the paper's CG is plain); the solution they converge to is the
 * same: the stopping test is on the true residual. */
enum {
  MSKM_PRECOND_NONE = 0,
  MSKM_PRECOND_LEARNED = 1,
  MSKM_PRECOND_BLOCK_JACOBI = 2,
  MSKM_PRECOND_FLEX_LEARNED = 3
};

/* Start of the per-level CG solves (mskm_solve_opts.warm_start):
 *   MSKM_START_ZERO      x0 = 0 (the paper's Algorithm 1);
 *   MSKM_START_PREVIOUS  Jacobi sweep m starts from sweep m-1's solution of the
 *                        same level, the final D alpha = beta from the last
 *                        sweep's (monolithic algorithm; zero elsewhere);
 *   MSKM_START_LEARNED   the network opts.mlp predicts x0 from the level's
 *                        right-hand side; combines with any precond. CG checks
 *                        it: a level with ||b - A x0|| >= ||b|| restarts from 0. */
enum { MSKM_START_ZERO = 0, MSKM_START_PREVIOUS = 1, MSKM_START_LEARNED = 2 };

typedef struct mskm_mlp mskm_mlp;

typedef struct {
  int32_t precision;      /* MSKM_PREC_FP64: plain path. MSKM_PREC_FP32: FP32 values and
                             accumulation inside, FP64 dots, FP64 residual refinement */
  int32_t algorithm;      /* MSKM_ALG_MONOLITHIC (Jacobi on T' + CG on D, eq. (split)) or
                             MSKM_ALG_SEQUENTIAL (block forward substitution, eq. (mas)) */
  double cg_rtol;         /* per-level CG stop: ||r|| <= cg_rtol * ||b|| */
  int32_t sweeps;         /* Jacobi sweeps; <= 0 means L */
  int32_t max_cg_iters;   /* cap per CG solve; <= 0 means 20000 */
  int32_t warm_start;     /* MSKM_START_ZERO, _PREVIOUS or _LEARNED */
  double target_rel_residual; /* mixed path: stop refining when ||f-T alpha||/||f|| <= this */
  int32_t max_refine;     /* mixed path: cap on refinement steps; <= 0 means 10 */
  int32_t precond;        /* MSKM_PRECOND_NONE, _BLOCK_JACOBI, _LEARNED (learned start, no preconditioner)
                             or _FLEX_LEARNED (learned preconditioner in flexible CG) */
  const mskm_mlp* mlp;    /* network for MSKM_START_LEARNED / MSKM_PRECOND_LEARNED / _FLEX_LEARNED */
  int32_t check_every;    /* CG convergence poll interval; <= 0 means 8 */
  int32_t flags;          /* MSKM_IO_DEVICE */
} mskm_solve_opts;

/* Defaults: FP64, monolithic, cg_rtol 1e-12, L sweeps, MSKM_START_ZERO, no
 * preconditioner. */
void mskm_solve_opts_default(mskm_solve_opts* o);

typedef struct {
  int32_t levels;
  int32_t sweeps_done;
  int32_t refine_steps;
  int64_t cg_iters_total;        /* sum over all CG solves and levels */
  int32_t cg_iters_last[64];     /* iterations of each level's last CG solve (levels <= 64) */
  double rel_residual;           /* ||f - T alpha|| / ||f|| (FP64), max over rhs */
  double solve_ms;               /* device time of the solve */
  int32_t warm_fallbacks;        /* learned warm starts rejected (||b - A x0|| >= ||b||), or levels
                                    whose flexible solve dropped the network */
} mskm_report;

/* alpha = T_L^-1 f per right-hand side (Section 3). f, alpha: [N][nrhs] FP64
 * in input order. With 2 <= nrhs <= 512 all right-hand sides are solved in
 * the same launches (one CG system per level and right-hand side, every
 * matrix entry applied to all of them at once; no warm start); above 512
 * they are solved one after another. rep may be NULL (cg_iters_last then
 * holds the maximum over right-hand sides, rel_residual the maximum over
 * right-hand sides and groups). MSKM_ENOCONV when a CG cap or max_refine
 * was hit. */
mskm_status mskm_solve(mskm_ctx* ctx, const mskm_hier* h, const double* f, int32_t nrhs,
                       const mskm_solve_opts* opts, double* alpha, mskm_report* rep);

/* Solves nh separately created hierarchies h[0..nh) in the same launches
 * (Section 3 for each; the levels of one depth of every hierarchy share each
 * CG launch, as in a batch object). f[g], alpha[g]: [N_g][nrhs[g]] FP64 in
 * hierarchy g's input order (host pointers, or device pointers with
 * MSKM_IO_DEVICE in opts->flags); 1 <= nrhs[g] <= 512. reps: nullable, [nh]:
 * reps[g] holds hierarchy g's levels, rel_residual (max over its right-hand
 * sides) and cg_iters_last (by depth); cg_iters_total, refine_steps and
 * solve_ms are those of the whole batch.
 * The hierarchies need the same dim and stored precisions, must not be
 * batch objects themselves, and must be distinct. The first call on a set of
 * hierarchies assembles one internal batch object from their points (device
 * memory about the sum of theirs, kept by the context and reused while the
 * same hierarchies are solved again; destroying any of them releases it).
 * Hierarchies solved with fewer right-hand sides than the largest nrhs are
 * padded with zero right-hand sides, which converge at once.
 * MSKM_ENOCONV if any hierarchy missed its tolerance. */
mskm_status mskm_solve_batch(mskm_ctx* ctx, const mskm_hier* const* h, int32_t nh, const double* const* f,
                             const int32_t* nrhs, const mskm_solve_opts* opts, double* const* alpha,
                             mskm_report* reps);

/* ||f - T_L alpha||_2 / ||f||_2 per right-hand side and per group (for a
 * batch, each hierarchy's own relative residual), FP64-accurate values
 * (eq. (bigt)). rel_out: host [nrhs][ngroups]. */
mskm_status mskm_residual(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, const double* f, int32_t nrhs,
                          double* rel_out, int32_t flags);

/* Allocation-free variant of mskm_residual, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). alpha, f: device [N][nrhs] FP64 in input order; rel_out:
 * device [nrhs][ngroups], receives ||f - T_L alpha||_2 / ||f||_2 per
 * right-hand side and group (||r||_2 where ||f||_2 = 0). All three must be
 * device memory of the context's device (MSKM_EINVAL otherwise); the caller
 * keeps ownership. The work is enqueued on the context stream and the call
 * returns without waiting: synchronise that stream before reading rel_out.
 * Nothing is allocated: the per-block partials live in a static 2 MiB device
 * array of the library (one per device, held until the process ends), so
 * hierarchies of more than 131072 row blocks of 64 rows (about 8.4M points)
 * get MSKM_ELIMIT. Calls on one device share that array: calls that overlap
 * on one device (other streams, other threads) race and must be ordered by
 * the caller. Sums differ from mskm_residual's only in summation order. */
mskm_status mskm_residual_noalloc(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, const double* f,
                                  int32_t nrhs, double* rel_out);

/* f_L at query points (eq. (fapproximation)): out[q][r] = sum over levels.
 * query: [nq][dim]; out: [nq][nrhs]. */
mskm_status mskm_evaluate(mskm_ctx* ctx, const mskm_hier* h, const double* alpha, int32_t nrhs, const double* query,
                          int64_t nq, double* out, int32_t flags);

/* ------------------------------------------------------- thresholded Jacobi
 *
 * Section 4 ("Thresholding"): the blocks of M = I - T' are frak X_{kj} =
 * B_{kj} A_j^-1 (k > j); entry (i, n) is the Lagrange function chi_n^(j) of
 * centre x_n^(j) (coefficients A_j^-1 e_n, so chi_n^(j)(x_m^(j)) = delta_nm)
 * evaluated at x_i^(k). The truncated block frak X~_{kj}(T) keeps entry
 * (i, n) iff ||x_i^(k) - x_n^(j)|| < T q_j, q_j the separation distance of
 * level j (half the smallest distance between two of its points; squared
 * distances as in the support test, compared with (T q_j)^2 in FP64), and is
 * zero elsewhere (eq. (perturbedmatrix)). The perturbed split
 * (eq. (perturbed_split)) solves (I - M~(T)) beta~ = f by Jacobi sweeps, one
 * product with the truncated blocks each and no inner solve, then
 * alpha~ = D^-1 beta~. */
typedef struct mskm_trunc mskm_trunc;

/* Builds every frak X~_{kj}(T), k > j, of hierarchy h (or of each hierarchy
 * of a batch object) on the device: q_j per level, the pattern by a cell
 * search of radius T q_j, and the values from A_j^-1 e_n computed by CG
 * (many right-hand sides, up to 512 centres per launch sequence, from zero,
 * to ||r|| <= cg_rtol) then chi_n(x_i) = sum_m B_kj[i][m] (A_j^-1 e_n)[m].
 * T = INFINITY keeps every entry (the dense M). Needs FP64 block values
 * (MSKM_ESTATE otherwise). The object keeps its own device memory (12 bytes
 * per kept entry); destroy it before or after h (after h is destroyed, the
 * calls below return MSKM_ESTATE). MSKM_ENOCONV (object returned) when a
 * coefficient solve hit its cap of 20000 iterations. MSKM_ELIMIT when a
 * level of more than 65536 points has no two points closer than its support
 * radius. */
mskm_status mskm_trunc_create(mskm_ctx* ctx, mskm_hier* h, double T, double cg_rtol, mskm_trunc** out);
mskm_status mskm_trunc_destroy(mskm_trunc* t);

/* q: host [L] separation distances (INFINITY for levels of fewer than two
 * points), nnz: kept entries over all blocks, cg_iters: CG iterations of the
 * coefficient solves (sum over centres), build_ms: device time of the build.
 * Each output is nullable. */
mskm_status mskm_trunc_info(const mskm_trunc* t, double* q, int64_t* nnz, int64_t* cg_iters, double* build_ms);

/* frak X~_{row_level, col_level}(T) in the canonical CSR of
 * mskm_export_block (rows in input order of row_level, columns = input index
 * within col_level, ascending; host arrays; col == NULL queries the count).
 * The column level must be coarser than the row level. */
mskm_status mskm_trunc_export_block(mskm_ctx* ctx, const mskm_trunc* t, int32_t row_level, int32_t col_level,
                                    int64_t* rowptr, int32_t* col, double* val, int64_t* nnz_out);

/* alpha~ of the perturbed split for one right-hand side f ([N] FP64, input
 * order; device pointers with MSKM_IO_DEVICE in opts->flags). FP64 only
 * (opts->precision = MSKM_PREC_FP64). Jacobi sweeps: opts->sweeps, <= 0
 * meaning L-1 (exact for the perturbed system, whose M~ is strictly block
 * lower); then CG on every level (opts->cg_rtol, max_cg_iters,
 * MSKM_PRECOND_NONE or _BLOCK_JACOBI). With opts->target_rel_residual > 0 (the
 * default options carry 1e-8) the perturbed solve is the inner solve of an
 * FP64 residual refinement of the exact system: alpha += alpha~(f - T_L alpha)
 * until ||f - T_L alpha|| / ||f|| <= target or max_refine rounds (MSKM_ENOCONV
 * then); with target <= 0, one perturbed solve, alpha = alpha~. rep (nullable)
 * reports sweeps per round, rounds (refine_steps), CG iterations, the final
 * FP64 relative residual of the exact system and the device time. */
mskm_status mskm_trunc_solve(mskm_ctx* ctx, const mskm_trunc* t, const double* f, const mskm_solve_opts* opts,
                             double* alpha, mskm_report* rep);

/* --------------------------------------------------------- learned warm start
 *
 * Not part of the paper (its CG starts from zero): a per-point network that
 * predicts each level's CG solution from that level's right-hand side b.
 * For point i of level l, with n_1..n_16 its 16 nearest other points of the
 * level (exact, squared FP64 distance, ties by input index; padded with i on
 * levels of fewer than 17 points):
 *   s_i  = sqrt(mean of b^2 over {i, n_1..n_16})
 *   feat = [b_i/s, (b_{n_m}/s, (x_{n_m} - x_i)/delta_l) for m = 1..16],
 *          zero-padded to a multiple of 8 (56 values in 2-D, 72 in 3-D)
 *   x0_i = s_i * (w2 . relu(W1 feat + b1) + b2), 64 hidden units; x0_i = 0
 *          where s_i = 0.
 * The first layer runs on BF16 MFMA with FP32 accumulation. CG starts from
 * x0 and decides convergence itself: a level with ||b - A x0|| >= ||b|| restarts from
 * zero (counted in mskm_report.warm_fallbacks). */
typedef struct {
  const mskm_hier* h;  /* hierarchy whose solves generate the training pairs */
  const double* f;     /* [N][nrhs] training right-hand sides (input order) */
  int32_t nrhs;        /* >= 1 */
  int64_t samples;     /* per-point (stencil -> correction / s) samples drawn, spread over the rhs */
  int32_t steps;       /* Adam steps, mini-batch 128 */
  float lr;            /* Adam step size (e.g. 1e-3) */
  uint64_t seed;       /* initial weights and sample positions */
  double cg_rtol;      /* tolerance of the plain FP64 solves that produce the pairs */
  int32_t flags;       /* MSKM_IO_DEVICE: f is a device pointer */
} mskm_train_desc;

/* Trains a network on pairs the method itself generates: each rhs is solved
 * by the plain FP64 sequential algorithm; level l contributes the pair
 * (b_l = f_l - sum_{k<l} B_{l,k} alpha_k, alpha_l). Sample points are drawn
 * uniformly over all points (SplitMix64(seed)). loss_log (nullable, host)
 * receives the mini-batch MSE (before the update) of steps 0, 50, 100, ...:
 * ceil(steps / 50) floats. */
mskm_status mskm_mlp_train(mskm_ctx* ctx, const mskm_train_desc* desc, mskm_mlp** out, float* loss_log);
mskm_status mskm_mlp_destroy(mskm_mlp* m);

/* Trains network m in place on caller-given samples, with the schedule of
 * mskm_mlp_train: Adam (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps
 * 1e-8) from zero moment estimates on the mean squared error of the network
 * output (before the s scaling) against y; step b (0-based) takes the rows
 * (128 b + q) mod ns, q = 0..127. The first layer computes with the
 * BF16-rounded weights and features that inference uses, and its gradient,
 * taken at those rounded values, updates the FP32 weights.
 *   X: [ns][F] FP32 features (F = 56 in 2-D, 72 in 3-D: the layout of the
 *      definition above), y: [ns] FP32 targets; host pointers, or device
 *      pointers with MSKM_IO_DEVICE in flags. The caller keeps ownership.
 *   loss_log: nullable host [steps], each mini-batch's MSE before its update.
 * MSKM_EINVAL for ns < 1, steps < 1, lr <= 0 or non-finite host inputs. */
mskm_status mskm_mlp_fit(mskm_ctx* ctx, mskm_mlp* m, const float* X, const float* y, int64_t ns, int32_t steps,
                         float lr, int32_t flags, float* loss_log);

/* Versioned weight blob (little endian): "MSKMMLP1", int32 dim, int32 F,
 * int32 hidden (64), then W1, b1, w2, b2 as float32. blob == NULL: *size
 * receives the byte count. */
mskm_status mskm_mlp_save(const mskm_mlp* m, void* blob, size_t* size);
mskm_status mskm_mlp_load(mskm_ctx* ctx, const void* blob, size_t size, mskm_mlp** out);

/* x0 = network prediction for b on every level (b, x0: [N] input order). */
mskm_status mskm_mlp_predict(mskm_ctx* ctx, const mskm_hier* h, const mskm_mlp* m, const double* b, double* x0,
                             int32_t flags);

/* The 16 nearest same-level points of every point of `level`, as indices
 * within the level's input order: out [n][16] (host). */
mskm_status mskm_knn_export(mskm_ctx* ctx, const mskm_hier* h, int32_t level, int32_t* out);

#ifdef __cplusplus
}
#endif
#endif /* MSKM_H */

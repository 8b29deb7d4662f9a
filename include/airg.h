/*
 * airg.h -- C ABI of the AIRG reduction multigrid library for MI355X (gfx950).
 *
 * AIRG (approximate ideal restriction with GMRES polynomials) as described
 * in Dargaville, Smedley-Stevenson, Smith & Pain, "Coarsening and
 * parallelism with reduction multigrids for hyperbolic Boltzmann
 * transport" (arXiv 2408.08262):
 *   setup (AIRG subsection, eleven-step recipe): per level a CF splitting by
 *     PMISR then DDC (CF splitting section, both algorithms), extraction of
 *     A_ff / A_fc / A_cf, a stationary GMRES polynomial q(A_ff) from a random
 *     normal rhs (gmres_poly equation) assembled with first-order fixed
 *     sparsity (fixed_sparsity equation), the approximate ideal restrictor
 *     Z = -A_cf q(A_ff) and a one-point prolongator (prolong equation), and
 *     the Galerkin operator R A P, with drop tolerances, truncation and a
 *     GMRES-polynomial coarse solve (Results: serial and parallel settings);
 *   solve: V-cycles with up F-point smoothing only, inside undamped
 *     Richardson (Results) or, for the mixed-precision form, inside FP64
 *     flexible GMRES with an FP32 V-cycle.
 *
 * Conventions for every call:
 *   - Matrices are square CSR with int32 row pointers (n+1 entries, starting
 *     at 0 and ending at nnz) and int32 column indices strictly ascending
 *     within each row, every row storing its diagonal; values are double.
 *     Exact-zero off-diagonal entries are dropped on input.
 *   - Pointers prefixed d_ are device pointers, h_ host pointers.  Inputs are
 *     borrowed for the duration of the call only; setup copies what it keeps.
 *   - Outputs are caller-allocated unless stated otherwise.
 *   - hip_stream is a hipStream_t (may be NULL for the default stream); all
 *     device work of a call is ordered on it.  Calls may synchronise the
 *     stream internally (sizes, convergence tests).
 *   - Errors are reported by status code only; airg_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.  A failed
 *     setup returns no handle.
 *   - A handle is not thread safe; distinct handles may be used on distinct
 *     streams concurrently.
 */
#ifndef AIRG_H
#define AIRG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct airg_handle airg_handle;

typedef enum airg_status {
    AIRG_OK = 0,
    AIRG_NOT_CONVERGED = 1,      /* warning: outputs hold the last iterate          */
    AIRG_ERR_INVALID_ARG = -1,
    AIRG_ERR_BAD_CSR = -2,       /* unsorted / duplicate / out-of-range / no diagonal */
    AIRG_ERR_ZERO_DIAG = -3,
    AIRG_ERR_NONFINITE = -4,
    AIRG_ERR_OOM = -5,           /* device allocation failed or device_bytes_cap hit */
    AIRG_ERR_HIP = -6,           /* HIP runtime error                               */
    AIRG_ERR_STALL = -7,         /* residual became non-finite                      */
    AIRG_ERR_LIMIT = -8          /* a size exceeds a documented kernel limit        */
} airg_status;

enum { AIRG_OUTER_RICHARDSON = 0, AIRG_OUTER_FGMRES = 1 };

/* Options.  airg_default_opts fills the paper's parallel defaults
 * (Results: strength 0.5, n_loops^max 3, drop 0.01 on Z and 0.001 on coarse
 * A, order-6 polynomial with first-order fixed sparsity, coarse solve of 3
 * iterations of an order-12 polynomial, two up F-point smooths) with
 * alpha_diag = 0.9 chosen directly. */
typedef struct airg_opts {
    int32_t struct_size;          /* sizeof(airg_opts)                                 */
    int32_t pmisr_max_rounds;     /* n_loops^max; 0 = until no node is unassigned       */
    double strong_threshold;      /* alpha of the strength definition                   */
    double ddc_threshold;         /* alpha_diag; < 0 selects the fraction rule          */
    double ddc_fraction;          /* fraction of F points converted by the fraction rule */
    double drop_R;                /* relative row drop tolerance on Z                   */
    double drop_A;                /* relative row drop tolerance on coarse operators    */
    int32_t poly_order;           /* order of q (m - 1), at most 14                      */
    int32_t poly_sparsity_order;  /* 1, 2 or 3: the powers keep the pattern of A^s      */
    int32_t coarse_poly_order;    /* polynomial order on the coarsest level, <= 14      */
    int32_t coarse_iters;         /* iterations of the coarse polynomial solve          */
    int64_t truncate_n;           /* a level with n <= truncate_n is coarsest; 0 = off  */
    int32_t max_levels;
    int32_t up_smooths;           /* F-point smooths after the coarse correction        */
    int32_t down_smooths;         /* must be 0                                          */
    int32_t precond_precision;    /* 64 or 32: precision of the V-cycle                 */
    int32_t outer;                /* AIRG_OUTER_RICHARDSON or AIRG_OUTER_FGMRES         */
    int32_t fgmres_restart;
    uint64_t seed;                /* seeds the PMISR measures and the random rhs        */
    int32_t build_adjoint;        /* 1: build the A^T hierarchy during setup            */
    int32_t onepoint_weight;      /* 0: weight 1; 1: -a_ij / a_ii                        */
    int32_t use_graph;            /* 1: replay the V-cycle as a captured HIP graph      */
                                  /* (a single hierarchy captures after its first 16    */
                                  /* cycles at a precision since the last (re)setup;    */
                                  /* the batched cycle at its first)                    */
    int32_t autotune;             /* 1: time candidate SpMM kernels per batch operator  */
    int64_t device_bytes_cap;     /* 0 = no cap; else a cap on the library's device     */
                                  /* memory in use while this setup runs                */
    int32_t coarse_matrix_free;   /* 1: the coarse polynomial is applied as q(A) x by   */
                                  /* products with A instead of an assembled matrix     */
                                  /* (truncation subsection); not in the batched form   */
    int32_t time_phases;          /* 1: time each setup phase per level on the device   */
                                  /* (phase_seconds, airg_level_info.setup_seconds);    */
                                  /* 0 (default): no timing events, which cost the      */
                                  /* setup about 3%; those times then read 0            */
} airg_opts;

typedef struct airg_solve_info {
    int32_t iterations;           /* V-cycles applied (maximum over right-hand sides)   */
    int32_t converged;            /* 1 if every right-hand side met rtol                */
    double rel_residual;          /* max over rhs of ||b - A x||_2 / ||b||_2 (FP64)     */
    double seconds;               /* device-synchronised wall time of the call          */
} airg_solve_info;

enum { AIRG_PHASE_CF = 0, AIRG_PHASE_EXTRACT, AIRG_PHASE_POLY, AIRG_PHASE_RESTRICTOR, AIRG_PHASE_PROLONG,
       AIRG_PHASE_COARSE, AIRG_PHASE_FINALIZE, AIRG_PHASE_COUNT };
typedef struct airg_level_info {
    int32_t level;
    int32_t coarsest;
    int64_t n, n_f, n_c;
    int64_t nnz_a, nnz_aff, nnz_afc, nnz_ainv, nnz_z, nnz_w;
    int32_t poly_terms;           /* coefficients kept after the breakdown test         */
    int32_t poly_requested;
    double alpha[16];             /* polynomial coefficients alpha_0 .. alpha_{m-1}     */
    double setup_seconds[AIRG_PHASE_COUNT]; /* device time of this level's setup by phase */
                                  /* (batched form: the level over all segments)         */
    int64_t setup_bytes;          /* bytes the level's setup steps must move, each step */
                                  /* reading its inputs and writing its outputs once    */
                                  /* (batched form: the level over all segments)        */
} airg_level_info;


typedef struct airg_stats {
    int32_t levels;
    int32_t reserved;
    double grid_complexity;       /* sum n_l / n_0                                      */
    double operator_complexity;   /* sum nnz(A_l) / nnz(A_0)                            */
    double storage_complexity;    /* storage equation of the Results section            */
    double setup_seconds;
    double phase_seconds[AIRG_PHASE_COUNT];
    int64_t vcycle_bytes_fp64;    /* algorithmic bytes of one V-cycle (8-byte values)   */
    int64_t vcycle_bytes_fp32;    /* same with 4-byte values                            */
    int64_t top_spmv_bytes_fp64;  /* bytes of one SpMV with the top operator            */
    int64_t device_bytes;         /* device memory held by the handle                   */
    double resetup_seconds;       /* last airg_resetup (0 before the first)             */
    int64_t vcycle_nnz;           /* stored entries of the matrices one V-cycle applies;  */
                                  /* / top_nnz = work units per cycle (WUs: the work     */
                                  /* over that of one product with the top operator,     */
                                  /* strong-tolerance subsection of the Results)         */
    int64_t top_nnz;              /* nnz(A_0)                                           */
    int64_t cycles_eager;         /* V-cycles applied since setup kernel by kernel      */
    int64_t cycles_graph;         /* ... and as replays of a captured HIP graph         */
    int64_t setup_bytes;          /* sum of the levels' setup_bytes                     */
    int64_t vcycle_index_bytes;   /* column and row-pointer bytes one V-cycle reads;    */
    int64_t vcycle_vec_entries;   /* vector entries it reads or writes per rhs: with  */
                                  /* v-byte values and k rhs a cycle moves             */
                                  /* index_bytes + v vcycle_nnz + v k vec_entries      */
} airg_stats;

/* Fills *opts with the defaults above.  Returns AIRG_ERR_INVALID_ARG if
 * opts is NULL. */
airg_status airg_default_opts(airg_opts *opts);

/* Builds the AIRG hierarchy of the n x n CSR matrix (setup recipe of the
 * AIRG subsection).  nseg > 1 with h_seg_row_offsets (nseg+1 host entries,
 * 0 .. n) declares a block-diagonal batch of independent problems: each
 * segment gets its own hierarchy (its own measures, polynomial and
 * termination) and the solve runs all of them together; an entry coupling
 * two segments is AIRG_ERR_BAD_CSR.  h_seg_seeds (nullable, nseg entries)
 * overrides opts->seed per segment.  On success *out receives a handle that
 * owns all device memory it uses; on error *out is NULL. */
airg_status airg_setup(const airg_opts *opts, int64_t n, int64_t nnz, const int32_t *d_rowptr,
                       const int32_t *d_col, const double *d_val, int32_t nseg,
                       const int64_t *h_seg_row_offsets, const uint64_t *h_seg_seeds, void *hip_stream,
                       airg_handle **out);

/* Solves A x = b for nrhs right-hand sides stored row-major (n x nrhs) from a
 * zero initial guess until ||b - A x||_2 <= rtol ||b||_2 for every rhs (and
 * segment), or max_it V-cycles.  d_x is overwritten.  Returns
 * AIRG_NOT_CONVERGED (x = last iterate) when max_it is reached.  info may be
 * NULL.  A batched handle (nseg > 1) with outer = FGMRES and
 * precond_precision = 32 solves every (segment, rhs) pair at once: one FGMRES
 * per pair in FP64, all preconditioned together by the batched FP32 V-cycle
 * whose every stage is one SpMM launch over all segments (a captured HIP
 * graph when use_graph = 1); nrhs must then be 1, 2, 4 or 8.  Other options
 * solve the segments one after another. */
airg_status airg_solve(airg_handle *h, int32_t nrhs, const double *d_b, double *d_x, double rtol, int32_t max_it,
                       void *hip_stream, airg_solve_info *info);

/* Solves A^T lambda = g with an AIRG hierarchy built on A^T (the downwind
 * operator), built during setup when build_adjoint = 1 or on the first call.
 * Same conventions as airg_solve. */
airg_status airg_adjoint_solve(airg_handle *h, int32_t nrhs, const double *d_g, double *d_lambda, double rtol,
                               int32_t max_it, void *hip_stream, airg_solve_info *info);

airg_status airg_get_stats(const airg_handle *h, airg_stats *stats);

/* Numeric re-setup: the reuse of the CF splittings and symbolic products
 * across operators that share a pattern, with a padded sparsity (Results
 * section, CF splitting and strong-tolerance discussions).  d_val (device,
 * nnz doubles) holds new values for the matrix given to airg_setup: same row
 * pointers and columns, entries in the same order.  Every level keeps its CF
 * splitting and the patterns of its operator, Z and W -- an entry dropped at
 * setup stays absent, a kept one stays whatever its new size -- while the
 * values, the polynomial coefficients and Ainv are recomputed (the A^T
 * hierarchies too, when built).  The inputs are borrowed for the call.
 * Errors: AIRG_ERR_NONFINITE, AIRG_ERR_ZERO_DIAG, AIRG_ERR_INVALID_ARG for a
 * nonzero where setup found an explicit zero, or for a handle set up in the
 * batched form (segments with FGMRES and the FP32 V-cycle).  Synchronises
 * hip_stream. */
airg_status airg_resetup(airg_handle *h, const double *d_val, void *hip_stream);

/* One V-cycle of the hierarchy (V-cycle of the AIRG subsection: restrict,
 * recurse, prolong, up F-point smooths; coarse polynomial iterations on the
 * coarsest level): d_e = V(d_g), device vectors of the segment's size in
 * natural order, computed in precision 64 or 32 (FP32 operators, FP64 in and
 * out).  segment as for airg_get_level; not for the batched form. */
airg_status airg_vcycle(const airg_handle *h, int32_t segment, const double *d_g, double *d_e, int32_t precision,
                        void *hip_stream);

/* One batched FP32 V-cycle (the preconditioner of the batched solve, the
 * batched form of airg_solve): d_e = V(d_g) for nrhs right-hand sides, n x
 * nrhs row-major FP64 device vectors in natural row order, every segment's
 * rows cycled through that segment's own hierarchy, all segments and
 * right-hand sides in one SpMM launch per stage (replayed from the captured
 * HIP graph when use_graph = 1).  nrhs must be 1, 2, 4 or 8.  Only for a
 * handle in the batched form (segments with outer = FGMRES and
 * precond_precision = 32); builds the batched operators on first use, as
 * airg_solve does.  Synchronises hip_stream. */
airg_status airg_batch_vcycle(airg_handle *h, int32_t nrhs, const double *d_g, double *d_e, void *hip_stream);

/* Per-level cost of the V-cycle (the per-level solve breakdown of the
 * parallel-results section): runs reps eager cycles (no graph) at precision
 * 64 or 32 on a zero input with events around each level's own work -- the
 * restriction to the next level plus the prolongation and smoothing after
 * the coarse correction; the whole coarse solve on the coarsest level -- and
 * writes the mean device seconds per cycle of level l to h_level_seconds[l]
 * for l < min(levels, max_levels).  The events add a few microseconds per
 * level, so the sum exceeds a graph-replayed cycle's time on small levels.
 * segment as for airg_get_level; not for the batched form.  Synchronises
 * hip_stream. */
airg_status airg_vcycle_profile(const airg_handle *h, int32_t segment, int32_t precision, int32_t reps,
                                double *h_level_seconds, int32_t max_levels, void *hip_stream);
/* The same for the batched FP32 cycle of a batched-form handle with nrhs
 * right-hand sides (1, 2, 4 or 8): level l's own stages over every segment
 * (restriction, prolongation, smoothing and the coarse solves of segments
 * whose hierarchy ends on that level), eager, mean of reps cycles. */
airg_status airg_batch_vcycle_profile(airg_handle *h, int32_t nrhs, int32_t reps, double *h_level_seconds,
                                      int32_t max_levels, void *hip_stream);

/* Describes one level of one segment; h_cf (nullable, n entries) receives
 * the CF markers (1 = F, 2 = C; all 1 on the coarsest level).  segment >= 0
 * selects the forward hierarchy of that segment (0 for a single problem);
 * segment = -1 - p selects the adjoint (A^T) hierarchy of segment p, which
 * must have been built. */
airg_status airg_get_level(const airg_handle *h, int32_t segment, int32_t level, airg_level_info *info,
                           int8_t *h_cf);

/* Copies one matrix of a level to host buffers sized from airg_level_info:
 * which = 0 A_l, 1 Ainv (approximate A_ff^-1; whole-level inverse on the
 * coarsest level), 2 Z, 3 W, 4 A_ff, 5 A_fc.  Natural (unpermuted) order,
 * F/C ranks by ascending index.  Any of the three buffers may be NULL.
 * segment as for airg_get_level. */
airg_status airg_get_level_matrix(const airg_handle *h, int32_t segment, int32_t level, int32_t which,
                                  int32_t *h_rowptr, int32_t *h_col, double *h_val);

/* Cell-block helpers of the differentiable solve (the adjoint form).  The
 * operator is A(sigma) = A_0 + sum_K sigma_K M_K with a dense bs x bs block
 * M_K per cell K (row-major, ncell*bs*bs doubles in d_mass, bs <= 8), placed
 * at the CSR value positions d_pos (ncell*bs*bs int32).
 *   airg_blockdiag_axpy:     d_val[pos] = d_base[pos] + sigma_K M_K[a][b]
 *                            (other entries of d_val are left untouched);
 *   airg_blockdiag_apply:    y_K = M_K x_K (vectors of ncell*bs entries);
 *   airg_blockdiag_bilinear: out_K = scale * lam_K^T M_K u_K (ncell entries).
 * With these, b = M s, and for a loss L(u) with A^T lambda = dL/du:
 * dL/ds = M^T lambda and dL/dsigma_K = -lambda_K^T M_K u_K. */
airg_status airg_blockdiag_axpy(int64_t ncell, int32_t bs, const double *d_mass, const double *d_sigma,
                                const int32_t *d_pos, const double *d_base, double *d_val, void *hip_stream);
airg_status airg_blockdiag_apply(int64_t ncell, int32_t bs, const double *d_mass, const double *d_x, double *d_y,
                                 void *hip_stream);
airg_status airg_blockdiag_bilinear(int64_t ncell, int32_t bs, const double *d_mass, const double *d_u,
                                    const double *d_lam, double scale, double *d_out, void *hip_stream);

/* Measurement aid.  While enabled, every plain product y = A x of the outer
 * iteration with the finest operator (the FGMRES Arnoldi product, a kernel
 * instantiation of its own) is bracketed by HIP events on its stream and its
 * algorithmic bytes (12 per nonzero, 4 per row pointer, 8 per vector entry
 * read or written) are recorded.  Enabling clears the record.  Not thread
 * safe across concurrent solves. */
airg_status airg_kernel_timing(int32_t enable);

/* Totals since timing was enabled: launches, algorithmic bytes and summed
 * event-measured seconds (synchronises on the recorded events). */
airg_status airg_kernel_timing_read(int64_t *launches, double *bytes, double *seconds);

/* Releases the handle and its device memory (NULL is ignored). */
void airg_destroy(airg_handle *h);

/* Static description of a status code. */
const char *airg_status_string(airg_status st);

/* Detail message of the last error on the calling thread ("" if none). */
const char *airg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AIRG_H */

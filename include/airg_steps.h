/*
 * airg_steps.h -- the individual setup steps of AIRG as C entry points, on
 * device buffers, so that each step can be checked and used on its own.
 *
 * Same conventions as airg.h: int32 CSR with ascending columns, double
 * values, d_ = device pointer, h_ = host pointer, all work ordered on
 * hip_stream (hipStream_t, NULL = default stream), status codes only.
 * Matrices whose size is only known after the call are returned as an
 * airg_csr owned by the library (device memory), read back with
 * airg_csr_info / airg_csr_to_host and released with airg_csr_free.
 * A NULL hip_stream is the default stream.
 */
#ifndef AIRG_STEPS_H
#define AIRG_STEPS_H
#include <stdint.h>

#include "airg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct airg_csr airg_csr;

airg_status airg_csr_info(const airg_csr *A, int64_t *nrows, int64_t *ncols, int64_t *nnz);
/* Copies rowptr (nrows+1), col and val (nnz) to host; any may be NULL. */
airg_status airg_csr_to_host(const airg_csr *A, int32_t *h_rowptr, int32_t *h_col, double *h_val);
void airg_csr_free(airg_csr *A);

/* Strength of connection (CF splitting section, strength equation with
 * absolute values): d_strong[k] = 1 iff entry k = (i, j) has j != i,
 * a_ij != 0 and |a_ij| >= alpha * max_{l != i} |a_il|.  d_deg (nullable, n)
 * receives |S_i u S_i^T|, the size of the symmetrised strong neighbourhood. */
airg_status airg_strength(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                          const double *d_val, double alpha, uint8_t *d_strong, int32_t *d_deg, void *hip_stream);

/* PMISR (PMISR algorithm): measures w_i = deg_i + rand(0,1) compared as the
 * integer key (deg_i, h_i, i); d_h (nullable, n) supplies the random parts
 * h_i, otherwise they are the upper 32 bits of SplitMix64 applied to the
 * counter seed ^ (level << 40) ^ i.  Initial F = isolated nodes; each round
 * the unassigned local minima over unassigned symmetrised strong neighbours
 * join F and their unassigned neighbours join C; max_rounds = 0 runs until
 * every node is assigned, otherwise leftovers join C.  d_cf (n) receives
 * 1 = F, 2 = C; *rounds (nullable) the rounds run. */
airg_status airg_pmisr(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                       double alpha, const uint32_t *d_h, uint64_t seed, int32_t level, int32_t max_rounds,
                       int8_t *d_cf, int32_t *rounds, void *hip_stream);

/* DDC (diagonal dominance cleanup algorithm): theta_i = sum over F columns
 * j != i of |a_ij| (ascending column order) / |a_ii|; every F point with
 * theta_i > alpha_diag and theta_i != 0, or a zero diagonal, becomes C, all
 * judged on d_cf_in.  d_theta (nullable, n) gets theta_i on F rows, -1 else. */
airg_status airg_ddc(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                     double alpha_diag, const int8_t *d_cf_in, int8_t *d_cf_out, double *d_theta,
                     void *hip_stream);

/* alpha_diag from the fraction rule (end of the CF splitting section): the
 * boundary b_k = theta_max k / 1000 whose count #{theta > b_k} is closest to
 * ceil(fraction * #F), ties to the larger k. */
airg_status airg_ddc_fraction_threshold(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                                        const double *d_val, const int8_t *d_cf, double fraction,
                                        double *alpha_diag, void *hip_stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same threshold
 * as airg_ddc_fraction_threshold, bit for bit, with no device allocation.
 * theta and the counters live in a fixed array of the library on each device
 * (4 KiB + 8 B per row for at most
 * airg_ddc_fraction_threshold_noalloc_max_rows() = 2,097,152 rows, held until
 * the process ends); larger n returns AIRG_ERR_LIMIT before any device work.
 * Every call on a device shares that device's array and leaves its contents
 * behind, so calls that overlap on one device (other threads or streams)
 * race.  Synchronises hip_stream twice (two small readbacks). */
airg_status airg_ddc_fraction_threshold_noalloc(int64_t n, int64_t nnz, const int32_t *d_rowptr,
                                                const int32_t *d_col, const double *d_val, const int8_t *d_cf,
                                                double fraction, double *alpha_diag, void *hip_stream);
int64_t airg_ddc_fraction_threshold_noalloc_max_rows(void);

/* PMISR followed by DDC with the options' parameters, measures seeded by
 * opts->seed at the given level.  d_cf (n): 1 = F, 2 = C. */
airg_status airg_cf_split(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                          const double *d_val, const airg_opts *opts, int32_t level, int8_t *d_cf, int64_t *n_f,
                          int64_t *n_c, void *hip_stream);

/* Block of the 2x2 CF block form (reduction multigrid section): rows marked
 * rowsel and columns marked colsel, ranked by ascending index. */
airg_status airg_extract(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                         const double *d_val, const int8_t *d_cf, int8_t rowsel, int8_t colsel, airg_csr **out,
                         void *hip_stream);

/* y = A x for an nrows x ncols CSR matrix. */
airg_status airg_spmv(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                      const double *d_val, const double *d_x, double *d_y, void *hip_stream);

/* Normal random rhs by Box-Muller (setup step 3): b_k = sqrt(-2 ln u1)
 * cos(2 pi u2) with 53-bit uniforms u1 in (0,1], u2 in [0,1) from SplitMix64
 * on the counters seed ^ (s << 56) ^ (level << 40) ^ k, s = 1 and 2. */
airg_status airg_gauss_rhs(int64_t n, uint64_t seed, int32_t level, double *d_b, void *hip_stream);

/* R factor of the Householder QR of K diag(1/||K_c||) (setup step 5):
 * d_K is rows x cols column-major, cols <= 16; h_R (cols x cols, row-major,
 * upper triangular) and h_colnorm (cols) on the host. */
airg_status airg_tsqr_r(int64_t rows, int32_t cols, const double *d_K, double *h_R, double *h_colnorm,
                        void *hip_stream);

/* Stationary GMRES polynomial of a square A (setup steps 3-6): m
 * coefficients alpha_0..alpha_{m-1} minimising ||b - A q(A) b|| for the random
 * rhs of airg_gauss_rhs, by the power basis, TSQR and a Givens least-squares
 * solve.  h_R ((m+1)^2) and h_colnorm (m+1) nullable; *used (nullable) the
 * coefficients kept after the Krylov breakdown test. */
airg_status airg_gmres_poly(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                            const double *d_val, uint64_t seed, int32_t level, int32_t m, double *h_alpha,
                            double *h_R, double *h_colnorm, int32_t *used, void *hip_stream);

/* Assembled first-order fixed-sparsity polynomial sum_k alpha_k A~^k
 * (fixed_sparsity equation) on the pattern of A, which must store its
 * diagonal: row i of A~^k is e_i^T M_i^k on J_i = pattern(row i), M_i =
 * A(J_i, J_i).  d_out_val has nnz entries (pattern of A).  Rows longer than
 * 2048 entries return AIRG_ERR_LIMIT. */
airg_status airg_poly_fixed_sparsity(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                                     const double *d_val, int32_t nalpha, const double *h_alpha, double *d_out_val,
                                     void *hip_stream);

/* C = A B (A: m x k, B: k x ncols_b), two-phase with LDS hash rows. */
airg_status airg_spgemm(int64_t m, int64_t k, int64_t nnz_a, const int32_t *d_arp, const int32_t *d_acol,
                        const double *d_aval, int64_t ncols_b, int64_t nnz_b, const int32_t *d_brp,
                        const int32_t *d_bcol, const double *d_bval, airg_csr **out, void *hip_stream);

/* Row drop by the relative row-wise infinity norm: keep |x_rj| >= tau
 * max_j |x_rj| (and the diagonal when keep_diag); negate = 1 flips signs. */
airg_status airg_drop(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                      const double *d_val, double tau, int32_t keep_diag, int32_t negate, airg_csr **out,
                      void *hip_stream);

/* One-point prolongator block W (n_F x n_C) for the given splitting. */
airg_status airg_onepoint_w(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                            const double *d_val, const int8_t *d_cf, int32_t weight_mode, airg_csr **out,
                            void *hip_stream);

/* A^T (rows sorted). */
airg_status airg_transpose(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr,
                           const int32_t *d_col, const double *d_val, airg_csr **out, void *hip_stream);

/* One full setup level (CF split, extraction, polynomial, approximate
 * inverse, Z, W and the dropped Galerkin operator) on A.  h_alpha_in
 * (nullable, poly_order+1 values) replaces the computed coefficients;
 * h_alpha_out (poly_order+1) receives those used.  d_cf (n) receives the
 * splitting.  Any of the four outputs may be NULL. */
airg_status airg_level_build(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                             const double *d_val, const airg_opts *opts, int32_t level, const double *h_alpha_in,
                             int8_t *d_cf, double *h_alpha_out, airg_csr **ainv, airg_csr **z, airg_csr **w,
                             airg_csr **ac, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* AIRG_STEPS_H */

/*
 * airg_oracle.h -- plain CPU reference of AIRG setup and solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library; it
 * is called from the tests, the smoke check and the benchmark's CPU-baseline
 * leg, never from the product path.  It shares no code with the HIP library.
 *
 * Everything is double precision, natural (unpermuted) index order, plain
 * loops; compiled with -O2 -ffp-contract=off.  Loops over independent rows
 * may run on several threads (OpenMP); the results do not depend on the
 * thread count.  Each function names the
 * passage of Dargaville et al., "Coarsening and parallelism with reduction
 * multigrids for hyperbolic Boltzmann transport" (arXiv 2408.08262) that it
 * follows.
 *
 * CF marker convention: 0 = unassigned (internal), 1 = F point, 2 = C point.
 */
#ifndef AIRG_ORACLE_H
#define AIRG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_U = 0, ORC_F = 1, ORC_C = 2 };

typedef struct orc_csr {
    int64_t nr, nc;        /* rows, columns                          */
    int64_t *rp;           /* nr+1 row pointers                        */
    int32_t *ci;           /* column indices, ascending within a row   */
    double  *v;            /* values (NULL for a pattern-only graph)   */
} orc_csr;

typedef struct orc_params {
    double   strong_threshold;   /* alpha in the strength definition            */
    double   ddc_threshold;      /* alpha_diag; < 0 selects the fraction mode    */
    double   ddc_fraction;       /* fraction of F points converted (fraction mode) */
    int32_t  pmisr_max_rounds;   /* n_loops^max; 0 = until no node is unassigned */
    int32_t  poly_order;         /* GMRES polynomial order (m - 1)               */
    double   drop_R;             /* relative row drop tolerance on Z             */
    double   drop_A;             /* relative row drop tolerance on coarse A      */
    int32_t  coarse_poly_order;  /* polynomial order on the coarsest level       */
    int32_t  coarse_iters;       /* coarse-solve iterations                      */
    int64_t  truncate_n;         /* level with n <= truncate_n is coarsest; 0 = off */
    int32_t  max_levels;
    int32_t  up_smooths;         /* F-point smooths after the coarse correction  */
    int32_t  onepoint_weight;    /* 0: weight 1, 1: weight -a_ij / a_ii          */
    uint64_t seed;
    int32_t  poly_sparsity_order;   /* fixed sparsity of the powers: pattern of A^s */
    int32_t  coarse_matrix_free;    /* 1: coarse polynomial applied by matvecs      */
} orc_params;

void orc_default_params(orc_params *p);
/* Threads for the row-parallel loops (OpenMP); results do not depend on it. */
void    orc_set_threads(int32_t n);
int32_t orc_get_threads(void);
void orc_csr_free(orc_csr *A);

/* counter-based generator (SplitMix64 output of a keyed counter) */
uint64_t orc_splitmix64(uint64_t x);
uint64_t orc_counter(uint64_t seed, uint32_t stream, uint32_t level, uint64_t i);

/* --- CF splitting ------------------------------------------------------ */
void    orc_strength(const orc_csr *A, double alpha, uint8_t *strong);
int     orc_sym_graph(const orc_csr *A, const uint8_t *strong, orc_csr *G);
void    orc_pmisr_keys(const orc_csr *G, uint64_t seed, int32_t level, int32_t *deg, uint32_t *h);
int32_t orc_pmisr(const orc_csr *G, const int32_t *deg, const uint32_t *h, int32_t max_rounds, int8_t *cf);
double  orc_ddc_fraction_threshold(const orc_csr *A, const int8_t *cf, double fraction);
int64_t orc_ddc(const orc_csr *A, double alpha_diag, int8_t *cf, double *theta);
int     orc_cf_split(const orc_csr *A, const orc_params *p, int32_t level, int8_t *cf);

/* --- extraction, products ------------------------------------------------ */
int  orc_submatrix(const orc_csr *A, const int8_t *cf, int8_t rowsel, int8_t colsel, orc_csr *out);
void orc_spmv(const orc_csr *A, const double *x, double *y);
int  orc_spgemm(const orc_csr *A, const orc_csr *B, orc_csr *C);
int  orc_drop(const orc_csr *A, double tau, int keep_diag, orc_csr *out);
int  orc_transpose(const orc_csr *A, orc_csr *T);

/* --- GMRES polynomial ----------------------------------------------------- */
void orc_gauss_rhs(int64_t n, uint64_t seed, int32_t level, double *b);
void orc_power_basis(const orc_csr *A, const double *b, int32_t m, double *K);
void orc_householder_r(int64_t rows, int32_t cols, const double *K, double *R, double *colnorm);
int  orc_poly_coeffs_from_r(const double *R, const double *colnorm, int32_t m, double *alpha);
int  orc_gmres_poly(const orc_csr *A, uint64_t seed, int32_t level, int32_t m, double *alpha);
int  orc_poly_fixed_sparsity(const orc_csr *A, const double *alpha, int32_t nalpha, orc_csr *out);
/* The same with the row patterns J_i taken from S (plus the diagonal);
 * M_i = A(J_i, J_i).  orc_power_pattern gives the pattern of A^order. */
int  orc_poly_fixed_sparsity_pattern(const orc_csr *A, const orc_csr *S, const double *alpha, int32_t nalpha,
                                     orc_csr *out);
int  orc_power_pattern(const orc_csr *A, int32_t order, orc_csr *out);

/* --- grid transfer and coarse operator ---------------------------------- */
int orc_onepoint_w(const orc_csr *A, const int8_t *cf, int32_t weight_mode, orc_csr *W);
int orc_restrictor(const orc_csr *Acf, const orc_csr *Ainv, double drop_R, orc_csr *Z);
int orc_coarse_operator(const orc_csr *A, const int8_t *cf, const orc_csr *Z, const orc_csr *W,
                        double drop_A, orc_csr *Ac);

/* --- hierarchy, cycle and outer iterations ------------------------------ */
typedef struct orc_hier orc_hier;

/* One level of the setup, for replay: given A (and optionally the polynomial
 * coefficients alpha_in of length poly_order+1) build cf, Aff, Afc, Ainv, Z,
 * W and the coarse operator Ac.  alpha_out receives the coefficients used. */
int orc_level_build(const orc_csr *A, const orc_params *p, int32_t level, const double *alpha_in,
                    int8_t *cf, double *alpha_out, orc_csr *Ainv, orc_csr *Z, orc_csr *W, orc_csr *Ac);

orc_hier *orc_setup(const orc_csr *A, const orc_params *p);
/* orc_setup with the coefficients of levels 0 .. nlev_in-1 given:
 * alpha_in[l * ORC_ALPHA_STRIDE + k], k < m of that level (poly_order + 1,
 * or coarse_poly_order + 1 on the coarsest level). */
#define ORC_ALPHA_STRIDE 16
orc_hier *orc_setup_replay(const orc_csr *A, const orc_params *p, int32_t nlev_in, const double *alpha_in);

/* Numeric re-setup (Results: reuse of the CF splitting and symbolic products
 * with a padded sparsity).  One level: given the new values of A on the
 * level's pattern and its CF splitting, recompute the coefficients (or take
 * alpha_in), Ainv, and the values of Z, W and the coarse operator on the
 * given patterns (no drops).  The hierarchy form applies it level by level
 * to vals (the canonical level-0 pattern of h); the coarsest level takes a
 * new coarse polynomial. */
int orc_level_renumeric(const orc_csr *A, const int8_t *cf, const orc_params *p, int32_t level,
                        const double *alpha_in, const orc_csr *Wpat, const orc_csr *Zpat, const orc_csr *Acpat,
                        double *alpha_out, orc_csr *Ainv, orc_csr *Z, orc_csr *W, orc_csr *Ac);
orc_hier *orc_resetup(const orc_hier *h, const double *vals);
void      orc_hier_free(orc_hier *h);
int32_t   orc_hier_levels(const orc_hier *h);
/* which: 0 A, 1 Ainv, 2 Z, 3 W, 4 Aff, 5 Afc ; returns a borrowed pointer or NULL */
const orc_csr *orc_hier_matrix(const orc_hier *h, int32_t level, int32_t which);
const int8_t  *orc_hier_cf(const orc_hier *h, int32_t level);
const double  *orc_hier_alpha(const orc_hier *h, int32_t level, int32_t *nalpha);
void orc_vcycle(const orc_hier *h, int32_t level, const double *g, double *e);
int  orc_richardson(const orc_hier *h, const double *b, double *x, double rtol, int32_t maxit, double *relres);
int  orc_fgmres(const orc_hier *h, const double *b, double *x, double rtol, int32_t maxit, int32_t restart,
                double *relres);
/* complexities per the storage formula of the Results section */
void orc_hier_complexity(const orc_hier *h, double *grid, double *op, double *storage);

#ifdef __cplusplus
}
#endif
#endif

// Stationary GMRES polynomial of the AIRG subsection: random rhs by
// Box-Muller, power basis, tall-skinny Householder QR, least squares for the
// coefficients, and the assembled fixed-sparsity approximate inverse.
#pragma once
#include <vector>

#include "common.hpp"
#include "csr.hpp"

namespace airg {

constexpr int kMaxPolyCols = 16;   // m + 1 <= 16

struct PolyInfo {
    int m = 0;                     // coefficients requested
    int used = 0;                  // coefficients kept after the breakdown test
    double alpha[kMaxPolyCols] = {};
    double R[kMaxPolyCols * kMaxPolyCols] = {};   // scaled R factor, row-major (m+1)^2
    double colnorm[kMaxPolyCols] = {};
};

// b_k = sqrt(-2 ln u1) cos(2 pi u2), u1 in (0,1] from stream 1, u2 in [0,1)
// from stream 2 of the counter generator.
void gauss_rhs(int64_t n, uint64_t seed, int32_t level, double *b, hipStream_t s);

// R factor (row-major, cols x cols) of the column-scaled K (n x cols,
// column-major) by a tall-skinny Householder QR tree, and the column norms.
void tsqr_r(const double *K, int64_t n, int cols, double *h_R, double *h_colnorm, hipStream_t s);

// Device int32 ranges a caller wants read back with the next host
// synchronisation of a routine (to h, back to back).
struct ExtraReads {
    std::vector<const int32_t *> src;
    std::vector<int32_t> cnt;
    int32_t *h = nullptr;
};

// alpha = argmin || beta e1 - R~ y || from the scaled R and the column norms,
// with the Krylov breakdown rule; returns the number of coefficients kept.
int poly_coeffs_from_r(const double *R, const double *colnorm, int m, double *alpha);

// Steps 3-6 of the setup on a square A (alpha has m entries).  The extra
// ranges come back in the same readback as the R factor.
PolyInfo gmres_poly(const CsrView &A, uint64_t seed, int32_t level, int m, hipStream_t s,
                    const ExtraReads *extra = nullptr);

// The same for a block-diagonal batch: segment p holds rows off[p] ..
// off[p+1]-1 (host offsets; d_off the same on the device) and draws its
// random vector with d_seeds[p] at indices local to the segment.  Each
// segment gets its own column scaling, R factor and coefficients.
std::vector<PolyInfo> gmres_poly_seg(const CsrView &A, const std::vector<int32_t> &off, const int32_t *d_off,
                                     const uint64_t *d_seeds, int32_t level, int m, hipStream_t s);
void tsqr_r_seg(const double *K, const std::vector<int32_t> &off, int cols, double *h_R, double *h_colnorm,
                hipStream_t s);

// Assembled fixed-sparsity polynomial on the pattern of A (which must store
// its diagonal): row i of A~^k is e_i^T M_i^k restricted to J_i, with
// M_i = A(J_i, J_i).  out_v has A.nnz entries (pattern of A).
void poly_fixed_sparsity(const CsrView &A, const double *alpha, int nalpha, double *out_v, hipStream_t s);
// The same with the row patterns J_i taken from Pt (which holds the
// diagonal; out_v has Pt.nnz entries); M_i = A(J_i, J_i).
void poly_fixed_sparsity_pattern(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha,
                                 double *out_v, hipStream_t s);
// The same in two halves: the rows of Pt binned by length (no
// synchronisation; kFixedBins + 1 totals at plan.bins.tot), then, with those
// totals on the host, the assembly.
constexpr int kFixedBins = 8;      // rows of <= 4, 8, 16, 24, 32, 48, 64 entries, longer
constexpr int kFixedLongBin = 7;
struct FixedPlan {
    DBuf<int8_t> bin;
    BinPlan bins;
};
FixedPlan fixed_sparsity_begin(const CsrView &Pt, hipStream_t s);
void poly_fixed_sparsity_planned(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha,
                                 double *out_v, FixedPlan &plan, const int32_t *h_tot, hipStream_t s);
// The assembly's row bins of a pattern (one host synchronisation), and the
// assembly on them, for repeated assemblies on one pattern.
Bins poly_pattern_bins(const CsrView &Pt, hipStream_t s);
void poly_fixed_sparsity_binned(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha, double *out_v,
                                const Bins &bins, hipStream_t s);
// Batch form: the rows of segment p (host offsets off) use P[p]'s
// coefficients; patterns from Pt.
void poly_fixed_sparsity_seg(const CsrView &A, const CsrView &Pt, const std::vector<int32_t> &off,
                             const std::vector<PolyInfo> &P, double *out_v, hipStream_t s);
// Pattern (and values) of A^order, order 2 or 3: the sparsity order of the
// fixed-sparsity powers.
Csr power_pattern(const CsrView &A, int order, hipStream_t s);

}  // namespace airg

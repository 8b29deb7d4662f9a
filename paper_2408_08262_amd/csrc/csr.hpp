// Sparse-matrix building blocks on the device: validation, SpMV, block
// extraction under a CF splitting, row drop filter, transpose, casts.
#pragma once
#include "common.hpp"

namespace airg {

// Checks the input CSR (columns in range, strictly ascending, diagonal present
// and nonzero, values finite) and returns a canonical copy with exact-zero
// off-diagonal entries removed.  Throws Error with ST_BAD_CSR / ST_ZERO_DIAG /
// ST_NONFINITE.
Csr canonical_copy(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, hipStream_t s);

// Copy of a view into an owned matrix.
Csr copy_csr(const CsrView &A, hipStream_t s);

// y = A x (mode 0), y = z - A x (mode 1), y = y + A x (mode 2).
enum SpmvMode { SPMV_SET = 0, SPMV_ZMINUS = 1, SPMV_ADD = 2 };
void spmv(const CsrView &A, const double *x, double *y, const double *z, int mode, hipStream_t s, int lanes = 0);
void spmv32(const CsrView &A, const float *x, float *y, const float *z, int mode, hipStream_t s, int lanes = 0);
// Whether spmv/spmv32 take the CSR-stream kernel for a matrix of this shape
// (otherwise one lanes_for(nnz, nr)-lane group per row).
bool spmv_streams(int32_t nr, int64_t nnz);
// The outer iterations' products with the finest operator (a separate kernel
// instantiation), optionally timed with events; see top_timing.
void spmv_top(const CsrView &A, const double *x, double *y, const double *z, int mode, hipStream_t s);
// k right-hand sides (row-major), the batched outer product; timed like spmv_top.
void spmm_top(const CsrView &A, int k, const double *x, double *y, const double *z, int mode, hipStream_t s);
void top_timing(bool enable);
void top_timing_read(int64_t *launches, double *bytes, double *seconds);
// Same with k right-hand sides stored row-major (n x k).  lanes: -1 picks
// the kernel from the row statistics, 0 forces the persistent CSR-stream
// kernel, G > 0 forces G lanes per row.
void spmm(const CsrView &A, int k, const double *x, double *y, const double *z, int mode, hipStream_t s,
          int lanes = -1);
void spmm32(const CsrView &A, int k, const float *x, float *y, const float *z, int mode, hipStream_t s,
            int lanes = -1);

// rank[i] = position of i among the points carrying its own marker
// (F rank for F points, C rank for C points); returns (nF, nC).
std::pair<int32_t, int32_t> cf_ranks(const int8_t *cf, int32_t n, int32_t *rank, hipStream_t s);
// The same with a third class, terminal rows (CF_T), ranked among themselves.
struct CfCounts {
    int32_t nF, nC, nT;
};
// extra: device ints read back with the counts into extra_out[0..].  flags3,
// when given, holds the class indicators already (3 n ints: cf == F,
// cf == C, cf == T, as the DDC pass writes them).
CfCounts cf_ranks3(const int8_t *cf, int32_t n, int32_t *rank, hipStream_t s,
                   const std::vector<const int32_t *> &extra = {}, int32_t *extra_out = nullptr,
                   const int32_t *flags3 = nullptr);
// cf_ranks3 plus, at the segment boundaries d_off[0..na] (device, ascending,
// d_off[na] = n), the numbers of F, C and terminal rows before each boundary:
// h_bounds[3 p + {0, 1, 2}] (host, 3 (na + 1) entries).
CfCounts cf_ranks_seg(const int8_t *cf, int32_t n, int32_t *rank, const int32_t *d_off, int na, int32_t *h_bounds,
                      hipStream_t s);
// fidx[f] = original index of the f-th F point (and likewise cidx for C).
void cf_index_lists(const int8_t *cf, const int32_t *rank, int32_t n, int32_t *fidx, int32_t *cidx, hipStream_t s);

// Block of A with rows marked rowsel and columns marked colsel, ranked by
// original index, entry order preserved.
Csr extract_block(const CsrView &A, const int8_t *cf, const int32_t *rank, int8_t rowsel, int8_t colsel,
                  int32_t nrows_out, int32_t ncols_out, hipStream_t s);
// A_ff, A_fc and A_cf together (one pass, one host synchronisation).
void extract_fc_blocks(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC, Csr &Aff,
                       Csr &Afc, Csr &Acf, hipStream_t s);
// The same in two halves: the counts and their scans need only cf, so the
// three block sizes (device ints at totals()) can be read back with other
// values; extract_finish takes them (tot[0..2]) and fills the blocks.
struct ExtractPlan {
    int32_t n = 0;
    DBuf<int32_t> off;   // 3 (n + 1): exclusive scans of the per-row counts of A_ff, A_fc, A_cf
    std::vector<const int32_t *> totals() const;
};
ExtractPlan extract_begin(const CsrView &A, const int8_t *cf, hipStream_t s);
// fidx / cidx (nullable) receive the index lists of cf_index_lists.
void extract_finish(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                    const int32_t *tot, ExtractPlan &P, Csr &Aff, Csr &Afc, Csr &Acf, hipStream_t s,
                    int32_t *fidx = nullptr, int32_t *cidx = nullptr);
// The values of the three blocks again, into blocks extracted earlier with
// the same plan and splitting (A's values changed, its pattern did not).
void extract_refill(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                    const ExtractPlan &P, Csr &Aff, Csr &Afc, Csr &Acf, hipStream_t s);

// Keep entries with |x| >= tau * max_j |x_rj| (and the diagonal when
// keep_diag); negate scales every kept value by -1 when set.
Csr drop_rows(const CsrView &A, double tau, bool keep_diag, bool negate, hipStream_t s);
// The same without the host synchronisation: B.rp is complete on the device
// and B.ci / B.v have room for A.nnz entries; B.nnz is left at that upper
// bound, and the caller replaces it by B.rp[nr] once it has read it.
Csr drop_rows_bound(const CsrView &A, double tau, bool keep_diag, bool negate, hipStream_t s);

// A^T with rows sorted (deterministic).
Csr transpose(const CsrView &A, hipStream_t s);

// v -> vf (single precision copy).
void make_f32(Csr &A, hipStream_t s);

// Dot products / norms with a fixed reduction order (deterministic).
double dot(const double *x, const double *y, int64_t n, hipStream_t s);
void multi_dot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *h_out, hipStream_t s);
// The same dot products left on the device (d_out[0..nvec)), no synchronisation.
void multi_dot_dev(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *d_out,
                   hipStream_t s);
// w *= 1 / sqrt(nn_dev[0]) when that is positive.
void normalize_dev(double *w, const double *nn_dev, int64_t n, hipStream_t s);
double nrm2(const double *x, int64_t n, hipStream_t s);

// Elementwise helpers.
void axpy(double a, const double *x, double *y, int64_t n, hipStream_t s);            // y += a x
void scal_copy(double a, const double *x, double *y, int64_t n, hipStream_t s);       // y = a x
void gemv_sub(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, hipStream_t s);
// w -= V h, then d_out[j] = dot(V_j, w) for j < nvec (<= 32) on the updated w:
// one pass over V, the sums equal to gemv_sub followed by multi_dot_dev.
void gemv_sub_dots(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, double *d_out,
                   hipStream_t s);
// w -= V h, then d_nn[0] = dot(w, w): equal to gemv_sub followed by
// multi_dot_dev(w, ., 1, w, ...); nvec <= 32.
void gemv_sub_norm(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, double *d_nn,
                   hipStream_t s);
void gemv_add(const double *V, int64_t ldv, int nvec, const double *h_dev, double *x, int64_t n, hipStream_t s);
void cast_d2f(const double *x, float *y, int64_t n, hipStream_t s);
void cast_f2d(const float *x, double *y, int64_t n, hipStream_t s);
void gather_d2f(const double *x, const int32_t *idx, float *y, int64_t n, hipStream_t s);   // y[i] = x[idx[i]]
void scatter_f2d(const float *x, const int32_t *idx, double *y, int64_t n, hipStream_t s);  // y[idx[i]] = x[i]
void gather(const double *x, const int32_t *idx, double *y, int64_t n, hipStream_t s);   // y[i] = x[idx[i]]
void scatter(const double *x, const int32_t *idx, double *y, int64_t n, hipStream_t s);  // y[idx[i]] = x[i]
void gather_k(const double *x, const int32_t *idx, double *y, int64_t n, int k, int64_t ldx, int64_t ldy,
              hipStream_t s);
void scatter_k(const double *x, const int32_t *idx, double *y, int64_t n, int k, int64_t ldx, int64_t ldy,
               hipStream_t s);

// Groups row indices by a small bin id (0..nbins-1): rows[off[b] .. off[b+1])
// hold the rows of bin b (order inside a bin unspecified).  Rows with a bin
// id outside the range are skipped.
struct Bins {
    DBuf<int32_t> rows;
    std::vector<int64_t> off;
    int64_t count(int b) const { return off[b + 1] - off[b]; }
    const int32_t *list(int b) const { return rows.p + off[b]; }
};
Bins bin_rows(const int8_t *bin, int32_t n, int nbins, hipStream_t s);
// The same in two halves around the caller's own readback: begin leaves the
// bin starts (nbins + 1 values) in tot on the device; end takes them from the
// host and lists the rows.
struct BinPlan {
    const int8_t *bin = nullptr;
    int32_t n = 0, nw = 0;
    int nbins = 0;
    DBuf<int32_t> boff, tot;
};
BinPlan bin_rows_begin(const int8_t *bin, int32_t n, int nbins, hipStream_t s);
// Bins computed in the counting pass: row i's value is val[i] (or
// val[i + 1] - val[i] with diff, a row length from a row pointer), its bin the
// number of thresholds below that value, also stored in bin_out[i].
struct BinRule {
    static constexpr int kMax = 12;
    int32_t thr[kMax];
    int nthr;
};
BinPlan bin_rows_begin_rule(const int32_t *val, bool diff, const BinRule &rule, int8_t *bin_out, int32_t n, int nbins,
                            hipStream_t s);
Bins bin_rows_end(BinPlan &P, const int32_t *h_tot, hipStream_t s);

// Wavefront-scope ordering of LDS traffic among the lanes of one wave.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Keeps the compiler from moving memory accesses across this point without
// waiting for outstanding ones: a wavefront's LDS operations are carried out
// in the order they are issued, so issue order is all that the per-slot
// order of LDS accumulations needs.
__device__ inline void lds_issue_order() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
}

}  // namespace airg

// Two-phase sparse matrix product with LDS hash rows.
#pragma once
#include <utility>

#include "common.hpp"
#include "csr.hpp"

namespace airg {

// A row drop applied as a product's rows are written, with the rule of
// drop_rows: thr_i = tau * max_j |c_ij|; c_ij is kept when |c_ij| >= thr_i
// (or j == i with keep_diag), times sign.  Each row's kept entries go to the
// front of its slots of the full product, in column order, and their count
// to kcnt[row]; drop_compact then packs them.
struct DropArgs {
    double tau = 0.0, sign = 1.0;
    int32_t keep_diag = 0;
    int32_t *kcnt = nullptr;   // nullptr: no drop
};

// C = A B; columns ascending per row; each entry accumulated in ascending
// order of the contributing A entry, without fused multiply-add.
Csr spgemm(const CsrView &A, const CsrView &B, hipStream_t s);

// The same in two halves.  spgemm_begin needs only A and B's row pointers
// and width: it picks the kernel family and, for the hash rows, starts the
// row binning by product bound without a synchronisation (totals() then names
// the device range the host must read, else has no entries).  spgemm_finish
// takes those totals from the host and forms the product.
struct SpgemmPlan {
    int32_t m = 0, bnc = 0;
    bool narrow = false;
    DBuf<int32_t> ub, cnt;   // per-row bound on the product's entries; its entry counts
    DBuf<int32_t> kcnt;      // kept entries per row under a fused drop (zeroed with cnt)
    DBuf<int8_t> sbin;
    BinPlan bins;
    std::pair<const int32_t *, int32_t> totals() const;
};
SpgemmPlan spgemm_begin(const CsrView &A, const int32_t *b_rp, int32_t b_nc, hipStream_t s);
// With drop (D.kcnt taken from the plan) the rows hold their kept entries
// only, at the front of their slots; pack them with drop_compact.
Csr spgemm_finish(const CsrView &A, const CsrView &B, SpgemmPlan &P, const int32_t *h_tot, hipStream_t s,
                  const DropArgs *drop = nullptr);
// The dropped product of spgemm_finish(..., drop) packed into a CSR: the
// rows' kept counts scanned, their entries copied.  bound: no readback, the
// result's nnz is only the product's (its row pointer holds the exact count).
Csr drop_compact(const Csr &C, const int32_t *kcnt, bool bound, hipStream_t s);
// The dropped product in one call: spgemm with the drop fused, then packed
// (exact entry count); *product_nnz (nullable) receives the undropped
// product's entry count.
Csr spgemm_drop(const CsrView &A, const CsrView &B, const DropArgs &drop, hipStream_t s,
                int64_t *product_nnz = nullptr);

// out_v (Pt.nnz values, Pt's order) = sign * (A B) at the stored positions of
// the pattern Pt (Pt.nr == A.nr; rows sorted, at most 4096 entries); entries
// of the product off the pattern are not formed.  Same accumulation as spgemm.
void spgemm_on_pattern(const CsrView &A, const CsrView &B, const Csr &Pt, double sign, double *out_v,
                       hipStream_t s);
// The same in two halves: the rows of Pt binned by length once (one host
// synchronisation), then products on those bins as often as the values of A
// and B change.
Bins pattern_bins(const Csr &Pt, hipStream_t s);
void spgemm_on_pattern_binned(const CsrView &A, const CsrView &B, const CsrView &Pt, const Bins &bins, double sign,
                              double *out_v, hipStream_t s);

}  // namespace airg

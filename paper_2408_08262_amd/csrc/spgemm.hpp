// Two-phase sparse matrix product with LDS hash rows.
#pragma once
#include <utility>

#include "common.hpp"
#include "csr.hpp"

namespace airg {

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
    DBuf<int8_t> sbin;
    BinPlan bins;
    std::pair<const int32_t *, int32_t> totals() const;
};
SpgemmPlan spgemm_begin(const CsrView &A, const int32_t *b_rp, int32_t b_nc, hipStream_t s);
Csr spgemm_finish(const CsrView &A, const CsrView &B, SpgemmPlan &P, const int32_t *h_tot, hipStream_t s);

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

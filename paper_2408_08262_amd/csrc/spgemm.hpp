// Two-phase sparse matrix product with LDS hash rows.
#pragma once
#include "common.hpp"

namespace airg {

// C = A B; columns ascending per row; each entry accumulated in ascending
// order of the contributing A entry, without fused multiply-add.
Csr spgemm(const CsrView &A, const CsrView &B, hipStream_t s);

// out_v (Pt.nnz values, Pt's order) = sign * (A B) at the stored positions of
// the pattern Pt (Pt.nr == A.nr; rows sorted, at most 4096 entries); entries
// of the product off the pattern are not formed.  Same accumulation as spgemm.
void spgemm_on_pattern(const CsrView &A, const CsrView &B, const Csr &Pt, double sign, double *out_v,
                       hipStream_t s);

}  // namespace airg

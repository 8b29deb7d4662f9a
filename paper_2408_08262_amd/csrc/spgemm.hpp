// Two-phase sparse matrix product with LDS hash rows.
#pragma once
#include "common.hpp"

namespace airg {

// C = A B; columns ascending per row; each entry accumulated in ascending
// order of the contributing A entry, without fused multiply-add.
Csr spgemm(const CsrView &A, const CsrView &B, hipStream_t s);

}  // namespace airg

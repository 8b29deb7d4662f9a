// Grid-transfer operators and the Galerkin coarse operator (setup steps 9-11).
#pragma once
#include "common.hpp"

namespace airg {

// Classical one-point prolongator: F row f(i) takes one entry at the C rank
// of j* = argmax_{j != i} |a_ij| (ties to the smallest j), weight 1
// (weight_mode 0) or -a_ij*/a_ii (1).  Returned as P = [W; I] (n x nC) in
// original row order, and W (nF x nC) alone.
void onepoint_prolongator(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                          int weight_mode, Csr *P, Csr *W, hipStream_t s);

// Numeric re-setup: [W; I] (n x nC, natural rows) from an existing W, and
// weight-mode-1 values recomputed at W's columns.
Csr prolongator_from_w(const Csr &W, const int8_t *cf, const int32_t *rank, int32_t n, int32_t nC, hipStream_t s);
void onepoint_values(const CsrView &A, const int32_t *fidx, const int32_t *cidx, Csr &W, hipStream_t s);

// R = [Z I] (nC x n) in original column order: row r holds Z's row with F
// ranks mapped back through fidx, plus 1 at cidx[r].
Csr restriction_full(const CsrView &Z, const int32_t *fidx, const int32_t *cidx, int32_t n, hipStream_t s);

}  // namespace airg

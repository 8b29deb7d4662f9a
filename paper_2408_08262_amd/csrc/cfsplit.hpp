// Two-pass CF splitting of the CF splitting section: PMISR (a Luby maximal
// independent set on the symmetrised strong connections, F points taking the
// smallest measure) followed by the DDC diagonal-dominance cleanup.
#pragma once
#include "common.hpp"

namespace airg {

struct StrengthGraph {
    int32_t n = 0;
    DBuf<uint8_t> strong;       // per nonzero of A: 1 if j in S_i
    DBuf<int32_t> srp, sci;     // S as its own CSR (columns ascending), room for nnz(A) columns
    DBuf<int32_t> cntT, mutual; // |S_i^T| and |S_i n S_i^T|
};

// Strength of connection, strength equation with absolute values:
// j in S_i iff j != i, a_ij != 0 and |a_ij| >= alpha * max_{k != i} |a_ik|.
StrengthGraph strength_graph(const CsrView &A, double alpha, hipStream_t s);
// deg[i] = |S_i u S_i^T| (n entries).
void strength_degree(const StrengthGraph &G, int32_t *deg, hipStream_t s);

// PMISR measure keys h_i (upper 32 bits of the counter generator, stream 0)
// and rounds on the graph; writes cf (1 = F, 2 = C).  max_rounds = 0 runs
// until no node is unassigned.  Returns the rounds run.
// Keys of a block-diagonal batch: segment p (rows off[p] .. off[p+1]-1, device
// offsets) uses seeds[p] and indices local to the segment.
void pmisr_hash_seg(int32_t n, const int32_t *off, int nseg, const uint64_t *seeds, int32_t level, uint32_t *h,
                    hipStream_t s);
// With h null the measures are drawn inside the first pass from (seed,
// level).
int pmisr(const CsrView &A, const StrengthGraph &G, const uint32_t *h, int max_rounds, int8_t *cf, hipStream_t s,
          uint64_t seed = 0, int32_t level = 0);

// DDC: F rows with theta_i > alpha_diag (theta != 0), or a zero diagonal,
// become C, all from the F set given in cf_in.  theta (nullable) receives
// theta_i for F rows and -1 elsewhere.
// flags3 (nullable, 3 n ints) receives the class indicators of cf_out:
// cf == F, cf == C, cf == T.
void ddc(const CsrView &A, double alpha_diag, const int8_t *cf_in, int8_t *cf_out, double *theta, hipStream_t s,
         int32_t *flags3 = nullptr);
// alpha_diag from the fraction rule (1000 uniform bins on [0, theta_max]).
double ddc_fraction_threshold(const CsrView &A, const int8_t *cf, double fraction, hipStream_t s);
// The same threshold with theta and the counters in a fixed device array of
// the library (no device allocation); at most ddc_fraction_noalloc_max_rows()
// rows, and calls that overlap on one device race.
double ddc_fraction_threshold_noalloc(const CsrView &A, const int8_t *cf, double fraction, hipStream_t s);
int64_t ddc_fraction_noalloc_max_rows();

struct CfParams {
    double strong_threshold, ddc_threshold, ddc_fraction;
    int max_rounds;
    uint64_t seed;
};
// Full splitting; returns (nF, nC).
std::pair<int32_t, int32_t> cf_split(const CsrView &A, const CfParams &p, int32_t level, int8_t *cf, hipStream_t s);

}  // namespace airg

// Batched form: many independent AIRG hierarchies (one per segment) solved
// together.  Level l of the batch concatenates the level-l operators of every
// segment still present: segments that coarsen further ("active") are laid
// out F points first then C points, segments whose coarsest level is l
// ("terminal") follow.  Each V-cycle stage is one SpMM launch over all
// segments and right-hand sides; the whole cycle is captured as a HIP graph.
#pragma once
#include <map>
#include <string>

#include "hierarchy.hpp"

namespace airg {

struct BatchLevel {
    int32_t nF = 0, nC = 0, nT = 0;
    int32_t n() const { return nF + nC + nT; }
    Csr AF, Ainv, Rp, Pp;    // active segments, in the batch level layout
    Csr AT, AinvT;           // terminal segments, indices relative to the terminal block
    int lAF = -1, lAinv = -1, lRp = -1, lPp = -1, lAT = -1, lAinvT = -1;   // kernel choice per matrix
    DBuf<float> g, e, t;     // n() x k
};

struct Batch {
    int k = 1;
    int nseg = 0;
    int64_t n = 0;
    int coarse_iters = 3, up_smooths = 2;
    std::vector<std::unique_ptr<BatchLevel>> lv;
    DBuf<int32_t> perm0;               // natural row -> level-0 batch position
    DBuf<float> g0, e0;                // level-0 input/output of the cycle
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;         // private stream the graph is captured on
    std::map<std::string, int> tuned;  // autotuner record: "rows:nnz:k" -> kernel choice
    int64_t cycles_eager = 0, cycles_graph = 0;   // cycles run kernel by kernel / as graph replays
    hipEvent_t *prof = nullptr;                   // per-level profile events (4 per level) when set
    ~Batch();
    void vcycle(int l, const float *g, float *e, hipStream_t s);
    void run(hipStream_t s, bool use_graph);   // e0 = V(g0)
};

// Builds the batch operators from per-segment hierarchies for k right-hand
// sides; tune runs the autotuner on every batch operator.
std::unique_ptr<Batch> build_batch(std::vector<std::unique_ptr<Hier>> &segs, int k, bool tune, hipStream_t s);
// Work vectors (zeroed) and, when tune is set, the autotuner over every batch
// operator; lv, k, n and perm0 must be in place.
void finish_batch(Batch &B, bool tune, hipStream_t s);

struct BatchResult {
    int iterations = 0;
    bool converged = false;
    double worst = 0.0;
};
// FGMRES(restart) in FP64 over every (segment, rhs) pair at once, right
// preconditioned by the batched FP32 V-cycle; natural row order, b and x are
// n x k row-major.  A is the block-diagonal finest operator.
BatchResult solve_batch(Batch &B, const Csr &A, const std::vector<int64_t> &seg, const double *b, double *x,
                        double rtol, int maxit, int restart, bool use_graph, hipStream_t s);

// One batched FP32 V-cycle on FP64 vectors in natural row order (n x k
// row-major): e = V(g), the cast into and out of the cycle included.
void batch_apply(Batch &B, const double *g, double *e, bool use_graph, hipStream_t s);

// Mean device seconds per eager batched cycle of each level's own work (the
// restriction, then the prolongation, smoothing and terminal coarse solves),
// over reps cycles on a zero input: out[l] for l < B.lv.size().
void batch_profile(Batch &B, int reps, double *out, hipStream_t s);

}  // namespace airg

// AIRG hierarchy: setup driver (level loop of the AIRG subsection) and the
// permuted solve-phase operators, V-cycle and outer iterations.
#pragma once
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <memory>
#include <tuple>
#include <vector>

#include "airg.h"
#include "common.hpp"
#include "csr.hpp"
#include "poly.hpp"
#include "trace.hpp"

namespace airg {

struct Level {
    int32_t n = 0, nF = 0, nC = 0;
    bool coarsest = false;
    // setup objects, natural order (F/C ranks by ascending index)
    Csr A;                        // operator of this level
    DBuf<int8_t> cf;
    DBuf<int32_t> rank, fidx, cidx;
    Csr Aff, Afc, Ainv, Z, W;
    PolyInfo poly;
    // solve objects, level order = F points first (by rank), then C points
    DBuf<int32_t> perm;           // natural index -> position in level order
    DBuf<int32_t> iperm;          // position -> natural index
    Csr AF;                       // [A_ff A_fc]: F rows, all columns in level order
    Csr Rp;                       // [Z I]: rows in the next level's order
    Csr Pp;                       // [W; I]: rows in level order, columns in the next level's order
    // V-cycle work vectors
    DBuf<double> g64, e64, t64;
    DBuf<float> g32, e32, t32;
    DBuf<double> p64, q64, u64;   // coarsest level, matrix-free polynomial
    DBuf<float> p32, q32, u32;
    // [W; I] as one (column, value) per row (pcol < 0: empty row), kept on
    // the small levels, where the prolongation is fused with the first
    // smoothing residual
    DBuf<int32_t> pcol;
    DBuf<double> pval64;
    DBuf<float> pval32;
    // setup device time of this level by phase, and the bytes its setup steps
    // must move (each step reading its inputs and writing its outputs once)
    double phase[AIRG_PHASE_COUNT] = {};
    int64_t setup_bytes = 0;
    // kept from setup for numeric re-setup: the extraction plan, A_cf, the
    // prolongator [W; I] (natural order) and the pattern of A P; the row bins
    // of the re-setup's assembly and products, made by the first re-setup
    ExtractPlan xplan;
    Csr Acf, P, APp;
    bool rbins = false;
    Bins rb_ainv, rb_z, rb_ap, rb_rap;
};

struct Hier {
    airg_opts opt{};
    uint64_t seed = 0;
    hipStream_t s = nullptr;
    std::vector<std::unique_ptr<Level>> lv;
    double setup_seconds = 0.0;
    double resetup_seconds = 0.0;
    double phase[AIRG_PHASE_COUNT] = {};
    DBuf<double> x, r, e, bp;     // top-level work vectors
    DBuf<float> r32, e32;
    // V-cycle graphs (use_graph): [0] FP64, [1] FP32, captured once on the
    // private stream cap over fixed buffers and replayed on s.  A slot is
    // captured only after kEagerCycles eager cycles at its precision since the
    // last (re)setup: capture and instantiation cost about as much as that
    // many replays save, so a hierarchy used for one short solve never pays it.
    static constexpr int kEagerCycles = 16;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int eager[2] = {0, 0};
    hipStream_t cap = nullptr;
    // V-cycles applied since setup: launched one kernel at a time, or as one
    // replay of a captured graph
    int64_t cycles_eager = 0, cycles_graph = 0;
    // when set, vcycle records 4 events per level: around the restriction
    // and around the work after the coarse correction (per-level profile)
    hipEvent_t *prof = nullptr;

    Hier() = default;
    Hier(const Hier &) = delete;
    Hier &operator=(const Hier &) = delete;
    ~Hier();
    int nlev() const { return (int)lv.size(); }
    Level &L(int l) { return *lv[l]; }

    template <class T>
    void vcycle(int l, const T *g, T *e);
    void precondition(const double *r, double *e, int precision);
    void drop_graphs();
};

// Per-phase device time from events recorded around each phase on the setup
// stream, tagged with the level being built (level is set by the driver
// before each level; -1 = after the level loop); span_on times work enqueued
// by another thread on another stream (its phase then overlaps the others).
inline const char *phase_name(int phase) {
    static const char *const names[AIRG_PHASE_COUNT] = {"cf", "extract", "poly", "restrictor",
                                                        "prolongator", "coarse", "finalize"};
    return phase >= 0 && phase < AIRG_PHASE_COUNT ? names[phase] : "phase";
}

struct PhaseTimer {
    hipStream_t s;
    bool on;   // off: phases still open and close roctx ranges, but record no events
    std::mutex mu;
    struct Span {
        int level, phase;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    int cur = -1;
    int level = -1;
    hipEvent_t start = nullptr;
    PhaseTimer(hipStream_t st, bool enabled) : s(st), on(enabled) {}
    ~PhaseTimer() {
        for (auto &t : spans) {
            release_event(t.a);
            release_event(t.b);
        }
        release_event(start);
    }
    void begin(int phase) {
        end();
        if (on) {
            start = pooled_event();
            AIRG_HIP(hipEventRecord(start, s));
        }
        cur = phase;
        trace_push(phase_name(phase));
    }
    void end() {
        if (cur < 0) return;
        trace_pop();
        if (!on) {
            cur = -1;
            return;
        }
        hipEvent_t stop = pooled_event();
        AIRG_HIP(hipEventRecord(stop, s));
        std::lock_guard<std::mutex> lk(mu);
        spans.push_back({level, cur, start, stop});
        start = nullptr;
        cur = -1;
    }
    template <class F>
    void span_on(int phase, int lvl, hipStream_t st, F &&f) {
        TraceRange tr(phase_name(phase));
        if (!on) {
            f();
            return;
        }
        hipEvent_t a = pooled_event(), b = pooled_event();
        {
            std::lock_guard<std::mutex> lk(mu);
            spans.push_back({lvl, phase, a, b});
        }
        AIRG_HIP(hipEventRecord(a, st));
        f();
        AIRG_HIP(hipEventRecord(b, st));
    }
    // Phase totals into out[phase]; per_level(level, phase, seconds) for every
    // span recorded inside the level loop.
    template <class PerLevel>
    void collect(double *out, PerLevel &&per_level) {
        end();
        AIRG_HIP(hipStreamSynchronize(s));
        for (auto &t : spans) {
            AIRG_HIP(hipEventSynchronize(t.b));
            float ms = 0.f;
            AIRG_HIP(hipEventElapsedTime(&ms, t.a, t.b));
            out[t.phase] += ms * 1e-3;
            if (t.level >= 0) per_level(t.level, t.phase, ms * 1e-3);
        }
    }
    void collect(double *out) {
        collect(out, [](int, int, double) {});
    }
};

struct NullTimer {
    int level = -1;
    void begin(int) {}
    void end() {}
    template <class F>
    void span_on(int, int, hipStream_t, F &&f) {
        f();
    }
};

// A second host thread with its own stream.  start() runs a job there after
// everything enqueued so far on the main stream; finish() waits for the job
// and makes later work on the main stream wait for the job's work.  The two
// threads enqueue and synchronise independently, so latency-bound work of one
// overlaps that of the other.
class Branch {
public:
    explicit Branch(hipStream_t main);
    ~Branch();
    Branch(const Branch &) = delete;
    Branch &operator=(const Branch &) = delete;
    hipStream_t stream() const { return s_; }
    // Starts a job on the worker thread and stream (after the previous job
    // has ended; its exception, if any, is rethrown here).
    void start(std::function<void()> job);
    void finish();        // rethrows the job's exception
    void wait_idle();     // waits for a running job, ignoring its outcome
    // Called by the job: the work it has queued so far is what the main
    // stream needs first.  wait_mark() makes the main stream wait for that
    // work only (rethrowing an exception raised before the mark); the rest
    // of the job is joined by the next start() or finish().
    void mark();
    void wait_mark();
    // Orders the branch stream's later work after the main stream's work so
    // far (called by the main thread before it returns blocks that were made
    // on the branch stream, and that its own stream has used, to the
    // allocator's cache for the branch stream, while a job may be running).
    void follow_main();
    struct Worker;        // the host thread; kept per device for later setups
private:
    hipStream_t main_, s_ = nullptr;
    hipEvent_t fork_ = nullptr, join_ = nullptr, mid_ = nullptr;
    int dev_ = 0;
    Worker *w_ = nullptr;
};

// Pieces of the setup shared by the single and batch drivers.
Csr pattern_copy(const CsrView &A, hipStream_t s);
// The fixed-sparsity polynomial on the pattern of A^order (order 1: A's).
Csr inverse_pattern(const CsrView &A, int order, hipStream_t s);
Csr assemble_inverse(const CsrView &A, const PolyInfo &P, int m, int order, hipStream_t s);
// perm: natural index -> level order (F by rank, then C, then terminal rows);
// iperm its inverse.
void make_level_perm(int32_t n, int32_t nF, int32_t nC, const int8_t *cf, const int32_t *rank, int32_t *perm,
                     int32_t *iperm, hipStream_t s);
// Rows src[0..nout) of A with F columns renumbered by rank and C columns as
// nF + rank.  The _begin/_fill halves leave the size readback to the caller
// (resolve_sizes), so that many matrices share one synchronisation.
Csr permute_fc(const CsrView &A, const int32_t *src, int32_t nout, const int8_t *cf, const int32_t *rank, int32_t nF,
               hipStream_t s);
Csr permute_fc_begin(const CsrView &A, const int32_t *src, int32_t nout, hipStream_t s);
void permute_fc_fill(Csr &B, const CsrView &A, const int32_t *src, const int8_t *cf, const int32_t *rank, int32_t nF,
                     hipStream_t s);
// [Z I] (nC x ncols) with rows in the next level's order (niperm, nullable).
Csr build_rp_begin(const Csr &Z, int32_t nC, int32_t ncols, const int32_t *niperm, hipStream_t s);
void build_rp_fill(Csr &R, const Csr &Z, int32_t nF, const int32_t *niperm, hipStream_t s);
// [W; I] ((nF + nC) x ncols) in level order, columns through nperm (nullable).
Csr build_pp_begin(const Csr &W, int32_t nF, int32_t nC, int32_t ncols, hipStream_t s);
void build_pp_fill(Csr &P, const Csr &W, int32_t nF, const int32_t *nperm, hipStream_t s);

// Builds the full hierarchy of the canonical operator A0 (takes ownership).
std::unique_ptr<Hier> build_hierarchy(Csr &&A0, const airg_opts &o, uint64_t seed, hipStream_t s);

// Numeric re-setup with new top-level values (canonical pattern of level 0,
// device): same splittings and patterns, recomputed values.
void resetup_hierarchy(Hier &H, const double *vals, hipStream_t s);

// Single-level build for replay/inspection: CF split, A_ff, polynomial
// (alpha_in nullable), Ainv, Z, W and the coarse operator.
struct LevelOut {
    DBuf<int8_t> cf;
    int32_t nF = 0, nC = 0;
    PolyInfo poly;
    Csr Ainv, Z, W, Ac;
};
LevelOut build_one_level(const CsrView &A, const airg_opts &o, uint64_t seed, int level, const double *alpha_in,
                         hipStream_t s);

// Outer iterations on one right-hand side (contiguous vectors, natural order).
struct SolveResult {
    int iterations = 0;
    double rel_residual = 0.0;
    bool converged = false;
};
SolveResult solve_richardson(Hier &H, const double *b, double *x, double rtol, int maxit);
// One V-cycle e = V(g) in natural order (precision 64 or 32).
void apply_vcycle(Hier &H, const double *g, double *e, int precision);
// Device time of each level's own work in one eager V-cycle (the restriction
// to the next level plus everything after the coarse correction; the whole
// coarse solve on the coarsest level), averaged over reps cycles on a zero
// input: out[l] for l < H.nlev().
void profile_vcycle(Hier &H, int precision, int reps, double *out);
SolveResult solve_fgmres(Hier &H, const double *b, double *x, double rtol, int maxit);

// One V-cycle's products: stored entries, index bytes (columns, row
// pointers) and vector entries read or written per right-hand side; its
// algorithmic bytes with v-byte values and k right-hand sides follow.
struct CycleCost {
    int64_t nnz = 0, index_bytes = 0, vec_entries = 0;
    void add(int64_t rows, int64_t cols, int64_t nz, bool reads_y, int64_t times);
    int64_t bytes(int vb, int k) const { return index_bytes + vb * nnz + (int64_t)vb * k * vec_entries; }
};
CycleCost vcycle_cost(const Hier &H);
// Algorithmic bytes of one V-cycle with vbytes-byte values.
int64_t vcycle_bytes(const Hier &H, int vbytes);
// Stored entries of every matrix one V-cycle applies (its work in units of
// multiply-adds; divided by nnz(A_0), the cycle's work units).
int64_t vcycle_nnz(const Hier &H);
void complexities(const Hier &H, double *grid, double *op, double *storage);
int64_t spmv_bytes(int64_t rows, int64_t cols, int64_t nnz, int vbytes, bool reads_y);
// Algorithmic bytes of the setup steps (each reads its inputs and writes its
// outputs once): an FP64 CSR matrix, the polynomial's coefficients on an
// F-block (m products, one TSQR pass) and the CF splitting of a level.
int64_t csr_bytes(const CsrView &M);
int64_t poly_bytes(const CsrView &Aff, int m);
int64_t split_bytes(const CsrView &A);

}  // namespace airg

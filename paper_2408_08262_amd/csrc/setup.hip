// AIRG setup driver: the per-level recipe of the AIRG subsection on the
// device, termination/truncation, and the permuted solve-phase operators.
#include <chrono>
#include <cmath>

#include "cfsplit.hpp"
#include "csr.hpp"
#include "group.hpp"
#include "hierarchy.hpp"
#include "poly.hpp"
#include "spgemm.hpp"
#include "transfer.hpp"

namespace airg {

// ----------------------------------------------------------------- branch --
// One branch stream per device for the life of the process, so that device
// blocks released on it return to the allocator's cache under a stream that
// later setups use again.  Work of concurrent setups on it stays ordered by
// their own fork and join events.
static hipStream_t branch_stream(int dev) {
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)streams.size() <= dev) streams.resize((size_t)dev + 1, nullptr);
    if (!streams[dev]) AIRG_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    return streams[dev];
}

// The branch's host thread.  Threads are kept per device after their setup
// and taken again by later ones (starting a thread and attaching it to the
// device cost tens of microseconds of host time per setup); they wait on
// their condition variable for the life of the process.
struct Branch::Worker {
    int dev = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::function<void()> job;
    std::exception_ptr err;
    bool has = false, busy = false, marked = false;

    void loop() {
        (void)hipSetDevice(dev);
        for (;;) {
            std::function<void()> j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return has; });
                j = std::move(job);
                has = false;
            }
            std::exception_ptr e;
            try {
                j();
            } catch (...) {
                e = std::current_exception();
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                err = e;
                busy = false;
            }
            cv.notify_all();
        }
    }
};

namespace {
std::mutex g_worker_mu;
std::vector<std::vector<Branch::Worker *>> g_idle_workers;   // per device

Branch::Worker *take_worker(int dev) {
    {
        std::lock_guard<std::mutex> lk(g_worker_mu);
        if ((int)g_idle_workers.size() <= dev) g_idle_workers.resize((size_t)dev + 1);
        auto &v = g_idle_workers[dev];
        if (!v.empty()) {
            Branch::Worker *w = v.back();
            v.pop_back();
            return w;
        }
    }
    auto *w = new Branch::Worker();
    w->dev = dev;
    std::thread([w] { w->loop(); }).detach();
    return w;
}

void give_worker(Branch::Worker *w) {
    std::lock_guard<std::mutex> lk(g_worker_mu);
    g_idle_workers[w->dev].push_back(w);
}
}  // namespace

Branch::Branch(hipStream_t main) : main_(main) {
    AIRG_HIP(hipGetDevice(&dev_));
    hipDevice_t sdev = 0;
    AIRG_HIP(hipStreamGetDevice(main, &sdev));
    AIRG_REQUIRE((int)sdev == dev_, ST_INVALID_ARG, "the stream belongs to another device than the current one");
    s_ = branch_stream(dev_);
    fork_ = pooled_event();
    join_ = pooled_event();
    mid_ = pooled_event();
    w_ = take_worker(dev_);
    std::lock_guard<std::mutex> lk(w_->mu);   // an idle worker: drop a failure left by its last owner
    w_->err = nullptr;
}

Branch::~Branch() {
    wait_idle();
    (void)hipStreamSynchronize(s_);
    release_event(fork_);
    release_event(join_);
    release_event(mid_);
    give_worker(w_);
}

void Branch::start(std::function<void()> job) {
    wait_idle();
    if (w_->err) std::rethrow_exception(w_->err);
    AIRG_HIP(hipEventRecord(fork_, main_));
    AIRG_HIP(hipStreamWaitEvent(s_, fork_, 0));
    {
        std::lock_guard<std::mutex> lk(w_->mu);
        w_->job = std::move(job);
        w_->err = nullptr;
        w_->has = true;
        w_->busy = true;
        w_->marked = false;
    }
    w_->cv.notify_all();
}

void Branch::mark() {
    AIRG_HIP(hipEventRecord(mid_, s_));
    {
        std::lock_guard<std::mutex> lk(w_->mu);
        w_->marked = true;
    }
    w_->cv.notify_all();
}

void Branch::follow_main() {
    AIRG_HIP(hipEventRecord(fork_, main_));
    AIRG_HIP(hipStreamWaitEvent(s_, fork_, 0));
}

void Branch::wait_mark() {
    bool marked;
    {
        std::unique_lock<std::mutex> lk(w_->mu);
        w_->cv.wait(lk, [&] { return w_->marked || !w_->busy; });
        marked = w_->marked;
    }
    if (!marked) {   // the job ended before its mark
        if (w_->err) std::rethrow_exception(w_->err);
        AIRG_HIP(hipEventRecord(join_, s_));
        AIRG_HIP(hipStreamWaitEvent(main_, join_, 0));
        return;
    }
    AIRG_HIP(hipStreamWaitEvent(main_, mid_, 0));
}

void Branch::wait_idle() {
    std::unique_lock<std::mutex> lk(w_->mu);
    w_->cv.wait(lk, [&] { return !w_->busy; });
}

void Branch::finish() {
    wait_idle();
    if (w_->err) std::rethrow_exception(w_->err);
    AIRG_HIP(hipEventRecord(join_, s_));
    AIRG_HIP(hipStreamWaitEvent(main_, join_, 0));
}

namespace {

// Waits for a started branch job when the main thread leaves the scope
// early (an exception), before the objects the job writes are destroyed.
struct BranchGuard {
    Branch *b = nullptr;
    ~BranchGuard() {
        if (b) b->wait_idle();
    }
};

CfParams cf_params(const airg_opts &o, uint64_t seed) {
    return CfParams{o.strong_threshold, o.ddc_threshold, o.ddc_fraction, o.pmisr_max_rounds, seed};
}

// CF splitting of one level; fills cf and rank, returns (nF, nC).  When
// nnz_out is given, A.nnz is only an upper bound (A's rows were kept by a
// drop whose total was not read) and the exact count A.rp[nr] is read back
// with the splitting's counts into *nnz_out.  With xp, the extraction's
// counting half runs too and the three block sizes come back with the
// counts into xtot[0..2].
std::pair<int32_t, int32_t> split(const CsrView &A, const airg_opts &o, uint64_t seed, int lvl, DBuf<int8_t> &cf,
                                  DBuf<int32_t> &rank, hipStream_t s, int64_t *nnz_out = nullptr,
                                  ExtractPlan *xp = nullptr, int32_t *xtot = nullptr) {
    int32_t n = A.nr;
    cf.alloc((size_t)n, s);
    rank.alloc((size_t)n, s);
    StrengthGraph G = strength_graph(A, o.strong_threshold, s);
    DBuf<int8_t> cf0((size_t)n, s);
    pmisr(A, G, nullptr, o.pmisr_max_rounds, cf0.p, s, seed, lvl);
    double ad = o.ddc_threshold;
    if (ad < 0.0) ad = ddc_fraction_threshold(A, cf0.p, o.ddc_fraction, s);
    DBuf<int32_t> flags((size_t)3 * n, s);   // class indicators for the rank scans
    ddc(A, ad, cf0.p, cf.p, nullptr, s, flags.p);
    std::vector<const int32_t *> extra;
    if (nnz_out) extra.push_back(A.rp + n);
    if (xp) {
        *xp = extract_begin(A, cf.p, s);
        for (const int32_t *t : xp->totals()) extra.push_back(t);
    }
    int32_t got[4] = {0, 0, 0, 0};
    CfCounts c = cf_ranks3(cf.p, n, rank.p, s, extra, got, flags.p);
    if (nnz_out) *nnz_out = got[0];
    if (xp) std::copy(got + (nnz_out ? 1 : 0), got + (nnz_out ? 4 : 3), xtot);
    return {c.nF, c.nC};
}

}  // namespace

Csr pattern_copy(const CsrView &A, hipStream_t s) {
    Csr X;
    X.alloc(A.nr, A.nc, A.nnz, s);
    const CopyReq req[2] = {{X.rp.p, A.rp, ((size_t)A.nr + 1) * sizeof(int32_t)},
                            {X.ci.p, A.ci, (size_t)A.nnz * sizeof(int32_t)}};
    copy_many(req, 2, s);
    return X;
}

// The fixed-sparsity polynomial on the pattern of A^order (order 1: A's own
// pattern).
Csr inverse_pattern(const CsrView &A, int order, hipStream_t s) {
    return order <= 1 ? pattern_copy(A, s) : power_pattern(A, order, s);
}

Csr assemble_inverse(const CsrView &A, const PolyInfo &P, int m, int order, hipStream_t s) {
    Csr X = inverse_pattern(A, order, s);
    poly_fixed_sparsity_pattern(A, view(X), P.alpha, m, X.v.p, s);
    return X;
}

// FP64 CSR bytes of a matrix (row pointers, columns, values).
int64_t csr_bytes(const CsrView &M) { return M.nnz * 12 + ((int64_t)M.nr + 1) * 4; }
// The polynomial's coefficients on an n_F-row block: m products with A_ff
// (each reading A_ff and x, writing y) and one TSQR pass over the m + 1
// basis columns.
int64_t poly_bytes(const CsrView &Aff, int m) {
    return (int64_t)m * (csr_bytes(Aff) + 16 * (int64_t)Aff.nr) + (int64_t)Aff.nr * (m + 1) * 8;
}
// The splitting of an n-row level: strength (A in, one flag per entry out),
// PMISR (the strong pattern in, states out), DDC (A and states in, states
// out) and the rank scans.
int64_t split_bytes(const CsrView &A) {
    const int64_t n = A.nr;
    return csr_bytes(A) + A.nnz + (A.nnz * 5 + (n + 1) * 4 + n) + (csr_bytes(A) + 2 * n) + 5 * n;
}

namespace {

// Steps 2 and 7-11 of the recipe once the splitting is known.  The
// prolongator and A P depend on the splitting only: with a Branch they are
// built by its thread on its stream while this thread builds the F-block
// polynomial, Ainv and Z.
template <class Timer>
void complete_level(const CsrView &A, const airg_opts &o, uint64_t seed, int lvl, const double *alpha_in,
                    const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC, DBuf<int32_t> &fidx,
                    DBuf<int32_t> &cidx, Csr &Aff, Csr *Afc, PolyInfo &poly, Csr &Ainv, Csr &Z, Csr &W, Csr &Ac,
                    Timer &tm, hipStream_t s, Branch *br = nullptr,
                    const std::function<void(hipStream_t)> &pre = nullptr, ExtractPlan *xp = nullptr,
                    const int32_t *xtot = nullptr, int64_t *cbytes = nullptr, Csr *acf_keep = nullptr,
                    Csr *p_keep = nullptr, Csr *ap_keep = nullptr) {
    int32_t n = A.nr;
    int m = o.poly_order + 1;
    Csr P, AP;
    int64_t nb = 0;   // the level's setup bytes: every step reads its inputs and writes its outputs once
    auto prolong = [&](hipStream_t st) {
        tm.span_on(AIRG_PHASE_PROLONG, lvl, st, [&] {
            onepoint_prolongator(A, cf, rank, nF, nC, o.onepoint_weight, &P, &W, st);
            AP = spgemm(A, view(P), st);
        });
    };
    BranchGuard guard;
    if (br) {
        // the prolongator and A P first (the coarse phase waits for them),
        // then `pre`, which runs on while this thread goes on; it owns a copy
        // of its callable, since it may outlive this call
        guard.b = br;
        std::function<void(hipStream_t)> after = pre;
        const hipStream_t bs = br->stream();
        Branch *b = br;
        br->start([&prolong, after, bs, b] {
            prolong(bs);
            b->mark();
            if (after) after(bs);
        });
    } else if (pre) {
        pre(s);
    }
    tm.begin(AIRG_PHASE_EXTRACT);
    fidx.alloc((size_t)nF + 1, s);
    cidx.alloc((size_t)nC + 1, s);
    Csr fc, Acf;
    if (xp) {
        extract_finish(A, cf, rank, nF, nC, xtot, *xp, Aff, fc, Acf, s, fidx.p, cidx.p);
    } else {
        cf_index_lists(cf, rank, n, fidx.p, cidx.p, s);
        extract_fc_blocks(A, cf, rank, nF, nC, Aff, fc, Acf, s);
    }
    nb += csr_bytes(A) + 5 * (int64_t)n + csr_bytes(view(Aff)) + csr_bytes(view(fc)) + csr_bytes(view(Acf));
    if (Afc) *Afc = std::move(fc);
    tm.begin(AIRG_PHASE_POLY);
    // With the first-order pattern, the row bins of the fixed-sparsity
    // assembly and of Z's product depend only on A_ff's and A_cf's patterns:
    // they are started first and their totals come back with the R factor.
    const bool planned = !alpha_in && o.poly_sparsity_order <= 1;
    FixedPlan fplan;
    SpgemmPlan zplan;
    std::vector<int32_t> htot;
    int32_t zoff = 0;
    if (alpha_in) {
        poly = PolyInfo{};
        poly.m = m;
        poly.used = m;
        for (int k = 0; k < m; ++k) poly.alpha[k] = alpha_in[k];
    } else if (planned) {
        fplan = fixed_sparsity_begin(view(Aff), s);
        zplan = spgemm_begin(view(Acf), Aff.rp.p, Aff.nc, s);   // Ainv has A_ff's pattern
        ExtraReads ex;
        ex.src = {fplan.bins.tot.p};
        ex.cnt = {kFixedBins + 1};
        zoff = kFixedBins + 1;
        auto zt = zplan.totals();
        if (zt.second > 0) {
            ex.src.push_back(zt.first);
            ex.cnt.push_back(zt.second);
        }
        htot.resize((size_t)zoff + std::max(zt.second, 1));
        ex.h = htot.data();
        poly = gmres_poly(view(Aff), seed, lvl, m, s, &ex);
    } else {
        poly = gmres_poly(view(Aff), seed, lvl, m, s);
    }
    if (planned) {
        Ainv = pattern_copy(view(Aff), s);
        poly_fixed_sparsity_planned(view(Aff), view(Ainv), poly.alpha, m, Ainv.v.p, fplan, htot.data(), s);
    } else {
        Ainv = assemble_inverse(view(Aff), poly, m, o.poly_sparsity_order, s);
    }
    tm.begin(AIRG_PHASE_RESTRICTOR);
    {
        // Z = -A_cf Ainv, dropped (in the planned form as its rows are written); its entry count is
        // read with R A P's plan
        DropArgs dz;
        dz.tau = o.drop_R;
        dz.sign = -1.0;
        dz.keep_diag = 0;
        Csr prod = planned ? spgemm_finish(view(Acf), view(Ainv), zplan, htot.data() + zoff, s, &dz)
                           : spgemm(view(Acf), view(Ainv), s);
        Z = planned ? drop_compact(prod, zplan.kcnt.p, true, s) : drop_rows_bound(view(prod), o.drop_R, false, true, s);
        // power basis (m products with A_ff), TSQR of the basis, assembly of
        // Ainv; Z's product and its drop (Z's size is bounded by the product's
        // until read below)
        nb += poly_bytes(view(Aff), m) + csr_bytes(view(Aff)) + csr_bytes(view(Ainv));
        nb += csr_bytes(view(Acf)) + csr_bytes(view(Ainv)) + 2 * csr_bytes(view(prod));
    }
    if (acf_keep) *acf_keep = std::move(Acf);
    if (br) {
        tm.end();
        guard.b = nullptr;
        br->wait_mark();
    } else {
        tm.end();
        prolong(s);
    }
    tm.begin(AIRG_PHASE_COARSE);
    {
        Csr R = restriction_full(view(Z), fidx.p, cidx.p, n, s);   // entry count bounded by Z's
        SpgemmPlan plan = spgemm_begin(view(R), AP.rp.p, AP.nc, s);
        auto [tsrc, tcnt] = plan.totals();
        std::vector<int32_t> h((size_t)tcnt + 1);
        if (tcnt > 0) read_ints({Z.rp.p + Z.nr, tsrc}, {1, tcnt}, h.data(), s);
        else read_ints({Z.rp.p + Z.nr}, {1}, h.data(), s);
        Z.nnz = h[0];
        R.nnz = Z.nnz + Z.nr;
        DropArgs da;   // the drop of the coarse operator, as R A P's rows are written
        da.tau = o.drop_A;
        da.sign = 1.0;
        da.keep_diag = 1;
        Csr RAP = spgemm_finish(view(R), view(AP), plan, h.data() + 1, s, &da);
        // with a Branch the entry count is read by the next level's splitting
        Ac = drop_compact(RAP, plan.kcnt.p, br != nullptr, s);
        // W and P from A; A P; R from Z; R (A P); the drop of R A P (A_c's
        // dropped count is counted as the product's, an upper bound)
        nb += csr_bytes(A) + 5 * (int64_t)n + csr_bytes(view(W)) + csr_bytes(view(P));
        nb += csr_bytes(A) + csr_bytes(view(P)) + csr_bytes(view(AP));
        nb += csr_bytes(view(Z)) + csr_bytes(view(R));
        nb += csr_bytes(view(R)) + csr_bytes(view(AP)) + 3 * csr_bytes(view(RAP));
    }
    tm.end();
    if (cbytes) *cbytes += nb;
    // A P's values were made on the branch stream and read by the Galerkin
    // product on this one; the branch job may still be running (and
    // allocating): its stream first waits for this one, then they go back
    if (br) br->follow_main();
    if (p_keep) *p_keep = std::move(P);
    if (ap_keep) {
        AP.v.reset();
        AP.vf.reset();
        *ap_keep = std::move(AP);
    }
}

}  // namespace

// ----------------------------------------------------------- permutation ---
// Level order: F points by rank, then C points, then terminal rows (batch).
__global__ void k_make_perm(int32_t n, int32_t nF, int32_t nC, const int8_t *__restrict__ cf,
                            const int32_t *__restrict__ rank, int32_t *__restrict__ perm, int32_t *__restrict__ iperm) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int8_t c = cf[i];
    int32_t p = c == CF_F ? rank[i] : c == CF_C ? nF + rank[i] : nF + nC + rank[i];
    perm[i] = p;
    iperm[p] = i;
}

void make_level_perm(int32_t n, int32_t nF, int32_t nC, const int8_t *cf, const int32_t *rank, int32_t *perm,
                     int32_t *iperm, hipStream_t s) {
    if (n <= 0) return;
    k_make_perm<<<grid_for(n, 256), 256, 0, s>>>(n, nF, nC, cf, rank, perm, iperm);
    AIRG_LAUNCH_CHECK();
}

__global__ void k_perm_count(int32_t nout, const int32_t *__restrict__ src, const int32_t *__restrict__ rp,
                             int32_t *__restrict__ cnt) {
    int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nout) return;
    int32_t i = src[p];
    cnt[p] = rp[i + 1] - rp[i];
}

// Output row p is input row src[p]; F columns first (as their ranks), then C
// columns (as nF + rank): both subsequences keep their ascending order.
template <int G>
__global__ void __launch_bounds__(256) k_perm_fill(int32_t nout, const int32_t *__restrict__ src,
                                                   const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, const int8_t *__restrict__ cf,
                                                   const int32_t *__restrict__ rank, int32_t nF,
                                                   const int32_t *__restrict__ orp, int32_t *__restrict__ oci,
                                                   double *__restrict__ ov) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t p = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (p >= nout) return;
    int32_t i = src[p];
    int32_t w = orp[p];
    int32_t e = rp[i + 1];
    for (int pass = 0; pass < 2; ++pass) {
        int8_t want = pass == 0 ? CF_F : CF_C;
        for (int32_t base = rp[i]; base < e; base += G) {
            int32_t k = base + lane;
            bool keep = false;
            int32_t j = 0;
            if (k < e) {
                j = ci[k];
                keep = cf[j] == want;
            }
            int tot;
            int pre = group_prefix<G>(keep, &tot);
            if (keep) {
                oci[w + pre] = pass == 0 ? rank[j] : nF + rank[j];
                ov[w + pre] = v[k];
            }
            w += tot;
        }
    }
}

Csr permute_fc_begin(const CsrView &A, const int32_t *src, int32_t nout, hipStream_t s) {
    Csr B;
    B.nr = nout;
    B.nc = A.nc;
    B.rp.alloc((size_t)nout + 1, s);
    DBuf<int32_t> cnt((size_t)nout + 1, s);
    if (nout > 0) {
        k_perm_count<<<grid_for(nout, 256), 256, 0, s>>>(nout, src, A.rp, cnt.p);
        AIRG_LAUNCH_CHECK();
    }
    exclusive_scan(cnt.p, B.rp.p, nout, s, false);
    return B;
}

void permute_fc_fill(Csr &B, const CsrView &A, const int32_t *src, const int8_t *cf, const int32_t *rank, int32_t nF,
                     hipStream_t s) {
    int32_t nout = B.nr;
    if (nout == 0) return;
    int g = lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int G>() {
        k_perm_fill<G><<<grid_for((int64_t)nout * G, 256), 256, 0, s>>>(nout, src, A.rp, A.ci, A.v, cf, rank, nF,
                                                                        B.rp.p, B.ci.p, B.v.p);
    });
    AIRG_LAUNCH_CHECK();
}

Csr permute_fc(const CsrView &A, const int32_t *src, int32_t nout, const int8_t *cf, const int32_t *rank, int32_t nF,
               hipStream_t s) {
    Csr B = permute_fc_begin(A, src, nout, s);
    resolve_sizes({&B}, s);
    permute_fc_fill(B, A, src, cf, rank, nF, s);
    return B;
}

// [Z I] with rows in the next level's order: row q is Z's row r = niperm[q]
// (identity when niperm is null) followed by the entry (nF + r, 1).
__global__ void k_rp_count(int32_t nC, const int32_t *__restrict__ niperm, const int32_t *__restrict__ zrp,
                           int32_t *__restrict__ cnt) {
    int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nC) return;
    int32_t r = niperm ? niperm[q] : q;
    cnt[q] = zrp[r + 1] - zrp[r] + 1;
}
template <int G>
__global__ void __launch_bounds__(256) k_rp_fill(int32_t nC, int32_t nF, const int32_t *__restrict__ niperm,
                                                 const int32_t *__restrict__ zrp, const int32_t *__restrict__ zci,
                                                 const double *__restrict__ zv, const int32_t *__restrict__ orp,
                                                 int32_t *__restrict__ oci, double *__restrict__ ov) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t q = (int32_t)(t / G);
    const int lane = group_lane<G>();
    if (q >= nC) return;
    const int32_t r = niperm ? niperm[q] : q;
    const int32_t b = zrp[r], e = zrp[r + 1], w = orp[q];
    for (int32_t k = b + lane; k < e; k += G) {
        oci[w + (k - b)] = zci[k];
        ov[w + (k - b)] = zv[k];
    }
    if (lane == 0) {
        oci[w + (e - b)] = nF + r;
        ov[w + (e - b)] = 1.0;
    }
}

// [W; I] in level order: row p < nF is W's row p, row nF + r is e_r; coarse
// columns mapped through the next level's permutation nperm.
__global__ void k_pp_count(int32_t n, int32_t nF, const int32_t *__restrict__ wrp, int32_t *__restrict__ cnt) {
    int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    cnt[p] = p < nF ? wrp[p + 1] - wrp[p] : 1;
}
__global__ void k_pp_fill(int32_t n, int32_t nF, const int32_t *__restrict__ nperm, const int32_t *__restrict__ wrp,
                          const int32_t *__restrict__ wci, const double *__restrict__ wv,
                          const int32_t *__restrict__ orp, int32_t *__restrict__ oci, double *__restrict__ ov) {
    int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t w = orp[p];
    if (p < nF) {
        for (int32_t k = wrp[p]; k < wrp[p + 1]; ++k, ++w) {
            int32_t c = wci[k];
            oci[w] = nperm ? nperm[c] : c;
            ov[w] = wv[k];
        }
    } else {
        int32_t r = p - nF;
        oci[w] = nperm ? nperm[r] : r;
        ov[w] = 1.0;
    }
}

Csr build_rp_begin(const Csr &Z, int32_t nC, int32_t ncols, const int32_t *niperm, hipStream_t s) {
    Csr R;
    R.nr = nC;
    R.nc = ncols;
    R.rp.alloc((size_t)nC + 1, s);
    DBuf<int32_t> cnt((size_t)nC + 1, s);
    if (nC > 0) {
        k_rp_count<<<grid_for(nC, 256), 256, 0, s>>>(nC, niperm, Z.rp.p, cnt.p);
        AIRG_LAUNCH_CHECK();
    }
    exclusive_scan(cnt.p, R.rp.p, nC, s, false);
    return R;
}

void build_rp_fill(Csr &R, const Csr &Z, int32_t nF, const int32_t *niperm, hipStream_t s) {
    int32_t nC = R.nr;
    if (nC == 0) return;
    dispatch_group(lanes_for(Z.nnz, nC), [&]<int G>() {
        k_rp_fill<G><<<grid_for((int64_t)nC * G, 256), 256, 0, s>>>(nC, nF, niperm, Z.rp.p, Z.ci.p, Z.v.p, R.rp.p,
                                                                     R.ci.p, R.v.p);
    });
    AIRG_LAUNCH_CHECK();
}

Csr build_pp_begin(const Csr &W, int32_t nF, int32_t nC, int32_t ncols, hipStream_t s) {
    Csr P;
    int32_t rows = nF + nC;
    P.nr = rows;
    P.nc = ncols;
    P.rp.alloc((size_t)rows + 1, s);
    DBuf<int32_t> cnt((size_t)rows + 1, s);
    if (rows > 0) {
        k_pp_count<<<grid_for(rows, 256), 256, 0, s>>>(rows, nF, W.rp.p, cnt.p);
        AIRG_LAUNCH_CHECK();
    }
    exclusive_scan(cnt.p, P.rp.p, rows, s, false);
    return P;
}

void build_pp_fill(Csr &P, const Csr &W, int32_t nF, const int32_t *nperm, hipStream_t s) {
    int32_t rows = P.nr;
    if (rows == 0) return;
    k_pp_fill<<<grid_for(rows, 256), 256, 0, s>>>(rows, nF, nperm, W.rp.p, W.ci.p, W.v.p, P.rp.p, P.ci.p, P.v.p);
    AIRG_LAUNCH_CHECK();
}

namespace {

// Level l's permutation to level order (F by rank, then C).
void level_perm(Level &L, hipStream_t s) {
    if (L.coarsest) return;
    L.perm.alloc((size_t)L.n, s);
    L.iperm.alloc((size_t)L.n, s);
    make_level_perm(L.n, L.nF, L.nC, L.cf.p, L.rank.p, L.perm.p, L.iperm.p, s);
}

// Level l's solve operators [A_ff A_fc], [Z I] and [W; I] in level order
// (the next level's permutation must exist): row counts and scans first, the
// sizes of many matrices then come back in one readback, then the fills.
void solve_ops_begin(Hier &H, int l, std::vector<Csr *> &pending, hipStream_t s) {
    Level &L = H.L(l), &N = H.L(l + 1);
    L.AF = permute_fc_begin(view(L.A), L.fidx.p, L.nF, s);
    L.Rp = build_rp_begin(L.Z, L.nC, L.n, N.coarsest ? nullptr : N.iperm.p, s);
    L.Pp = build_pp_begin(L.W, L.nF, L.nC, L.nC, s);
    pending.insert(pending.end(), {&L.AF, &L.Rp, &L.Pp});
}
// One (column, value) per row of [W; I] (at most one entry per row).
__global__ void k_pp_dense(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const float *__restrict__ vf, int32_t *__restrict__ pcol,
                           double *__restrict__ pval, float *__restrict__ pvalf) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const bool has = rp[r + 1] > rp[r];
    pcol[r] = has ? ci[rp[r]] : -1;
    pval[r] = has ? v[rp[r]] : 0.0;
    pvalf[r] = has ? vf[rp[r]] : 0.0f;
}

void solve_ops_fill(Hier &H, int l, hipStream_t s) {
    Level &L = H.L(l), &N = H.L(l + 1);
    permute_fc_fill(L.AF, view(L.A), L.fidx.p, L.cf.p, L.rank.p, L.nF, s);
    build_rp_fill(L.Rp, L.Z, L.nF, N.coarsest ? nullptr : N.iperm.p, s);
    build_pp_fill(L.Pp, L.W, L.nF, N.coarsest ? nullptr : N.perm.p, s);
    make_f32(L.AF, s);
    make_f32(L.Rp, s);
    make_f32(L.Pp, s);
    make_f32(L.Ainv, s);
    // small levels (lane-group SpMVs throughout): prolongation rows for the
    // fused prolongation + residual kernel
    L.pcol.reset();
    L.pval64.reset();
    L.pval32.reset();
    if (!spmv_streams(L.Pp.nr, L.Pp.nnz) && !spmv_streams(L.AF.nr, L.AF.nnz) && L.n > 0) {
        L.pcol.alloc((size_t)L.n, s);
        L.pval64.alloc((size_t)L.n, s);
        L.pval32.alloc((size_t)L.n, s);
        k_pp_dense<<<grid_for(L.n, 256), 256, 0, s>>>(L.n, L.Pp.rp.p, L.Pp.ci.p, L.Pp.v.p, L.Pp.vf.p, L.pcol.p,
                                                      L.pval64.p, L.pval32.p);
        AIRG_LAUNCH_CHECK();
    }
}
void solve_ops(Hier &H, int l, hipStream_t s) {
    std::vector<Csr *> pending;
    solve_ops_begin(H, l, pending, s);
    resolve_sizes(pending, s);
    solve_ops_fill(H, l, s);
}

// Solve-phase objects of levels [built, coarsest) (permutations of every
// level made where missing), the coarsest level's FP32 copies, the top
// operator in level order and the work vectors.
void finalize(Hier &H, int built = 0) {
    hipStream_t s = H.s;
    H.drop_graphs();   // the work vectors are reallocated below
    int nl = H.nlev();
    for (int l = 0; l < nl; ++l)
        if (!H.L(l).perm.p) level_perm(H.L(l), s);
    std::vector<Csr *> pending;
    for (int l = built; l < nl; ++l)
        if (!H.L(l).coarsest) solve_ops_begin(H, l, pending, s);
    resolve_sizes(pending, s);
    for (int l = built; l < nl; ++l) {
        Level &L = H.L(l);
        if (L.coarsest) {
            make_f32(L.A, s);
            if (L.Ainv.rp.p) make_f32(L.Ainv, s);
            continue;
        }
        solve_ops_fill(H, l, s);
    }
    // work vectors
    for (int l = 0; l < nl; ++l) {
        Level &L = H.L(l);
        L.g64.alloc((size_t)L.n, s);
        L.e64.alloc((size_t)L.n, s);
        L.t64.alloc((size_t)L.n, s);
        L.g32.alloc((size_t)L.n, s);
        L.e32.alloc((size_t)L.n, s);
        L.t32.alloc((size_t)L.n, s);
        if (L.coarsest && H.opt.coarse_matrix_free) {
            for (DBuf<double> *b : {&L.p64, &L.q64, &L.u64}) b->alloc((size_t)L.n, s);
            for (DBuf<float> *b : {&L.p32, &L.q32, &L.u32}) b->alloc((size_t)L.n, s);
        }
    }
    int32_t n0 = H.L(0).n;
    H.x.alloc((size_t)n0, s);
    H.r.alloc((size_t)n0, s);
    H.e.alloc((size_t)n0, s);
    H.bp.alloc((size_t)n0, s);
    H.r32.alloc((size_t)n0, s);
    H.e32.alloc((size_t)n0, s);
}

// After a numeric re-setup: the values of every solve operator and FP32
// copy again, into the operators of the same patterns (no size readback).
void refresh_solve_values(Hier &H) {
    hipStream_t s = H.s;
    H.drop_graphs();
    for (int l = 0; l < H.nlev(); ++l) {
        Level &L = H.L(l);
        if (L.coarsest) {
            make_f32(L.A, s);
            if (L.Ainv.rp.p) make_f32(L.Ainv, s);
            continue;
        }
        solve_ops_fill(H, l, s);
    }
}

}  // namespace

// ------------------------------------------------------------------ build --
std::unique_ptr<Hier> build_hierarchy(Csr &&A0, const airg_opts &o, uint64_t seed, hipStream_t s) {
    TraceRange trace("airg setup");
    auto t0 = std::chrono::steady_clock::now();
    auto H = std::make_unique<Hier>();
    H->opt = o;
    H->seed = seed;
    H->s = s;
    PhaseTimer tm(s, o.time_phases != 0);
    auto first = std::make_unique<Level>();
    first->n = A0.nr;
    first->A = std::move(A0);
    H->lv.push_back(std::move(first));
    int maxl = o.max_levels > 0 ? o.max_levels : 64;
    // the branch's jobs look levels up while this thread appends new ones:
    // the level table must not move (past its reserve, an append first
    // waits for the branch)
    H->lv.reserve((size_t)std::min(maxl, 256) + 1);
    Branch br(s);
    for (int l = 0;; ++l) {
        TraceRange trace_level("setup level %d", l);
        Level &L = H->L(l);
        int32_t n = L.n;
        tm.level = l;
        bool coarsest = (o.truncate_n > 0 && n <= o.truncate_n) || l == maxl - 1;
        // below the top, A's entry count is an upper bound until read: with
        // the splitting's counts, or on its own for a coarsest level
        const bool bound = l > 0;
        ExtractPlan xplan;
        int32_t xtot[3] = {0, 0, 0};
        if (!coarsest) {
            tm.begin(AIRG_PHASE_CF);
            int64_t nz = 0;
            auto [nF, nC] = split(view(L.A), o, seed, l, L.cf, L.rank, s, bound ? &nz : nullptr, &xplan, xtot);
            if (bound) L.A.nnz = nz;
            L.nF = nF;
            L.nC = nC;
            L.setup_bytes += split_bytes(view(L.A));
            tm.end();
            if (nF == 0 || nC < o.poly_order) coarsest = true;
        } else if (bound) {
            int32_t nz = 0;
            d2h(&nz, L.A.rp.p + n, 1, s);
            L.A.nnz = nz;
        }
        if (coarsest) {
            tm.begin(AIRG_PHASE_POLY);
            L.coarsest = true;
            L.cf.reset();
            L.rank.reset();
            L.nF = n;
            L.nC = 0;
            int m = o.coarse_poly_order + 1;
            L.poly = gmres_poly(view(L.A), seed, l, m, s);
            L.setup_bytes += poly_bytes(view(L.A), m);
            if (!o.coarse_matrix_free) {
                L.Ainv = assemble_inverse(view(L.A), L.poly, m, o.poly_sparsity_order, s);
                L.setup_bytes += csr_bytes(view(L.A)) + csr_bytes(view(L.Ainv));
            }
            tm.end();
            break;
        }
        auto next = std::make_unique<Level>();
        // after the prolongator, the branch makes this level's permutation
        // and the previous level's solve operators, which need it; that work
        // overlaps this level's coarse phase and the next splitting
        Hier &HH = *H;
        auto pre = [&HH, l](hipStream_t st) {
            level_perm(HH.L(l), st);
            if (l > 0) solve_ops(HH, l - 1, st);
        };
        complete_level(view(L.A), o, seed, l, nullptr, L.cf.p, L.rank.p, L.nF, L.nC, L.fidx, L.cidx, L.Aff, &L.Afc,
                       L.poly, L.Ainv, L.Z, L.W, next->A, tm, s, &br, pre, &xplan, xtot, &L.setup_bytes, &L.Acf,
                       &L.P, &L.APp);
        L.xplan = std::move(xplan);
        next->n = next->A.nr;
        if (H->lv.size() == H->lv.capacity()) br.wait_idle();
        H->lv.push_back(std::move(next));
    }
    br.finish();
    tm.level = -1;
    tm.begin(AIRG_PHASE_FINALIZE);
    finalize(*H, std::max(0, H->nlev() - 2));
    Hier &HH = *H;
    tm.collect(H->phase, [&HH](int l, int ph, double sec) { HH.L(l).phase[ph] += sec; });
    H->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return H;
}

// ----------------------------------------------------- numeric re-setup --
// The CF splittings, the pattern of every level operator (after its drop),
// the patterns of Z and W, the extraction plan and the pattern of A P are
// kept; the values are recomputed level by level from the new top-level
// values: the blocks, coefficients and Ainv, Z = -A_cf Ainv, A P and
// A_c = R (A P) on the kept patterns (no drops), then the values of the solve
// operators.  The first re-setup bins the rows of the kept patterns for the
// assembly and the products (one host synchronisation each); later ones only
// synchronise for the polynomial's R factor.
void resetup_hierarchy(Hier &H, const double *vals, hipStream_t s) {
    TraceRange trace("airg re-setup");
    auto t0 = std::chrono::steady_clock::now();
    H.s = s;
    const airg_opts &o = H.opt;
    const int m = o.poly_order + 1, mc = o.coarse_poly_order + 1;
    Level &T = H.L(0);
    d2d(T.A.v.p, vals, (size_t)T.A.nnz, s);
    for (int l = 0; l < H.nlev(); ++l) {
        Level &L = H.L(l);
        if (L.coarsest) {
            L.poly = gmres_poly(view(L.A), H.seed, l, mc, s);
            if (!o.coarse_matrix_free) {
                if (!L.rbins) {
                    L.rb_ainv = poly_pattern_bins(view(L.Ainv), s);
                    L.rbins = true;
                }
                poly_fixed_sparsity_binned(view(L.A), view(L.Ainv), L.poly.alpha, mc, L.Ainv.v.p, L.rb_ainv, s);
            }
            break;
        }
        Level &N = H.L(l + 1);
        AIRG_REQUIRE(L.xplan.n == L.n && L.P.rp.p && L.APp.rp.p && L.Acf.rp.p, ST_INVALID_ARG,
                     "hierarchy has no kept patterns for a numeric re-setup");
        if (!L.rbins) {
            L.rb_ainv = poly_pattern_bins(view(L.Ainv), s);
            L.rb_z = pattern_bins(L.Z, s);
            L.rb_ap = pattern_bins(L.APp, s);
            L.rb_rap = pattern_bins(N.A, s);
            L.rbins = true;
        }
        extract_refill(view(L.A), L.cf.p, L.rank.p, L.nF, L.nC, L.xplan, L.Aff, L.Afc, L.Acf, s);
        L.poly = gmres_poly(view(L.Aff), H.seed, l, m, s);
        poly_fixed_sparsity_binned(view(L.Aff), view(L.Ainv), L.poly.alpha, m, L.Ainv.v.p, L.rb_ainv, s);
        spgemm_on_pattern_binned(view(L.Acf), view(L.Ainv), view(L.Z), L.rb_z, -1.0, L.Z.v.p, s);
        if (o.onepoint_weight == 1) {
            onepoint_values(view(L.A), L.fidx.p, L.cidx.p, L.W, s);
            L.P = prolongator_from_w(L.W, L.cf.p, L.rank.p, L.n, L.nC, s);
        }
        Csr R = restriction_full(view(L.Z), L.fidx.p, L.cidx.p, L.n, s);
        DBuf<double> apv((size_t)L.APp.nnz, s);
        CsrView AP = view(L.APp);
        AP.v = apv.p;
        spgemm_on_pattern_binned(view(L.A), view(L.P), AP, L.rb_ap, 1.0, apv.p, s);
        spgemm_on_pattern_binned(view(R), AP, view(N.A), L.rb_rap, 1.0, N.A.v.p, s);
    }
    refresh_solve_values(H);
    AIRG_HIP(hipStreamSynchronize(s));
    H.resetup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

LevelOut build_one_level(const CsrView &A, const airg_opts &o, uint64_t seed, int level, const double *alpha_in,
                         hipStream_t s) {
    LevelOut out;
    DBuf<int32_t> rank;
    auto [nF, nC] = split(A, o, seed, level, out.cf, rank, s);
    out.nF = nF;
    out.nC = nC;
    DBuf<int32_t> fidx, cidx;
    Csr Aff;
    NullTimer tm;
    complete_level(A, o, seed, level, alpha_in, out.cf.p, rank.p, nF, nC, fidx, cidx, Aff, nullptr, out.poly,
                   out.Ainv, out.Z, out.W, out.Ac, tm, s);
    return out;
}

// ------------------------------------------------------------- metrics ---
int64_t spmv_bytes(int64_t rows, int64_t cols, int64_t nnz, int vbytes, bool reads_y) {
    return nnz * (vbytes + 4) + 4 * (rows + 1) + (int64_t)vbytes * (cols + rows + (reads_y ? rows : 0));
}

// One V-cycle's products: stored entries, index bytes (columns and row
// pointers) and vector entries read or written per right-hand side.
void CycleCost::add(int64_t rows, int64_t cols, int64_t nz, bool reads_y, int64_t times) {
    nnz += times * nz;
    index_bytes += times * (4 * nz + 4 * (rows + 1));
    vec_entries += times * (cols + rows + (reads_y ? rows : 0));
}

CycleCost vcycle_cost(const Hier &H) {
    CycleCost c;
    for (int l = 0; l < (int)H.lv.size(); ++l) {
        const Level &L = *H.lv[l];
        if (L.coarsest) {
            const int vc = H.opt.coarse_iters;
            if (H.opt.coarse_matrix_free) {
                // vc applications of q(A): m - 1 products each; vc - 1 residuals
                c.add(L.n, L.n, L.A.nnz, false, (int64_t)vc * (L.poly.m - 1));
                c.add(L.n, L.n, L.A.nnz, true, vc - 1);
                continue;
            }
            // e = Ainv g, then (vc - 1) times: t = g - A e; e += Ainv t
            c.add(L.n, L.n, L.Ainv.nnz, false, 1);
            c.add(L.n, L.n, L.A.nnz, true, vc - 1);
            c.add(L.n, L.n, L.Ainv.nnz, true, vc - 1);
            continue;
        }
        c.add(L.Rp.nr, L.Rp.nc, L.Rp.nnz, false, 1);
        c.add(L.Pp.nr, L.Pp.nc, L.Pp.nnz, false, 1);
        c.add(L.AF.nr, L.AF.nc, L.AF.nnz, true, H.opt.up_smooths);
        c.add(L.Ainv.nr, L.Ainv.nc, L.Ainv.nnz, true, H.opt.up_smooths);
    }
    return c;
}

int64_t vcycle_bytes(const Hier &H, int vb) { return vcycle_cost(H).bytes(vb, 1); }

int64_t vcycle_nnz(const Hier &H) { return vcycle_cost(H).nnz; }

void complexities(const Hier &H, double *grid, double *op, double *storage) {
    const Level &T = *H.lv[0];
    double n0 = T.n, z0 = (double)T.A.nnz, g = 0, o = 0, st = 0;
    for (auto &lp : H.lv) {
        const Level &L = *lp;
        g += L.n;
        o += (double)L.A.nnz;
        if (L.coarsest) {
            st += (double)L.Ainv.nnz + (H.opt.coarse_iters > 1 || H.opt.coarse_matrix_free ? (double)L.A.nnz : 0.0);
        } else {
            st += (double)L.Ainv.nnz + (double)L.Aff.nnz + (double)L.Afc.nnz + (double)(L.Z.nnz + L.nC) +
                  (double)(L.W.nnz + L.nC);
        }
    }
    *grid = g / n0;
    *op = o / z0;
    *storage = st / z0;
}

}  // namespace airg

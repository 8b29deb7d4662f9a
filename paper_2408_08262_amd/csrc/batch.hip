// Batched AIRG: concatenated per-level operators of many segments, the
// batched FP32 V-cycle (one SpMM launch per stage, captured as a HIP graph),
// a self-written autotuner for the SpMM kernel choice, and FGMRES over every
// (segment, right-hand side) pair.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>

#include "batch.hpp"
#include "csr.hpp"
#include "trace.hpp"

namespace airg {

// --------------------------------------------------------------- layouts --
namespace {

// Position map of one segment's level order into the batch level layout:
// q < split -> fbase + q, else cbase + (q - split).
struct Map {
    int32_t split = INT_MAX, fbase = 0, cbase = 0;
};

__host__ __device__ inline int32_t apply_map(int32_t q, const Map &m) {
    return q < m.split ? m.fbase + q : m.cbase + (q - m.split);
}

struct PlaceDesc {
    const int32_t *rp;
    const int32_t *ci;
    const double *v;
    int32_t nrows;
    Map rmap, cmap;
};

__device__ inline int find_seg(const int64_t *pre, int nseg, int64_t t) {
    int lo = 0, hi = nseg;   // last p with pre[p] <= t
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_place_count(const PlaceDesc *__restrict__ d, const int64_t *__restrict__ pre, int nseg,
                              int32_t *__restrict__ cnt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pre[nseg]) return;
    int p = find_seg(pre, nseg, t);
    int32_t q = (int32_t)(t - pre[p]);
    const PlaceDesc &D = d[p];
    cnt[apply_map(q, D.rmap)] = D.rp[q + 1] - D.rp[q];
}

__global__ void k_place_fill(const PlaceDesc *__restrict__ d, const int64_t *__restrict__ pre, int nseg,
                             const int32_t *__restrict__ orp, int32_t *__restrict__ oci, double *__restrict__ ov) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pre[nseg]) return;
    int p = find_seg(pre, nseg, t);
    int32_t q = (int32_t)(t - pre[p]);
    const PlaceDesc &D = d[p];
    int32_t w = orp[apply_map(q, D.rmap)];
    for (int32_t k = D.rp[q]; k < D.rp[q + 1]; ++k, ++w) {
        oci[w] = apply_map(D.ci[k], D.cmap);
        ov[w] = D.v[k];
    }
}

// Concatenates the given segment blocks into one nr x nc CSR.
Csr place(const std::vector<PlaceDesc> &descs, int32_t nr, int32_t nc, hipStream_t s) {
    Csr C;
    C.nr = nr;
    C.nc = nc;
    C.rp.alloc((size_t)nr + 1, s);
    std::vector<int64_t> pre(descs.size() + 1, 0);
    for (size_t p = 0; p < descs.size(); ++p) pre[p + 1] = pre[p] + descs[p].nrows;
    DBuf<int32_t> cnt((size_t)nr + 1, s);
    fill_zero(cnt.p, ((size_t)nr + 1) * 4, s);
    if (pre.back() > 0) {
        DBuf<PlaceDesc> dd(descs.size(), s);
        DBuf<int64_t> dp(pre.size(), s);
        h2d(dd.p, descs.data(), descs.size(), s);
        h2d(dp.p, pre.data(), pre.size(), s);
        k_place_count<<<grid_for(pre.back(), 256), 256, 0, s>>>(dd.p, dp.p, (int)descs.size(), cnt.p);
        AIRG_LAUNCH_CHECK();
        C.nnz = exclusive_scan(cnt.p, C.rp.p, nr, s);
        C.ci.alloc((size_t)C.nnz, s);
        C.v.alloc((size_t)C.nnz, s);
        k_place_fill<<<grid_for(pre.back(), 256), 256, 0, s>>>(dd.p, dp.p, (int)descs.size(), C.rp.p, C.ci.p, C.v.p);
        AIRG_LAUNCH_CHECK();
        AIRG_HIP(hipStreamSynchronize(s));   // descriptors are freed on return
    } else {
        C.nnz = exclusive_scan(cnt.p, C.rp.p, nr, s);
        C.ci.alloc(0, s);
        C.v.alloc(0, s);
    }
    make_f32(C, s);
    return C;
}

PlaceDesc desc(const Csr &M, Map r, Map c) { return PlaceDesc{M.rp.p, M.ci.p, M.v.p, M.nr, r, c}; }

__global__ void k_perm0(int32_t n, const int32_t *__restrict__ perm, Map m, int32_t *__restrict__ out) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = apply_map(perm ? perm[i] : i, m);
}

// --------------------------------------------------------------- autotune --
// Candidate kernels for one operator: the persistent CSR-stream kernel (0)
// and G lanes per row (G = 1 .. 32).  Each is timed with events over a few
// launches on the real operator; the fastest is kept, and remembered by
// shape ("rows:nnz:k") in memory and, when AIRG_TUNE_CACHE names a file, on
// disk as a flat JSON object.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_path() {
    const char *p = std::getenv("AIRG_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::string path = tune_path();
    if (path.empty()) return;
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        std::string key = t.substr(i + 1, j - i - 1);
        size_t c = t.find(':', j);
        if (c == std::string::npos) break;
        g_tune_cache[key] = std::atoi(t.c_str() + c + 1);
        i = t.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
}

void tune_save() {
    std::string path = tune_path();
    if (path.empty()) return;
    std::ofstream f(path);
    f << "{";
    bool first = true;
    for (auto &kv : g_tune_cache) {
        f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
        first = false;
    }
    f << "}\n";
}

int autotune(const Csr &M, int k, float *x, float *y, std::map<std::string, int> &rec, hipStream_t s) {
    if (M.nr == 0) return -1;
    std::string key = std::to_string(M.nr) + ":" + std::to_string(M.nnz) + ":" + std::to_string(k);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            rec[key] = it->second;
            return it->second;
        }
    }
    const int cands[] = {0, 1, 2, 4, 8, 16, 32};
    hipEvent_t a, b;
    AIRG_HIP(hipEventCreate(&a));
    AIRG_HIP(hipEventCreate(&b));
    int best = -1;
    float best_ms = 1e30f;
    for (int c : cands) {
        spmm32(view(M), k, x, y, nullptr, SPMV_SET, s, c);   // warm
        AIRG_HIP(hipEventRecord(a, s));
        for (int r = 0; r < 3; ++r) spmm32(view(M), k, x, y, nullptr, SPMV_SET, s, c);
        AIRG_HIP(hipEventRecord(b, s));
        AIRG_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        AIRG_HIP(hipEventElapsedTime(&ms, a, b));
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    rec[key] = best;
    tune_save();
    return best;
}

}  // namespace

Batch::~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
}

// -------------------------------------------------------------- building --
std::unique_ptr<Batch> build_batch(std::vector<std::unique_ptr<Hier>> &segs, int k, bool tune, hipStream_t s) {
    auto B = std::make_unique<Batch>();
    int nseg = (int)segs.size();
    B->k = k;
    B->nseg = nseg;
    B->coarse_iters = segs[0]->opt.coarse_iters;
    B->up_smooths = segs[0]->opt.up_smooths;
    int depth = 0;
    for (auto &h : segs) depth = std::max(depth, h->nlev());
    // per level: kinds and maps
    std::vector<std::vector<int>> kind(depth, std::vector<int>(nseg, 0));   // 0 absent, 1 active, 2 terminal
    std::vector<std::vector<Map>> lmap(depth, std::vector<Map>(nseg));      // level layout map
    std::vector<std::vector<Map>> fmap(depth, std::vector<Map>(nseg));      // F rows (active) / terminal-relative
    for (int l = 0; l < depth; ++l) {
        auto BL = std::make_unique<BatchLevel>();
        for (int p = 0; p < nseg; ++p) {
            Hier &H = *segs[p];
            if (l >= H.nlev()) continue;
            Level &L = H.L(l);
            kind[l][p] = L.coarsest ? 2 : 1;
            if (!L.coarsest) {
                BL->nF += L.nF;
                BL->nC += L.nC;
            } else {
                BL->nT += L.n;
            }
        }
        int32_t fo = 0, co = 0, to = 0;
        for (int p = 0; p < nseg; ++p) {
            if (!kind[l][p]) continue;
            Level &L = segs[p]->L(l);
            if (kind[l][p] == 1) {
                lmap[l][p] = Map{L.nF, fo, BL->nF + co};
                fmap[l][p] = Map{INT_MAX, fo, 0};
                fo += L.nF;
                co += L.nC;
            } else {
                lmap[l][p] = Map{INT_MAX, BL->nF + BL->nC + to, 0};
                fmap[l][p] = Map{INT_MAX, to, 0};
                to += L.n;
            }
        }
        B->lv.push_back(std::move(BL));
    }
    for (int l = 0; l < depth; ++l) {
        BatchLevel &BL = *B->lv[l];
        std::vector<PlaceDesc> dAF, dAinv, dRp, dPp, dAT, dAinvT;
        for (int p = 0; p < nseg; ++p) {
            if (!kind[l][p]) continue;
            Level &L = segs[p]->L(l);
            if (kind[l][p] == 1) {
                dAF.push_back(desc(L.AF, fmap[l][p], lmap[l][p]));
                dAinv.push_back(desc(L.Ainv, fmap[l][p], fmap[l][p]));
                dRp.push_back(desc(L.Rp, lmap[l + 1][p], lmap[l][p]));
                dPp.push_back(desc(L.Pp, lmap[l][p], lmap[l + 1][p]));
            } else {
                dAT.push_back(desc(L.A, fmap[l][p], fmap[l][p]));
                dAinvT.push_back(desc(L.Ainv, fmap[l][p], fmap[l][p]));
            }
        }
        int32_t nl = BL.n();
        int32_t nnext = l + 1 < depth ? B->lv[l + 1]->n() : 0;
        if (!dAF.empty()) {
            BL.AF = place(dAF, BL.nF, nl, s);
            BL.Ainv = place(dAinv, BL.nF, BL.nF, s);
            BL.Rp = place(dRp, nnext, nl, s);
            BL.Pp = place(dPp, BL.nF + BL.nC, nnext, s);
        }
        if (!dAT.empty()) {
            BL.AT = place(dAT, BL.nT, BL.nT, s);
            BL.AinvT = place(dAinvT, BL.nT, BL.nT, s);
        }
    }
    // natural rows -> level-0 positions
    int64_t n = 0;
    for (auto &h : segs) n += h->L(0).n;
    B->n = n;
    B->perm0.alloc((size_t)n, s);
    int64_t off = 0;
    for (int p = 0; p < nseg; ++p) {
        Level &L = segs[p]->L(0);
        k_perm0<<<grid_for(L.n, 256), 256, 0, s>>>(L.n, L.coarsest ? nullptr : L.perm.p, lmap[0][p], B->perm0.p + off);
        AIRG_LAUNCH_CHECK();
        off += L.n;
    }
    finish_batch(*B, tune, s);
    return B;
}

void finish_batch(Batch &Bt, bool tune, hipStream_t s) {
    Batch *B = &Bt;
    const int k = B->k;
    for (auto &lp : B->lv) {
        BatchLevel &BL = *lp;
        int32_t nl = BL.n();
        BL.g.alloc((size_t)nl * k, s);
        BL.e.alloc((size_t)nl * k, s);
        BL.t.alloc((size_t)nl * k, s);
        fill_zero(BL.g.p, BL.g.bytes(), s);
        fill_zero(BL.e.p, BL.e.bytes(), s);
        fill_zero(BL.t.p, BL.t.bytes(), s);
    }
    B->g0.alloc((size_t)B->n * k, s);
    B->e0.alloc((size_t)B->n * k, s);
    fill_zero(B->g0.p, B->g0.bytes(), s);
    fill_zero(B->e0.p, B->e0.bytes(), s);
    if (tune) {
        for (auto &lp : B->lv) {
            BatchLevel &BL = *lp;
            float *x = BL.g.p, *y = BL.t.p;
            BL.lAF = autotune(BL.AF, k, BL.e.p, y, B->tuned, s);
            BL.lAinv = autotune(BL.Ainv, k, BL.t.p, BL.e.p, B->tuned, s);
            BL.lAT = autotune(BL.AT, k, BL.e.p, y, B->tuned, s);
            BL.lAinvT = autotune(BL.AinvT, k, x, BL.e.p, B->tuned, s);
        }
        for (size_t l = 0; l + 1 < B->lv.size(); ++l) {
            BatchLevel &BL = *B->lv[l], &NX = *B->lv[l + 1];
            BL.lRp = autotune(BL.Rp, k, BL.g.p, NX.g.p, B->tuned, s);
            BL.lPp = autotune(BL.Pp, k, NX.e.p, BL.e.p, B->tuned, s);
        }
        for (auto &lp : B->lv) {
            fill_zero(lp->g.p, lp->g.bytes(), s);
            fill_zero(lp->e.p, lp->e.bytes(), s);
            fill_zero(lp->t.p, lp->t.bytes(), s);
        }
    }
    AIRG_HIP(hipStreamSynchronize(s));
}

// --------------------------------------------------------------- V-cycle --
// Level l, vectors n_l x k in the batch layout:
//   active part:  g' = R g;  e' = V(g');  e[F,C] = P e';
//                 up_smooths times: e_F += Ainv (g_F - AF e)
//   terminal part: e_T = Ainv_T g_T, then (coarse_iters - 1) times
//                 e_T += Ainv_T (g_T - A_T e_T).
void Batch::vcycle(int l, const float *g, float *e, hipStream_t s) {
    BatchLevel &BL = *lv[l];
    float *t = BL.t.p;
    auto mark = [&](int q) {
        if (prof) AIRG_HIP(hipEventRecord(prof[4 * l + q], s));
    };
    mark(0);
    if (BL.nF + BL.nC > 0) {
        BatchLevel &NX = *lv[l + 1];
        spmm32(view(BL.Rp), k, g, NX.g.p, nullptr, SPMV_SET, s, BL.lRp);
        mark(1);
        vcycle(l + 1, NX.g.p, NX.e.p, s);
        mark(2);
        spmm32(view(BL.Pp), k, NX.e.p, e, nullptr, SPMV_SET, s, BL.lPp);
        for (int q = 0; q < up_smooths; ++q) {
            spmm32(view(BL.AF), k, e, t, g, SPMV_ZMINUS, s, BL.lAF);
            spmm32(view(BL.Ainv), k, t, e, nullptr, SPMV_ADD, s, BL.lAinv);
        }
    }
    if (BL.nT > 0) {
        int64_t o = (int64_t)(BL.nF + BL.nC) * k;
        spmm32(view(BL.AinvT), k, g + o, e + o, nullptr, SPMV_SET, s, BL.lAinvT);
        for (int it = 1; it < coarse_iters; ++it) {
            spmm32(view(BL.AT), k, e + o, t + o, g + o, SPMV_ZMINUS, s, BL.lAT);
            spmm32(view(BL.AinvT), k, t + o, e + o, nullptr, SPMV_ADD, s, BL.lAinvT);
        }
    }
    if (BL.nF + BL.nC == 0) {
        mark(1);
        mark(2);
    }
    mark(3);
}

void batch_profile(Batch &B, int reps, double *out, hipStream_t s) {
    const int nl = (int)B.lv.size();
    for (int l = 0; l < nl; ++l) out[l] = 0.0;
    std::vector<hipEvent_t> ev((size_t)4 * nl);
    for (auto &e : ev) e = pooled_event();
    try {
        fill_zero(B.g0.p, B.g0.bytes(), s);
        for (int r = 0; r < reps; ++r) {
            B.prof = ev.data();
            B.vcycle(0, B.g0.p, B.e0.p, s);
            B.prof = nullptr;
            AIRG_HIP(hipStreamSynchronize(s));
            for (int l = 0; l < nl; ++l) {
                float a = 0.f, b = 0.f;
                AIRG_HIP(hipEventElapsedTime(&a, ev[4 * l], ev[4 * l + 1]));
                AIRG_HIP(hipEventElapsedTime(&b, ev[4 * l + 2], ev[4 * l + 3]));
                out[l] += (a + b) * 1e-3 / reps;
            }
        }
    } catch (...) {
        B.prof = nullptr;
        for (auto &e : ev) release_event(e);
        throw;
    }
    for (auto &e : ev) release_event(e);
}

// The graph is captured once on a private non-blocking stream (the legacy
// default stream cannot be captured) and then launched on the caller's
// stream; it holds only kernel nodes over the batch's own buffers.
void Batch::run(hipStream_t s, bool use_graph) {
    TraceRange trace("batched V-cycle fp32");
    if (!use_graph) {
        ++cycles_eager;
        vcycle(0, g0.p, e0.p, s);
        return;
    }
    if (!exec) {
        if (!cap) AIRG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        AIRG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
        try {
            vcycle(0, g0.p, e0.p, cap);
        } catch (...) {
            hipGraph_t dummy = nullptr;
            (void)hipStreamEndCapture(cap, &dummy);
            if (dummy) (void)hipGraphDestroy(dummy);
            throw;
        }
        AIRG_HIP(hipStreamEndCapture(cap, &graph));
        AIRG_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    ++cycles_graph;
    AIRG_HIP(hipGraphLaunch(exec, s));
}

// ------------------------------------------------------- batched FGMRES ---
namespace {

constexpr int kTile = 2048;

// Block reduction of per-thread sums whose column is c = threadIdx.x % K
// (256 % K == 0): lanes of equal column combine by shuffles, then the four
// wavefronts through LDS; returns the total on threads 0..K-1 (their own c).
template <int K>
__device__ inline double col_block_sum(double x, double (*sh)[8]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int o = 32; o >= K; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane < K) sh[wid][lane] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < K) t = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
    __syncthreads();
    return t;
}

// partial[(tile * nvec + i) * k + c] = sum over the tile's rows of V_i[r,c] W[r,c].
// Vectors are taken kDotGroup at a time, so W is read once per group.
constexpr int kDotGroup = 8;
template <int K>
__global__ void __launch_bounds__(256) k_segdot(const double *__restrict__ V, int64_t vstride, int nvec,
                                                const double *__restrict__ W, const int64_t *__restrict__ trow,
                                                double *__restrict__ partial) {
    __shared__ double sh[4][8];
    const int64_t e0 = trow[blockIdx.x] * K, e1 = trow[blockIdx.x + 1] * K;
    for (int i0 = 0; i0 < nvec; i0 += kDotGroup) {
        double acc[kDotGroup];
#pragma unroll
        for (int v = 0; v < kDotGroup; ++v) acc[v] = 0.0;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
            const double w = W[e];
#pragma unroll
            for (int v = 0; v < kDotGroup; ++v)
                if (i0 + v < nvec) acc[v] += V[(int64_t)(i0 + v) * vstride + e] * w;
        }
#pragma unroll
        for (int v = 0; v < kDotGroup; ++v) {
            if (i0 + v < nvec) {
                const double t = col_block_sum<K>(acc[v], sh);
                if (threadIdx.x < K) partial[((int64_t)blockIdx.x * nvec + i0 + v) * K + threadIdx.x] = t;
            }
        }
    }
}

// One pass of classical Gram-Schmidt fused with what follows it:
//   W[r,c] -= sum_i V_i[r,c] H[(i * nseg + p(r)) * K + c]
// and then, per tile, either the dots of the V_i with the new W (DOTS: the
// second Gram-Schmidt pass's coefficients) into partial[(tile * nvec + i) *
// K + c], or the squared norm of the new W into partial[tile * K + c].  Each
// thread keeps the V_i of its element in registers between the update and
// the dots, so V is read from memory once (NV >= nvec bounds the registers).
// Tiles lie in one segment.
constexpr int kMaxKrylov = 32;
template <int K, bool DOTS, int NV>
__global__ void __launch_bounds__(256) k_seg_update_fused(const double *__restrict__ V, int64_t vstride, int nvec,
                                                          const double *__restrict__ H, int nseg,
                                                          const int32_t *__restrict__ segrow,
                                                          double *__restrict__ W, const int64_t *__restrict__ trow,
                                                          double *__restrict__ partial) {
    __shared__ double sh[4][8];
    const int64_t r0 = trow[blockIdx.x];
    const int64_t e0 = r0 * K, e1 = trow[blockIdx.x + 1] * K;
    const int c = threadIdx.x % K;
    const int p = segrow[r0];
    double h[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = i < nvec ? H[((int64_t)i * nseg + p) * K + c] : 0.0;
    double acc[DOTS ? NV : 1];
#pragma unroll
    for (int i = 0; i < (DOTS ? NV : 1); ++i) acc[i] = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        double vv[NV];
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            vv[i] = i < nvec ? V[(int64_t)i * vstride + e] : 0.0;
            if (i < nvec) sum += vv[i] * h[i];
        }
        const double w = W[e] - sum;
        W[e] = w;
        if (DOTS) {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < nvec) acc[i] += vv[i] * w;
        } else {
            acc[0] += w * w;
        }
    }
#pragma unroll
    for (int i = 0; i < (DOTS ? NV : 1); ++i) {
        if (i < (DOTS ? nvec : 1)) {
            const double t = col_block_sum<K>(acc[i], sh);
            if (threadIdx.x < K) partial[((int64_t)blockIdx.x * (DOTS ? nvec : 1) + i) * K + threadIdx.x] = t;
        }
    }
}

// out[(i * nseg + p) * K + c] = sum over segment p's tiles: one workgroup per
// (i, p), its threads striding over the tiles, then a workgroup reduction.
template <int K>
__global__ void __launch_bounds__(256) k_segdot_finish(const double *__restrict__ partial,
                                                       const int32_t *__restrict__ segtile, int nseg, int nvec,
                                                       double *__restrict__ out) {
    __shared__ double sh[4][8];
    const int i = blockIdx.x / nseg, p = blockIdx.x % nseg;
    const int c = threadIdx.x % K;
    double x = 0.0;
    for (int q = segtile[p] + threadIdx.x / K; q < segtile[p + 1]; q += 256 / K)
        x += partial[((int64_t)q * nvec + i) * K + c];
    const double t = col_block_sum<K>(x, sh);
    if (threadIdx.x < K) out[((int64_t)i * nseg + p) * K + threadIdx.x] = t;
}

// W[r,c] += sign * sum_i V_i[r,c] H[(i * nseg + p(r)) * k + c]
__global__ void k_seg_update(const double *__restrict__ V, int64_t vstride, int nvec, const double *__restrict__ H,
                             const int32_t *__restrict__ segrow, int nseg, int k, double sign, double *__restrict__ W,
                             int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int64_t r = t / k;
    int c = (int)(t % k);
    int p = segrow[r];
    double s = 0.0;
    for (int i = 0; i < nvec; ++i) s += V[(int64_t)i * vstride + t] * H[((int64_t)i * nseg + p) * k + c];
    W[t] += sign * s;
}

// dst[r,c] = src[r,c] * S[p(r) * k + c]
__global__ void k_seg_scale(const double *__restrict__ src, const double *__restrict__ S,
                            const int32_t *__restrict__ segrow, int k, double *__restrict__ dst, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    dst[t] = src[t] * S[(int64_t)segrow[t / k] * k + (t % k)];
}

__global__ void k_gather_cast(const double *__restrict__ r, const int32_t *__restrict__ perm, int k,
                              float *__restrict__ g, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int64_t i = t / k;
    g[(int64_t)perm[i] * k + (t % k)] = (float)r[t];
}
__global__ void k_scatter_cast(const float *__restrict__ e, const int32_t *__restrict__ perm, int k,
                               double *__restrict__ z, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int64_t i = t / k;
    z[t] = (double)e[(int64_t)perm[i] * k + (t % k)];
}

__global__ void k_segrow(int32_t lo, int32_t hi, int32_t p, int32_t *__restrict__ segrow) {
    int32_t i = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < hi) segrow[i] = p;
}

struct SegDots {
    int nseg, k;
    int64_t n;
    DBuf<int64_t> trow;
    DBuf<int32_t> segtile;
    int ntile;
    DBuf<double> partial, out;
    int maxvec;
    SegDots(const std::vector<int64_t> &seg, int kk, int64_t nn, int maxv, hipStream_t s)
        : nseg((int)seg.size() - 1), k(kk), n(nn), maxvec(maxv) {
        std::vector<int64_t> tr;
        std::vector<int32_t> st;
        for (int p = 0; p < nseg; ++p) {
            st.push_back((int32_t)tr.size());
            for (int64_t r = seg[p]; r < seg[p + 1]; r += kTile) tr.push_back(r);
        }
        st.push_back((int32_t)tr.size());
        ntile = (int)tr.size();
        tr.push_back(seg[nseg]);
        trow.alloc(tr.size(), s);
        segtile.alloc(st.size(), s);
        h2d(trow.p, tr.data(), tr.size(), s);
        h2d(segtile.p, st.data(), st.size(), s);
        partial.alloc((size_t)ntile * maxvec * k, s);
        out.alloc((size_t)maxvec * nseg * k, s);
    }
    // dots of V_0..V_{nvec-1} with W per (segment, column) into host h
    void run(const double *V, int64_t vstride, int nvec, const double *W, double *h, hipStream_t s) {
        switch (k) {
        case 1: k_segdot<1><<<ntile, 256, 0, s>>>(V, vstride, nvec, W, trow.p, partial.p); break;
        case 2: k_segdot<2><<<ntile, 256, 0, s>>>(V, vstride, nvec, W, trow.p, partial.p); break;
        case 4: k_segdot<4><<<ntile, 256, 0, s>>>(V, vstride, nvec, W, trow.p, partial.p); break;
        case 8: k_segdot<8><<<ntile, 256, 0, s>>>(V, vstride, nvec, W, trow.p, partial.p); break;
        default: throw Error(ST_INVALID_ARG, "batched solve supports 1, 2, 4 or 8 right-hand sides");
        }
        AIRG_LAUNCH_CHECK();
        finish(nvec, h, s);
    }
    // W -= sum_i V_i H_i per pair, then (DOTS) the dots of V_0..V_{nvec-1}
    // with the new W, or its squared norm, per (segment, column) into host h
    template <bool DOTS>
    void update(const double *V, int64_t vstride, int nvec, const double *Hd, const int32_t *segrow, double *W,
                double *h, hipStream_t s) {
        AIRG_REQUIRE(nvec <= kMaxKrylov, ST_INVALID_ARG, "Krylov basis too long for the fused update");
        auto launch = [&]<int K>() {
            if (nvec <= 8) k_seg_update_fused<K, DOTS, 8><<<ntile, 256, 0, s>>>(V, vstride, nvec, Hd, nseg, segrow, W, trow.p, partial.p);
            else if (nvec <= 16) k_seg_update_fused<K, DOTS, 16><<<ntile, 256, 0, s>>>(V, vstride, nvec, Hd, nseg, segrow, W, trow.p, partial.p);
            else k_seg_update_fused<K, DOTS, kMaxKrylov><<<ntile, 256, 0, s>>>(V, vstride, nvec, Hd, nseg, segrow, W, trow.p, partial.p);
        };
        switch (k) {
        case 1: launch.template operator()<1>(); break;
        case 2: launch.template operator()<2>(); break;
        case 4: launch.template operator()<4>(); break;
        case 8: launch.template operator()<8>(); break;
        default: throw Error(ST_INVALID_ARG, "batched solve supports 1, 2, 4 or 8 right-hand sides");
        }
        AIRG_LAUNCH_CHECK();
        finish(DOTS ? nvec : 1, h, s);
    }
    void finish(int nvec, double *h, hipStream_t s) {
        const unsigned blocks = (unsigned)(nvec * nseg);
        switch (k) {
        case 1: k_segdot_finish<1><<<blocks, 256, 0, s>>>(partial.p, segtile.p, nseg, nvec, out.p); break;
        case 2: k_segdot_finish<2><<<blocks, 256, 0, s>>>(partial.p, segtile.p, nseg, nvec, out.p); break;
        case 4: k_segdot_finish<4><<<blocks, 256, 0, s>>>(partial.p, segtile.p, nseg, nvec, out.p); break;
        default: k_segdot_finish<8><<<blocks, 256, 0, s>>>(partial.p, segtile.p, nseg, nvec, out.p); break;
        }
        AIRG_LAUNCH_CHECK();
        d2h(h, out.p, (size_t)nvec * nseg * k, s);
    }
};

}  // namespace

BatchResult solve_batch(Batch &B, const Csr &A, const std::vector<int64_t> &seg, const double *b, double *x,
                        double rtol, int maxit, int restart, bool use_graph, hipStream_t s) {
    TraceRange trace("airg batched solve: FGMRES");
    const int k = B.k, nseg = B.nseg;
    const int64_t n = B.n;
    const int np = nseg * k;   // (segment, rhs) pairs
    int m = std::max(1, std::min(restart > 0 ? restart : 30, std::max(maxit, 1)));
    m = std::min(m, kMaxKrylov - 1);   // the fused Gram-Schmidt passes keep the basis in registers
    BatchResult res;
    DBuf<int32_t> segrow((size_t)n, s);
    for (int p = 0; p < nseg; ++p) {
        k_segrow<<<grid_for(seg[p + 1] - seg[p], 256), 256, 0, s>>>((int32_t)seg[p], (int32_t)seg[p + 1], p, segrow.p);
        AIRG_LAUNCH_CHECK();
    }
    SegDots dots(seg, k, n, m + 1, s);
    int64_t nk = n * k;
    DBuf<double> V((size_t)nk * (m + 1), s), Zb((size_t)nk * m, s), r((size_t)nk, s), hd((size_t)(m + 1) * np, s);
    std::vector<double> bn(np), beta(np), tmp((size_t)(m + 1) * np), h1((size_t)(m + 1) * np),
        h2((size_t)(m + 1) * np);
    dots.run(b, 0, 1, b, bn.data(), s);
    for (auto &v : bn) v = std::sqrt(v);
    fill_zero(x, (size_t)nk * 8, s);
    d2d(r.p, b, (size_t)nk, s);
    for (int q = 0; q < np; ++q) beta[q] = bn[q];
    auto all_done = [&]() {
        for (int q = 0; q < np; ++q)
            if (beta[q] > rtol * bn[q]) return false;
        return true;
    };
    // per-pair Hessenberg, Givens and right-hand side
    std::vector<double> H((size_t)np * (m + 1) * m), cs((size_t)np * m), sn((size_t)np * m), gv((size_t)np * (m + 1)),
        y((size_t)np * m);
    while (!all_done() && res.iterations < maxit) {
        for (int q = 0; q < np; ++q) tmp[q] = beta[q] > 0.0 ? 1.0 / beta[q] : 0.0;
        h2d(hd.p, tmp.data(), (size_t)np, s);
        k_seg_scale<<<grid_for(nk, 256), 256, 0, s>>>(r.p, hd.p, segrow.p, k, V.p, n);
        AIRG_LAUNCH_CHECK();
        std::fill(gv.begin(), gv.end(), 0.0);
        for (int q = 0; q < np; ++q) gv[(size_t)q * (m + 1)] = beta[q];
        int j = 0;
        while (j < m && res.iterations < maxit) {
            double *vj = V.p + (int64_t)j * nk, *zj = Zb.p + (int64_t)j * nk, *w = V.p + (int64_t)(j + 1) * nk;
            // z_j = M v_j  (FP32 batched V-cycle)
            k_gather_cast<<<grid_for(nk, 256), 256, 0, s>>>(vj, B.perm0.p, k, B.g0.p, n);
            AIRG_LAUNCH_CHECK();
            B.run(s, use_graph);
            k_scatter_cast<<<grid_for(nk, 256), 256, 0, s>>>(B.e0.p, B.perm0.p, k, zj, n);
            AIRG_LAUNCH_CHECK();
            res.iterations++;
            spmm_top(view(A), k, zj, w, nullptr, SPMV_SET, s);
            // classical Gram-Schmidt twice, per pair: the first pass's dots; the
            // first update fused with the second pass's dots; the second update
            // fused with the new vector's squared norm (three passes over V)
            dots.run(V.p, nk, j + 1, w, h1.data(), s);
            h2d(hd.p, h1.data(), (size_t)(j + 1) * np, s);
            dots.update<true>(V.p, nk, j + 1, hd.p, segrow.p, w, h2.data(), s);
            h2d(hd.p, h2.data(), (size_t)(j + 1) * np, s);
            std::vector<double> hn(np);
            dots.update<false>(V.p, nk, j + 1, hd.p, segrow.p, w, hn.data(), s);
            for (int q = 0; q < np; ++q) {
                hn[q] = std::sqrt(hn[q]);
                AIRG_REQUIRE(std::isfinite(hn[q]), ST_STALL, "batched Arnoldi vector became non-finite");
                tmp[q] = hn[q] > 0.0 ? 1.0 / hn[q] : 0.0;
            }
            h2d(hd.p, tmp.data(), (size_t)np, s);
            k_seg_scale<<<grid_for(nk, 256), 256, 0, s>>>(w, hd.p, segrow.p, k, w, n);
            AIRG_LAUNCH_CHECK();
            bool done = true;
            for (int q = 0; q < np; ++q) {
                double *Hq = H.data() + (size_t)q * (m + 1) * m;
                double *cq = cs.data() + (size_t)q * m, *sq = sn.data() + (size_t)q * m, *gq = gv.data() + (size_t)q * (m + 1);
                for (int i = 0; i <= j; ++i) Hq[(size_t)i * m + j] = h1[(size_t)i * np + q] + h2[(size_t)i * np + q];
                Hq[(size_t)(j + 1) * m + j] = hn[q];
                for (int i = 0; i < j; ++i) {
                    double a = Hq[(size_t)i * m + j], c = Hq[(size_t)(i + 1) * m + j];
                    Hq[(size_t)i * m + j] = cq[i] * a + sq[i] * c;
                    Hq[(size_t)(i + 1) * m + j] = cq[i] * c - sq[i] * a;
                }
                double a = Hq[(size_t)j * m + j], c = Hq[(size_t)(j + 1) * m + j];
                double rr = std::hypot(a, c);
                cq[j] = rr > 0.0 ? a / rr : 1.0;
                sq[j] = rr > 0.0 ? c / rr : 0.0;
                Hq[(size_t)j * m + j] = rr;
                Hq[(size_t)(j + 1) * m + j] = 0.0;
                gq[j + 1] = -sq[j] * gq[j];
                gq[j] = cq[j] * gq[j];
                if (std::fabs(gq[j + 1]) > rtol * bn[q] && hn[q] > 0.0) done = false;
            }
            ++j;
            if (done) break;
        }
        // y per pair, then x += sum_i Z_i y_i
        for (int q = 0; q < np; ++q) {
            double *Hq = H.data() + (size_t)q * (m + 1) * m, *gq = gv.data() + (size_t)q * (m + 1);
            double *yq = y.data() + (size_t)q * m;
            for (int i = j - 1; i >= 0; --i) {
                double t = gq[i];
                for (int c = i + 1; c < j; ++c) t -= Hq[(size_t)i * m + c] * yq[c];
                yq[i] = Hq[(size_t)i * m + i] != 0.0 ? t / Hq[(size_t)i * m + i] : 0.0;
            }
            for (int i = 0; i < j; ++i) tmp[(size_t)i * np + q] = yq[i];
        }
        h2d(hd.p, tmp.data(), (size_t)j * np, s);
        k_seg_update<<<grid_for(nk, 256), 256, 0, s>>>(Zb.p, nk, j, hd.p, segrow.p, nseg, k, 1.0, x, n);
        AIRG_LAUNCH_CHECK();
        spmm_top(view(A), k, x, r.p, b, SPMV_ZMINUS, s);
        dots.run(r.p, 0, 1, r.p, beta.data(), s);
        for (auto &v : beta) {
            v = std::sqrt(v);
            AIRG_REQUIRE(std::isfinite(v), ST_STALL, "batched residual became non-finite");
        }
    }
    res.converged = all_done();
    for (int q = 0; q < np; ++q) res.worst = std::max(res.worst, bn[q] > 0.0 ? beta[q] / bn[q] : 0.0);
    return res;
}

void batch_apply(Batch &B, const double *g, double *e, bool use_graph, hipStream_t s) {
    const int64_t nk = B.n * B.k;
    k_gather_cast<<<grid_for(nk, 256), 256, 0, s>>>(g, B.perm0.p, B.k, B.g0.p, B.n);
    AIRG_LAUNCH_CHECK();
    B.run(s, use_graph);
    k_scatter_cast<<<grid_for(nk, 256), 256, 0, s>>>(B.e0.p, B.perm0.p, B.k, e, B.n);
    AIRG_LAUNCH_CHECK();
}

}  // namespace airg

// Solve phase: the V-cycle with up F-point smoothing only (Results), the
// undamped Richardson outer iteration, and flexible GMRES in FP64 around an
// FP32 or FP64 V-cycle.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

#include "csr.hpp"
#include "group.hpp"
#include "hierarchy.hpp"

namespace airg {

namespace {
inline void spmvT(const Csr &A, const double *x, double *y, const double *z, int mode, hipStream_t s) {
    spmv(view(A), x, y, z, mode, s);
}
inline void spmvT(const Csr &A, const float *x, float *y, const float *z, int mode, hipStream_t s) {
    spmv32(view(A), x, y, z, mode, s);
}
template <class T> struct Bufs;
template <class T> struct PVal;
template <> struct PVal<double> {
    static const double *get(const Level &L) { return L.pval64.p; }
};
template <> struct PVal<float> {
    static const float *get(const Level &L) { return L.pval32.p; }
};

// The prolongation e = [W; I] e_c (one entry or none per row) fused with the
// first smoothing residual t_F = g_F - [A_ff A_fc] e: each product forms the
// e entry it needs from e_c as the prolongation would store it, so the
// result equals the two separate lane-group products.
template <int G, class T>
__global__ void __launch_bounds__(256) k_prolong_resid(int32_t n, int32_t nF, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                       const int32_t *__restrict__ pcol, const T *__restrict__ pval,
                                                       const T *__restrict__ ec, const T *__restrict__ g,
                                                       T *__restrict__ e, T *__restrict__ t) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t row = (int32_t)(tid / G);
    const int lane = group_lane<G>();
    if (row >= n) return;
    if (lane == 0) {
        const int32_t pc = pcol[row];
        e[row] = pc >= 0 ? pval[row] * ec[pc] : (T)0;
    }
    if (row >= nF) return;
    T acc = 0;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) {
        const int32_t j = ci[k];
        const int32_t pc = pcol[j];
        const T ej = pc >= 0 ? pval[j] * ec[pc] : (T)0;
        acc += v[k] * ej;
    }
    acc = group_sum<G>(acc);
    if (lane == 0) t[row] = g[row] - acc;
}

template <class T>
void prolong_resid(Level &Lv, const T *ec, const T *g, T *e, T *t, hipStream_t s) {
    const T *v;
    if constexpr (std::is_same_v<T, float>) v = Lv.AF.vf.p;
    else v = Lv.AF.v.p;
    dispatch_group(lanes_for(Lv.AF.nnz, Lv.AF.nr), [&]<int G>() {
        k_prolong_resid<G, T><<<grid_for((int64_t)Lv.n * G, 256), 256, 0, s>>>(
            Lv.n, Lv.nF, Lv.AF.rp.p, Lv.AF.ci.p, v, Lv.pcol.p, PVal<T>::get(Lv), ec, g, e, t);
    });
    AIRG_LAUNCH_CHECK();
}

template <> struct Bufs<double> {
    static double *g(Level &L) { return L.g64.p; }
    static double *e(Level &L) { return L.e64.p; }
    static double *t(Level &L) { return L.t64.p; }
    static double *p(Level &L) { return L.p64.p; }
    static double *q(Level &L) { return L.q64.p; }
    static double *u(Level &L) { return L.u64.p; }
};
template <> struct Bufs<float> {
    static float *g(Level &L) { return L.g32.p; }
    static float *e(Level &L) { return L.e32.p; }
    static float *t(Level &L) { return L.t32.p; }
    static float *p(Level &L) { return L.p32.p; }
    static float *q(Level &L) { return L.q32.p; }
    static float *u(Level &L) { return L.u32.p; }
};

// y = a x (SET) or y += a x (ADD), contraction off as in the power sums
template <class T>
__global__ void k_scale_acc(int64_t n, T a, const T *__restrict__ x, T *__restrict__ y, int add) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v = a * x[i];
    y[i] = add ? y[i] + v : v;
}

// Coarse polynomial on the coarsest level: the assembled fixed-sparsity
// matrix, or q(A) x = sum_k alpha_k A^k x by products with A in ascending
// powers (matrix-free; the truncation subsection's alternative).  mode as in
// spmv: SET writes y, ADD adds to it.
template <class T>
void coarse_apply(Hier &H, Level &Lv, const T *x, T *y, int mode) {
    hipStream_t s = H.s;
    if (!H.opt.coarse_matrix_free) {
        spmvT(Lv.Ainv, x, y, (const T *)nullptr, mode, s);
        return;
    }
    const int64_t n = Lv.n;
    T *pk = Bufs<T>::p(Lv), *pn = Bufs<T>::q(Lv), *acc = mode == SPMV_SET ? y : Bufs<T>::u(Lv);
    const unsigned grid = grid_for(n, 256);
    k_scale_acc<T><<<grid, 256, 0, s>>>(n, (T)1, x, pk, 0);   // pk = x (kernel: the cycle may be captured)
    k_scale_acc<T><<<grid, 256, 0, s>>>(n, (T)Lv.poly.alpha[0], pk, acc, 0);
    for (int k = 1; k < Lv.poly.m; ++k) {
        spmvT(Lv.A, pk, pn, (const T *)nullptr, SPMV_SET, s);
        std::swap(pk, pn);
        k_scale_acc<T><<<grid, 256, 0, s>>>(n, (T)Lv.poly.alpha[k], pk, acc, 1);
    }
    if (mode != SPMV_SET) k_scale_acc<T><<<grid, 256, 0, s>>>(n, (T)1, acc, y, 1);
    AIRG_LAUNCH_CHECK();
}
}  // namespace

// e = V(g) on level l, vectors in level order (F points first):
//   g_c = [Z I] g;  e_c = V(g_c);  e = [W; I] e_c;
//   up_smooths times: e_F += Ainv (g_F - [A_ff A_fc] e).
// Coarsest level: e = Ainv g, then (coarse_iters - 1) times e += Ainv (g - A e),
// with Ainv the assembled coarse polynomial or q(A) applied matrix-free.
template <class T>
void Hier::vcycle(int l, const T *g, T *e) {
    Level &Lv = L(l);
    T *t = Bufs<T>::t(Lv);
    auto mark = [&](int k) {
        if (prof) AIRG_HIP(hipEventRecord(prof[4 * l + k], s));
    };
    if (Lv.coarsest) {
        mark(0);
        coarse_apply<T>(*this, Lv, g, e, SPMV_SET);
        for (int it = 1; it < opt.coarse_iters; ++it) {
            spmvT(Lv.A, e, t, g, SPMV_ZMINUS, s);
            coarse_apply<T>(*this, Lv, t, e, SPMV_ADD);
        }
        mark(1);
        mark(2);
        mark(3);
        return;
    }
    Level &N = L(l + 1);
    T *gc = Bufs<T>::g(N);
    T *ec = Bufs<T>::e(N);
    mark(0);
    spmvT(Lv.Rp, g, gc, (const T *)nullptr, SPMV_SET, s);
    mark(1);
    vcycle<T>(l + 1, gc, ec);
    mark(2);
    int k0 = 0;
    if (Lv.pcol.p && opt.up_smooths > 0) {
        prolong_resid<T>(Lv, ec, g, e, t, s);
        spmvT(Lv.Ainv, t, e, (const T *)nullptr, SPMV_ADD, s);
        k0 = 1;
    } else {
        spmvT(Lv.Pp, ec, e, (const T *)nullptr, SPMV_SET, s);
    }
    for (int k = k0; k < opt.up_smooths; ++k) {
        spmvT(Lv.AF, e, t, g, SPMV_ZMINUS, s);
        spmvT(Lv.Ainv, t, e, (const T *)nullptr, SPMV_ADD, s);
    }
    mark(3);
}

template void Hier::vcycle<double>(int, const double *, double *);
template void Hier::vcycle<float>(int, const float *, float *);

Hier::~Hier() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
}

void Hier::drop_graphs() {
    for (int k = 0; k < 2; ++k) {
        if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
        if (graph[k]) (void)hipGraphDestroy(graph[k]);
        gexec[k] = nullptr;
        graph[k] = nullptr;
        eager[k] = 0;
    }
}

namespace {
// Runs f eagerly for the slot's first kEagerCycles calls; then captures its
// launches on the private stream once (the legacy default stream cannot be
// captured) and replays them on the hierarchy's stream.
template <class F>
void run_captured(Hier &H, int k, F &&f) {
    if (!H.gexec[k]) {
        if (H.eager[k] < Hier::kEagerCycles) {
            ++H.eager[k];
            ++H.cycles_eager;
            f();
            return;
        }
        if (!H.cap) AIRG_HIP(hipStreamCreateWithFlags(&H.cap, hipStreamNonBlocking));
        hipStream_t user = H.s;
        AIRG_HIP(hipStreamBeginCapture(H.cap, hipStreamCaptureModeRelaxed));
        H.s = H.cap;
        try {
            f();
        } catch (...) {
            H.s = user;
            hipGraph_t dummy = nullptr;
            (void)hipStreamEndCapture(H.cap, &dummy);
            if (dummy) (void)hipGraphDestroy(dummy);
            throw;
        }
        H.s = user;
        AIRG_HIP(hipStreamEndCapture(H.cap, &H.graph[k]));
        AIRG_HIP(hipGraphInstantiate(&H.gexec[k], H.graph[k], nullptr, nullptr, 0));
    }
    ++H.cycles_graph;
    AIRG_HIP(hipGraphLaunch(H.gexec[k], H.s));
}
}  // namespace

// The outer iterations keep their vectors in natural order and apply the
// top operator as stored; the cycle runs in level order (F points first)
// between fixed buffers (level 0's g and e for FP64, r32/e32 for FP32), which
// the casts in and out permute.  With use_graph one captured graph per
// precision serves every call after the first Hier::kEagerCycles.
void Hier::precondition(const double *rv, double *ev, int precision) {
    TraceRange trace(precision == 32 ? "V-cycle fp32" : "V-cycle fp64");
    Level &T = L(0);
    const int64_t n0 = T.n;
    const int32_t *ip = T.coarsest ? nullptr : T.iperm.p;   // level position -> natural index
    const bool graphed = opt.use_graph != 0;
    if (precision == 32) {
        if (ip) gather_d2f(rv, ip, r32.p, n0, s);
        else cast_d2f(rv, r32.p, n0, s);
        if (graphed) {
            run_captured(*this, 1, [&] { vcycle<float>(0, r32.p, e32.p); });
        } else {
            ++cycles_eager;
            vcycle<float>(0, r32.p, e32.p);
        }
        if (ip) scatter_f2d(e32.p, ip, ev, n0, s);
        else cast_f2d(e32.p, ev, n0, s);
        return;
    }
    if (ip) gather(rv, ip, T.g64.p, n0, s);
    else d2d(T.g64.p, rv, (size_t)n0, s);
    if (graphed) {
        run_captured(*this, 0, [&] { vcycle<double>(0, T.g64.p, T.e64.p); });
    } else {
        ++cycles_eager;
        vcycle<double>(0, T.g64.p, T.e64.p);
    }
    if (ip) scatter(T.e64.p, ip, ev, n0, s);
    else d2d(ev, T.e64.p, (size_t)n0, s);
}

namespace {
CsrView top_view(Hier &H) { return view(H.L(0).A); }
void copy_vec(Hier &H, const double *src, double *dst) { d2d(dst, src, (size_t)H.L(0).n, H.s); }
}  // namespace

void apply_vcycle(Hier &H, const double *g, double *e, int precision) { H.precondition(g, e, precision); }

void profile_vcycle(Hier &H, int precision, int reps, double *out) {
    const int nl = H.nlev();
    for (int l = 0; l < nl; ++l) out[l] = 0.0;
    Level &T = H.L(0);
    if (precision == 32) fill_zero(T.g32.p, (size_t)T.n * 4, H.s);
    else fill_zero(T.g64.p, (size_t)T.n * 8, H.s);
    std::vector<hipEvent_t> ev((size_t)4 * nl);
    for (auto &e : ev) e = pooled_event();
    try {
        for (int r = 0; r < reps; ++r) {
            H.prof = ev.data();
            if (precision == 32) H.vcycle<float>(0, T.g32.p, T.e32.p);
            else H.vcycle<double>(0, T.g64.p, T.e64.p);
            H.prof = nullptr;
            AIRG_HIP(hipStreamSynchronize(H.s));
            for (int l = 0; l < nl; ++l) {
                float a = 0.f, b = 0.f;
                AIRG_HIP(hipEventElapsedTime(&a, ev[4 * l], ev[4 * l + 1]));
                AIRG_HIP(hipEventElapsedTime(&b, ev[4 * l + 2], ev[4 * l + 3]));
                out[l] += (a + b) * 1e-3 / reps;
            }
        }
    } catch (...) {
        H.prof = nullptr;
        for (auto &e : ev) release_event(e);
        throw;
    }
    for (auto &e : ev) release_event(e);
}

// Undamped Richardson from a zero guess: x += V(b - A x) until
// ||b - A x||_2 <= rtol ||b||_2 (true FP64 residual every iteration).
SolveResult solve_richardson(Hier &H, const double *b, double *x, double rtol, int maxit) {
    TraceRange trace("airg solve: Richardson");
    hipStream_t s = H.s;
    int64_t n = H.L(0).n;
    SolveResult res;
    CsrView A = top_view(H);
    copy_vec(H, b, H.bp.p);
    fill_zero(H.x.p, (size_t)n * 8, s);
    double nb = nrm2(H.bp.p, n, s);
    if (nb == 0.0) {
        copy_vec(H, H.x.p, x);
        res.converged = true;
        return res;
    }
    d2d(H.r.p, H.bp.p, (size_t)n, s);
    double rr = nb;
    int prec = H.opt.precond_precision == 32 ? 32 : 64;
    while (rr > rtol * nb && res.iterations < maxit) {
        H.precondition(H.r.p, H.e.p, prec);
        axpy(1.0, H.e.p, H.x.p, n, s);
        spmv_top(A, H.x.p, H.r.p, H.bp.p, SPMV_ZMINUS, s);
        rr = nrm2(H.r.p, n, s);
        res.iterations++;
        AIRG_REQUIRE(std::isfinite(rr), ST_STALL, "residual became non-finite in the Richardson iteration");
    }
    copy_vec(H, H.x.p, x);
    res.rel_residual = rr / nb;
    res.converged = rr <= rtol * nb;
    return res;
}

// Flexible GMRES(restart), right preconditioned by one V-cycle per Arnoldi
// step (FP32 or FP64), classical Gram-Schmidt applied twice in FP64, Givens
// rotations on the host, true FP64 residual at every restart.  The
// Gram-Schmidt coefficients and the new vector's norm stay on the device
// until one readback per Arnoldi step brings all of them to the host.
constexpr int kMaxFusedBasis = 32;   // basis vectors gemv_sub_dots takes

SolveResult solve_fgmres(Hier &H, const double *b, double *x, double rtol, int maxit) {
    TraceRange trace("airg solve: FGMRES");
    hipStream_t s = H.s;
    int64_t n = H.L(0).n;
    int m = H.opt.fgmres_restart > 0 ? H.opt.fgmres_restart : 30;
    SolveResult res;
    CsrView A = top_view(H);
    DBuf<double> V((size_t)n * (m + 1), s), Zb((size_t)n * m, s), hd((size_t)m + 1, s);
    DBuf<double> hdev((size_t)2 * (m + 1) + 1, s);   // [h1 (m+1) | h2 (m+1) | ||w||^2]
    copy_vec(H, b, H.bp.p);
    fill_zero(H.x.p, (size_t)n * 8, s);
    double nb = nrm2(H.bp.p, n, s);
    if (nb == 0.0) {
        copy_vec(H, H.x.p, x);
        res.converged = true;
        return res;
    }
    d2d(H.r.p, H.bp.p, (size_t)n, s);
    double beta = nb;
    int prec = H.opt.precond_precision == 32 ? 32 : 64;
    std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h1(m + 1), h2(m + 1);
    std::vector<double> rb((size_t)2 * (m + 1) + 1);
    while (beta > rtol * nb && res.iterations < maxit) {
        scal_copy(1.0 / beta, H.r.p, V.p, n, s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        for (; j < m && res.iterations < maxit;) {
            double *vj = V.p + (int64_t)j * n, *zj = Zb.p + (int64_t)j * n, *w = V.p + (int64_t)(j + 1) * n;
            H.precondition(vj, zj, prec);
            res.iterations++;
            spmv_top(A, zj, w, nullptr, SPMV_SET, s);
            double *d1 = hdev.p, *d2 = hdev.p + (m + 1), *dn = hdev.p + 2 * (m + 1);
            multi_dot_dev(V.p, n, j + 1, w, n, d1, s);            // h1 = V^T w
            if (j + 1 <= kMaxFusedBasis) {
                gemv_sub_dots(V.p, n, j + 1, d1, w, n, d2, s);    // w -= V h1; h2 = V^T w
                gemv_sub_norm(V.p, n, j + 1, d2, w, n, dn, s);    // w -= V h2; ||w||^2
            } else {
                gemv_sub(V.p, n, j + 1, d1, w, n, s);
                multi_dot_dev(V.p, n, j + 1, w, n, d2, s);
                gemv_sub(V.p, n, j + 1, d2, w, n, s);
                multi_dot_dev(w, n, 1, w, n, dn, s);
            }
            normalize_dev(w, dn, n, s);
            read_ints({reinterpret_cast<const int32_t *>(d1), reinterpret_cast<const int32_t *>(d2),
                       reinterpret_cast<const int32_t *>(dn)},
                      {2 * (j + 1), 2 * (j + 1), 2},
                      reinterpret_cast<int32_t *>(rb.data()), s);
            std::copy(rb.begin(), rb.begin() + j + 1, h1.begin());
            std::copy(rb.begin() + j + 1, rb.begin() + 2 * (j + 1), h2.begin());
            const double nn = rb[2 * (j + 1)];
            for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = h1[i] + h2[i];
            double hn = std::sqrt(nn);
            AIRG_REQUIRE(std::isfinite(hn), ST_STALL, "Arnoldi vector became non-finite");
            Hm[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = Hm[(size_t)i * m + j], c = Hm[(size_t)(i + 1) * m + j];
                Hm[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                Hm[(size_t)(i + 1) * m + j] = cs[i] * c - sn[i] * a;
            }
            double a = Hm[(size_t)j * m + j], c = Hm[(size_t)(j + 1) * m + j];
            double rr = std::hypot(a, c);
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? c / rr : 0.0;
            Hm[(size_t)j * m + j] = rr;
            Hm[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (std::fabs(g[j]) <= rtol * nb || hn == 0.0) break;
        }
        for (int i = j - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < j; ++q) t -= Hm[(size_t)i * m + q] * y[q];
            y[i] = Hm[(size_t)i * m + i] != 0.0 ? t / Hm[(size_t)i * m + i] : 0.0;
        }
        h2d(hd.p, y.data(), (size_t)j, s);
        gemv_add(Zb.p, n, j, hd.p, H.x.p, n, s);
        spmv_top(A, H.x.p, H.r.p, H.bp.p, SPMV_ZMINUS, s);
        beta = nrm2(H.r.p, n, s);
        AIRG_REQUIRE(std::isfinite(beta), ST_STALL, "residual became non-finite in FGMRES");
    }
    copy_vec(H, H.x.p, x);
    res.rel_residual = beta / nb;
    res.converged = beta <= rtol * nb;
    return res;
}

}  // namespace airg

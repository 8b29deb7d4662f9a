// One-point prolongator and full-space restriction for the Galerkin product.
#include <cmath>

#include "csr.hpp"
#include "group.hpp"
#include "transfer.hpp"

namespace airg {

// Per F row: strongest off-diagonal (largest |a_ij|, smallest j on ties).
template <int G>
__global__ void __launch_bounds__(256) k_onepoint(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                                                  int weight_mode, int32_t *__restrict__ wcol,
                                                  double *__restrict__ wval) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n || cf[row] != CF_F) return;
    double best = 0.0, bval = 0.0, diag = 0.0;
    int32_t bj = 0x7fffffff;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) {
        int32_t j = ci[k];
        double a = v[k];
        if (j == row) { diag = a; continue; }
        if (fabs(a) > best) { best = fabs(a); bj = j; bval = a; }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, G);
        int32_t oj = __shfl_xor(bj, o, G);
        double ov = __shfl_xor(bval, o, G);
        if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; bval = ov; }
    }
    diag = group_sum<G>(diag);
    if (lane == 0) {
        int32_t f = rank[row];
        if (best > 0.0 && cf[bj] == CF_C) {
            wcol[f] = rank[bj];
            wval[f] = weight_mode == 1 ? -bval / diag : 1.0;
        } else {
            wcol[f] = -1;
            wval[f] = 0.0;
        }
    }
}

__global__ void k_p_count(int32_t n, const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                          const int32_t *__restrict__ wcol, int32_t *__restrict__ cntP, int32_t *__restrict__ cntW) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == CF_F) {
        int32_t has = wcol[rank[i]] >= 0;
        cntP[i] = has;
        cntW[rank[i]] = has;
    } else {
        cntP[i] = cf[i] == CF_C;   // terminal rows of a batch have no prolongation
    }
}

__global__ void k_p_fill(int32_t n, const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                         const int32_t *__restrict__ wcol, const double *__restrict__ wval,
                         const int32_t *__restrict__ prp, int32_t *__restrict__ pci, double *__restrict__ pv,
                         const int32_t *__restrict__ wrp, int32_t *__restrict__ wci, double *__restrict__ wv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t r = rank[i];
    if (cf[i] == CF_F) {
        int32_t c = wcol[r];
        if (c >= 0) {
            pci[prp[i]] = c;
            pv[prp[i]] = wval[r];
            wci[wrp[r]] = c;
            wv[wrp[r]] = wval[r];
        }
    } else if (cf[i] == CF_C) {
        pci[prp[i]] = r;
        pv[prp[i]] = 1.0;
    }
}

void onepoint_prolongator(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                          int weight_mode, Csr *P, Csr *W, hipStream_t s) {
    int32_t n = A.nr;
    DBuf<int32_t> wcol((size_t)nF + 1, s), cntP((size_t)n + 1, s), cntW((size_t)nF + 1, s);
    DBuf<double> wval((size_t)nF + 1, s);
    int g = lanes_for(A.nnz, n);
    dispatch_group(g, [&]<int G>() {
        k_onepoint<G><<<grid_for((int64_t)n * G, 256), 256, 0, s>>>(n, A.rp, A.ci, A.v, cf, rank, weight_mode,
                                                                    wcol.p, wval.p);
    });
    AIRG_LAUNCH_CHECK();
    k_p_count<<<grid_for(n, 256), 256, 0, s>>>(n, cf, rank, wcol.p, cntP.p, cntW.p);
    AIRG_LAUNCH_CHECK();
    P->nr = n;
    P->nc = nC;
    P->rp.alloc((size_t)n + 1, s);
    W->nr = nF;
    W->nc = nC;
    W->rp.alloc((size_t)nF + 1, s);
    exclusive_scans({cntP.p, cntW.p}, {P->rp.p, W->rp.p}, {n, nF}, s);
    resolve_sizes({P, W}, s);
    k_p_fill<<<grid_for(n, 256), 256, 0, s>>>(n, cf, rank, wcol.p, wval.p, P->rp.p, P->ci.p, P->v.p, W->rp.p,
                                              W->ci.p, W->v.p);
    AIRG_LAUNCH_CHECK();
}

// [W; I] in natural row order from an existing W (numeric re-setup keeps
// W's columns): F rows copy W's row, C rows hold the identity entry,
// terminal rows nothing.
__global__ void k_pw_count(int32_t n, const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                           const int32_t *__restrict__ wrp, int32_t *__restrict__ cnt) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int8_t c = cf[i];
    cnt[i] = c == CF_F ? wrp[rank[i] + 1] - wrp[rank[i]] : c == CF_C ? 1 : 0;
}
__global__ void k_pw_fill(int32_t n, const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                          const int32_t *__restrict__ wrp, const int32_t *__restrict__ wci,
                          const double *__restrict__ wv, const int32_t *__restrict__ prp, int32_t *__restrict__ pci,
                          double *__restrict__ pv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int8_t c = cf[i];
    int32_t w = prp[i], r = rank[i];
    if (c == CF_F) {
        for (int32_t k = wrp[r]; k < wrp[r + 1]; ++k, ++w) {
            pci[w] = wci[k];
            pv[w] = wv[k];
        }
    } else if (c == CF_C) {
        pci[w] = r;
        pv[w] = 1.0;
    }
}

Csr prolongator_from_w(const Csr &W, const int8_t *cf, const int32_t *rank, int32_t n, int32_t nC, hipStream_t s) {
    Csr P;
    P.nr = n;
    P.nc = nC;
    P.rp.alloc((size_t)n + 1, s);
    DBuf<int32_t> cnt((size_t)n + 1, s);
    k_pw_count<<<grid_for(n, 256), 256, 0, s>>>(n, cf, rank, W.rp.p, cnt.p);
    AIRG_LAUNCH_CHECK();
    exclusive_scan(cnt.p, P.rp.p, n, s, false);
    resolve_sizes({&P}, s);
    k_pw_fill<<<grid_for(n, 256), 256, 0, s>>>(n, cf, rank, W.rp.p, W.ci.p, W.v.p, P.rp.p, P.ci.p, P.v.p);
    AIRG_LAUNCH_CHECK();
    return P;
}

// Weight mode 1 at W's existing columns: w = -a_ij / a_ii with j the C point
// of the column.
__global__ void k_w_values(int32_t nF, const int32_t *__restrict__ fidx, const int32_t *__restrict__ cidx,
                           const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const int32_t *__restrict__ wrp,
                           const int32_t *__restrict__ wci, double *__restrict__ wv) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nF) return;
    int32_t i = fidx[r];
    for (int32_t k = wrp[r]; k < wrp[r + 1]; ++k) {
        int32_t j = cidx[wci[k]];
        double aij = 0.0, aii = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            if (ci[q] == j) aij = v[q];
            if (ci[q] == i) aii = v[q];
        }
        wv[k] = -aij / aii;
    }
}

void onepoint_values(const CsrView &A, const int32_t *fidx, const int32_t *cidx, Csr &W, hipStream_t s) {
    if (W.nr == 0) return;
    k_w_values<<<grid_for(W.nr, 256), 256, 0, s>>>(W.nr, fidx, cidx, A.rp, A.ci, A.v, W.rp.p, W.ci.p, W.v.p);
    AIRG_LAUNCH_CHECK();
}

__global__ void k_r_rowptr(int32_t nC, const int32_t *__restrict__ zrp, int32_t *__restrict__ rrp) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= nC) rrp[r] = zrp[r] + r;
}

// R row r = Z row r with columns mapped to level numbering by fidx (ascending,
// since fidx is) and the entry (cidx[r], 1) in its sorted place.  A G-lane
// group per row: an entry goes to its own offset, one further when its
// column passes cidx[r]; the identity goes after the entries below it.
template <int G>
__global__ void __launch_bounds__(256) k_r_fill(int32_t nC, const int32_t *__restrict__ zrp,
                                                const int32_t *__restrict__ zci, const double *__restrict__ zv,
                                                const int32_t *__restrict__ fidx, const int32_t *__restrict__ cidx,
                                                const int32_t *__restrict__ rrp, int32_t *__restrict__ rci,
                                                double *__restrict__ rv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t r = (int32_t)(t / G);
    const int lane = group_lane<G>();
    if (r >= nC) return;
    const int32_t me = cidx[r];
    const int32_t b = zrp[r], e = zrp[r + 1];
    const int32_t w0 = rrp[r];
    int32_t below = 0;
    for (int32_t base = b; base < e; base += G) {
        const int32_t k = base + lane;
        const bool in = k < e;
        const int32_t g = in ? fidx[zci[k]] : 0;
        below += __popcll(group_ballot<G>(in && g < me));
        if (in) {
            const int32_t pos = w0 + (k - b) + (g > me ? 1 : 0);
            rci[pos] = g;
            rv[pos] = zv[k];
        }
    }
    if (lane == 0) {
        rci[w0 + below] = me;
        rv[w0 + below] = 1.0;
    }
}

Csr restriction_full(const CsrView &Z, const int32_t *fidx, const int32_t *cidx, int32_t n, hipStream_t s) {
    Csr R;
    R.nr = Z.nr;
    R.nc = n;
    R.nnz = Z.nnz + Z.nr;
    R.rp.alloc((size_t)Z.nr + 1, s);
    R.ci.alloc((size_t)R.nnz, s);
    R.v.alloc((size_t)R.nnz, s);
    k_r_rowptr<<<grid_for((int64_t)Z.nr + 1, 256), 256, 0, s>>>(Z.nr, Z.rp, R.rp.p);
    AIRG_LAUNCH_CHECK();
    if (Z.nr > 0) {
        dispatch_group(lanes_for(Z.nnz, Z.nr), [&]<int G>() {
            k_r_fill<G><<<grid_for((int64_t)Z.nr * G, 256), 256, 0, s>>>(Z.nr, Z.rp, Z.ci, Z.v, fidx, cidx, R.rp.p,
                                                                         R.ci.p, R.v.p);
        });
        AIRG_LAUNCH_CHECK();
    }
    return R;
}

}  // namespace airg

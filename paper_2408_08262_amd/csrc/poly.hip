// GMRES-polynomial kernels for gfx950: Box-Muller rhs, column norms, a
// tall-skinny Householder QR tree in LDS, and the row-local fixed-sparsity
// power sum (one lane group per row, M_i staged in LDS).
#include <cmath>

#include "csr.hpp"
#include "group.hpp"
#include "poly.hpp"

namespace airg {

// ------------------------------------------------------------ random rhs ---
__global__ void k_gauss(int64_t n, uint64_t seed, int32_t level, double *__restrict__ b) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double two53 = 1.0 / 9007199254740992.0;
    uint64_t r1 = splitmix64(rng_counter(seed, 1, (uint32_t)level, (uint64_t)k));
    uint64_t r2 = splitmix64(rng_counter(seed, 2, (uint32_t)level, (uint64_t)k));
    double u1 = ((double)(r1 >> 11) + 1.0) * two53;
    double u2 = (double)(r2 >> 11) * two53;
    b[k] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

void gauss_rhs(int64_t n, uint64_t seed, int32_t level, double *b, hipStream_t s) {
    if (n <= 0) return;
    k_gauss<<<grid_for(n, 256), 256, 0, s>>>(n, seed, level, b);
    AIRG_LAUNCH_CHECK();
}

// ------------------------------------------------------------ reductions ---
constexpr int kQrThreads = 256;
constexpr int kQrRows = 384;          // rows per leaf: cols*384*8 <= 48 KiB of LDS

template <int N>
__device__ inline void block_sum_vec(double (&v)[N], int cnt, double *sh /* [4][N] */) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (c < cnt) {
            double x = group_sum<64>(v[c]);
            if (lane == 0) sh[wid * N + c] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (c < cnt) {
            double x = 0.0;
            for (int w = 0; w < kQrThreads / 64; ++w) x += sh[w * N + c];
            v[c] = x;
        }
    }
    __syncthreads();
}

// partial[c * nb + b] = sum over block b's rows of K[:, c]^2.
__global__ void __launch_bounds__(kQrThreads) k_colsq(const double *__restrict__ K, int64_t n, int cols,
                                                      double *__restrict__ partial) {
    __shared__ double sh[4 * kMaxPolyCols];
    double v[kMaxPolyCols];
#pragma unroll
    for (int c = 0; c < kMaxPolyCols; ++c) v[c] = 0.0;
    int nb = gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * kQrThreads + threadIdx.x; i < n; i += (int64_t)nb * kQrThreads) {
#pragma unroll
        for (int c = 0; c < kMaxPolyCols; ++c)
            if (c < cols) {
                double x = K[(int64_t)c * n + i];
                v[c] += x * x;
            }
    }
    block_sum_vec<kMaxPolyCols>(v, cols, sh);
    if (threadIdx.x < cols) partial[(int64_t)threadIdx.x * nb + blockIdx.x] = v[threadIdx.x];
}

__global__ void __launch_bounds__(kQrThreads) k_colsq_finish(const double *__restrict__ partial, int nb, int cols,
                                                             double *__restrict__ norm, double *__restrict__ inv) {
    __shared__ double sh[4 * kMaxPolyCols];
    double v[kMaxPolyCols];
#pragma unroll
    for (int c = 0; c < kMaxPolyCols; ++c) {
        v[c] = 0.0;
        if (c < cols)
            for (int b = threadIdx.x; b < nb; b += kQrThreads) v[c] += partial[(int64_t)c * nb + b];
    }
    block_sum_vec<kMaxPolyCols>(v, cols, sh);
    if (threadIdx.x < cols) {
        double nr = sqrt(v[threadIdx.x]);
        norm[threadIdx.x] = nr;
        inv[threadIdx.x] = nr > 0.0 ? 1.0 / nr : 1.0;
    }
}

// -------------------------------------------------------------- TSQR leaf ---
// Householder QR of a kQrRows x cols panel staged in LDS (column-major); the
// R factor of block b is written as rows b*cols .. b*cols+cols-1 of the next
// (column-major) stacked matrix.
__global__ void __launch_bounds__(kQrThreads) k_tsqr_leaf(const double *__restrict__ K, int64_t n, int64_t ldk,
                                                          int cols, const double *__restrict__ scale,
                                                          double *__restrict__ Rs, int64_t ldr) {
    extern __shared__ double W[];               // cols * kQrRows
    __shared__ double sh[4 * kMaxPolyCols];
    int64_t r0 = (int64_t)blockIdx.x * kQrRows;
    for (int c = 0; c < cols; ++c) {
        double sc = scale ? scale[c] : 1.0;
        for (int r = threadIdx.x; r < kQrRows; r += kQrThreads) {
            int64_t row = r0 + r;
            W[c * kQrRows + r] = row < n ? K[(int64_t)c * ldk + row] * sc : 0.0;
        }
    }
    __syncthreads();
    int steps = cols < kQrRows ? cols : kQrRows;
    for (int col = 0; col < steps; ++col) {
        double *x = W + col * kQrRows;
        double part[1] = {0.0};
        for (int r = col + threadIdx.x; r < kQrRows; r += kQrThreads) part[0] += x[r] * x[r];
        block_sum_vec<1>(part, 1, sh);
        double nx2 = part[0];
        double x0 = x[col];
        double nx = sqrt(nx2);
        double alpha = x0 >= 0.0 ? -nx : nx;
        double vv = 2.0 * nx * (nx + fabs(x0));
        if (vv > 0.0) {
            double d[kMaxPolyCols];
#pragma unroll
            for (int c = 0; c < kMaxPolyCols; ++c) d[c] = 0.0;
            for (int r = col + threadIdx.x; r < kQrRows; r += kQrThreads) {
                double vr = r == col ? x0 - alpha : x[r];
#pragma unroll
                for (int c = 0; c < kMaxPolyCols; ++c)
                    if (c > col && c < cols) d[c] += vr * W[c * kQrRows + r];
            }
            block_sum_vec<kMaxPolyCols>(d, cols, sh);
            for (int r = col + threadIdx.x; r < kQrRows; r += kQrThreads) {
                double vr = r == col ? x0 - alpha : x[r];
#pragma unroll
                for (int c = 0; c < kMaxPolyCols; ++c)
                    if (c > col && c < cols) W[c * kQrRows + r] -= (2.0 * d[c] / vv) * vr;
            }
            __syncthreads();
            if (threadIdx.x == 0) x[col] = alpha;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < cols * cols; idx += kQrThreads) {
        int r = idx / cols, c = idx % cols;
        double val = (r <= c && r < steps) ? W[c * kQrRows + r] : 0.0;
        Rs[(int64_t)c * ldr + (int64_t)blockIdx.x * cols + r] = val;
    }
}

void tsqr_r(const double *K, int64_t n, int cols, double *h_R, double *h_colnorm, hipStream_t s) {
    AIRG_REQUIRE(cols >= 1 && cols <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order too large");
    int nbn = (int)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 1024));
    DBuf<double> part((size_t)nbn * cols, s), norm((size_t)cols, s), inv((size_t)cols, s);
    k_colsq<<<nbn, kQrThreads, 0, s>>>(K, n, cols, part.p);
    AIRG_LAUNCH_CHECK();
    k_colsq_finish<<<1, kQrThreads, 0, s>>>(part.p, nbn, cols, norm.p, inv.p);
    AIRG_LAUNCH_CHECK();
    size_t lds = (size_t)cols * kQrRows * sizeof(double);
    const double *src = K;
    int64_t rows = n, ld = n;
    const double *scale = inv.p;
    DBuf<double> bufs[2];
    int which = 0;
    for (;;) {
        int64_t nb = (rows + kQrRows - 1) / kQrRows;
        if (nb < 1) nb = 1;
        int64_t out_rows = nb * cols;
        bufs[which].alloc((size_t)out_rows * cols, s);
        k_tsqr_leaf<<<(unsigned)nb, kQrThreads, lds, s>>>(src, rows, ld, cols, scale, bufs[which].p, out_rows);
        AIRG_LAUNCH_CHECK();
        src = bufs[which].p;
        rows = out_rows;
        ld = out_rows;
        scale = nullptr;
        which ^= 1;
        if (nb == 1) break;
    }
    std::vector<double> R((size_t)cols * cols);
    d2h(R.data(), src, (size_t)cols * cols, s);      // column-major cols x cols
    for (int r = 0; r < cols; ++r)
        for (int c = 0; c < cols; ++c) h_R[r * cols + c] = R[(size_t)c * cols + r];
    d2h(h_colnorm, norm.p, (size_t)cols, s);
}

// -------------------------------------------------------- least squares ---
// Upper Hessenberg least squares by Givens rotations on the scaled factor.
int poly_coeffs_from_r(const double *R, const double *colnorm, int m, double *alpha) {
    const int nc = m + 1;
    for (int k = 0; k < m; ++k) alpha[k] = 0.0;
    // Krylov breakdown: |R_jj| tiny relative to the leading columns
    int keep = m;
    double fro2 = 0.0;
    for (int j = 0; j <= m; ++j) {
        for (int r = 0; r <= j; ++r) fro2 += R[r * nc + j] * R[r * nc + j];
        if (j >= 1 && (std::fabs(R[j * nc + j]) <= 1e-14 * std::sqrt(fro2) || colnorm[j] == 0.0)) {
            keep = colnorm[j] == 0.0 ? j - 1 : j;
            break;
        }
    }
    if (keep <= 0 || colnorm[0] == 0.0) return 0;
    // H = R[0..keep, 1..keep], rhs = R00 e1
    double H[kMaxPolyCols][kMaxPolyCols];
    double g[kMaxPolyCols + 1];
    for (int r = 0; r <= keep; ++r) {
        g[r] = r == 0 ? R[0] : 0.0;
        for (int c = 0; c < keep; ++c) H[r][c] = R[r * nc + c + 1];
    }
    for (int c = 0; c < keep; ++c) {
        double a = H[c][c], b = H[c + 1][c];
        double h = std::hypot(a, b);
        if (h == 0.0) continue;
        double cs = a / h, sn = b / h;
        for (int q = c; q < keep; ++q) {
            double u = H[c][q], w = H[c + 1][q];
            H[c][q] = cs * u + sn * w;
            H[c + 1][q] = cs * w - sn * u;
        }
        double u = g[c], w = g[c + 1];
        g[c] = cs * u + sn * w;
        g[c + 1] = cs * w - sn * u;
    }
    double y[kMaxPolyCols];
    for (int r = keep - 1; r >= 0; --r) {
        double acc = g[r];
        for (int q = r + 1; q < keep; ++q) acc -= H[r][q] * y[q];
        y[r] = H[r][r] != 0.0 ? acc / H[r][r] : 0.0;
    }
    for (int k = 0; k < keep; ++k) alpha[k] = y[k] * (colnorm[0] / colnorm[k + 1]);
    return keep;
}

PolyInfo gmres_poly(const CsrView &A, uint64_t seed, int32_t level, int m, hipStream_t s) {
    AIRG_REQUIRE(m >= 1 && m + 1 <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order out of range");
    PolyInfo P;
    P.m = m;
    int64_t n = A.nr;
    if (n == 0) return P;
    DBuf<double> K((size_t)n * (m + 1), s);
    gauss_rhs(n, seed, level, K.p, s);
    for (int k = 1; k <= m; ++k) spmv(A, K.p + (int64_t)(k - 1) * n, K.p + (int64_t)k * n, nullptr, SPMV_SET, s);
    tsqr_r(K.p, n, m + 1, P.R, P.colnorm, s);
    P.used = poly_coeffs_from_r(P.R, P.colnorm, m, P.alpha);
    return P;
}

// --------------------------------------------- fixed-sparsity assembly ----
struct Coeffs {
    double a[kMaxPolyCols];
};

__global__ void k_rowlen_bin(int32_t n, const int32_t *__restrict__ rp, int8_t *__restrict__ bin) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t L = rp[i + 1] - rp[i];
    bin[i] = L <= 4 ? 0 : L <= 8 ? 1 : L <= 16 ? 2 : L <= 32 ? 3 : L <= 64 ? 4 : 5;
}

// One G-lane group per row (L = row length <= G).  M_i = A(J_i, J_i) is built
// in LDS by merging each gathered row with J_i; then v_k = v_{k-1} M_i with
// lane a owning column a, the sum over p ascending.
template <int G, int TPB>
__global__ void __launch_bounds__(TPB) k_poly_rows(const int32_t *__restrict__ list, int64_t count,
                                                   const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, Coeffs al, int nalpha,
                                                   double *__restrict__ out) {
#pragma clang fp contract(off)
    constexpr int NG = TPB / G;
    __shared__ double Ms[NG][G * G];
    __shared__ int32_t Js[NG][G];
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t b = rp[row];
    int32_t L = rp[row + 1] - b;
    double *M = Ms[gid];
    int32_t *J = Js[gid];
    if (lane < L) J[lane] = ci[b + lane];
    for (int t = lane; t < G * G; t += G) M[t] = 0.0;
    wave_sync();
    if (lane < L) {
        int32_t r = J[lane];
        int q = 0;
        for (int32_t kk = rp[r]; kk < rp[r + 1]; ++kk) {
            int32_t c = ci[kk];
            while (q < L && J[q] < c) ++q;
            if (q == L) break;
            if (J[q] == c) M[lane * G + q] = v[kk];
        }
    }
    wave_sync();
    double x = (lane < L && J[lane] == row) ? 1.0 : 0.0;
    double acc = al.a[0] * x;
    for (int k = 1; k < nalpha; ++k) {
        double xn = 0.0;
        for (int p = 0; p < L; ++p) xn += group_bcast<G>(x, p) * M[p * G + lane];
        x = xn;
        acc += al.a[k] * x;
    }
    if (lane < L) out[b + lane] = acc;
}

constexpr int kLongRowMax = 2048;

// Rows longer than 64: one block per row, J_i and the vectors in LDS, the
// gathered rows streamed once per power in ascending p.
__global__ void __launch_bounds__(256) k_poly_long(const int32_t *__restrict__ list, int64_t count,
                                                   const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, Coeffs al, int nalpha,
                                                   double *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ int32_t J[kLongRowMax];
    __shared__ double x[kLongRowMax], xn[kLongRowMax], acc[kLongRowMax];
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t b = rp[row];
    int32_t L = rp[row + 1] - b;
    for (int a = threadIdx.x; a < L; a += blockDim.x) {
        J[a] = ci[b + a];
        x[a] = J[a] == row ? 1.0 : 0.0;
        acc[a] = al.a[0] * x[a];
    }
    __syncthreads();
    for (int k = 1; k < nalpha; ++k) {
        for (int a = threadIdx.x; a < L; a += blockDim.x) xn[a] = 0.0;
        __syncthreads();
        for (int p = 0; p < L; ++p) {
            int32_t r = J[p];
            double xp = x[p];
            for (int32_t kk = rp[r] + threadIdx.x; kk < rp[r + 1]; kk += blockDim.x) {
                int32_t c = ci[kk];
                int lo = 0, hi = L;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (J[mid] < c) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < L && J[lo] == c) xn[lo] += xp * v[kk];
            }
            __syncthreads();
        }
        for (int a = threadIdx.x; a < L; a += blockDim.x) {
            x[a] = xn[a];
            acc[a] += al.a[k] * x[a];
        }
        __syncthreads();
    }
    for (int a = threadIdx.x; a < L; a += blockDim.x) out[b + a] = acc[a];
}

void poly_fixed_sparsity(const CsrView &A, const double *alpha, int nalpha, double *out_v, hipStream_t s) {
    AIRG_REQUIRE(nalpha >= 1 && nalpha <= kMaxPolyCols, ST_INVALID_ARG, "bad number of coefficients");
    int32_t n = A.nr;
    if (n == 0) return;
    Coeffs c{};
    for (int k = 0; k < nalpha; ++k) c.a[k] = alpha[k];
    DBuf<int8_t> bin((size_t)n, s);
    k_rowlen_bin<<<grid_for(n, 256), 256, 0, s>>>(n, A.rp, bin.p);
    AIRG_LAUNCH_CHECK();
    Bins B = bin_rows(bin.p, n, 6, s);
    if (B.count(0)) k_poly_rows<4, 256><<<grid_for(B.count(0), 64), 256, 0, s>>>(B.list(0), B.count(0), A.rp, A.ci, A.v, c, nalpha, out_v);
    if (B.count(1)) k_poly_rows<8, 256><<<grid_for(B.count(1), 32), 256, 0, s>>>(B.list(1), B.count(1), A.rp, A.ci, A.v, c, nalpha, out_v);
    if (B.count(2)) k_poly_rows<16, 256><<<grid_for(B.count(2), 16), 256, 0, s>>>(B.list(2), B.count(2), A.rp, A.ci, A.v, c, nalpha, out_v);
    if (B.count(3)) k_poly_rows<32, 128><<<grid_for(B.count(3), 4), 128, 0, s>>>(B.list(3), B.count(3), A.rp, A.ci, A.v, c, nalpha, out_v);
    if (B.count(4)) k_poly_rows<64, 64><<<grid_for(B.count(4), 1), 64, 0, s>>>(B.list(4), B.count(4), A.rp, A.ci, A.v, c, nalpha, out_v);
    AIRG_LAUNCH_CHECK();
    if (B.count(5)) {
        int32_t maxlen = 0;
        {
            // longest row among the long ones, checked against the LDS capacity
            std::vector<int32_t> rows((size_t)B.count(5)), rpl((size_t)n + 1);
            d2h(rows.data(), B.list(5), rows.size(), s);
            d2h(rpl.data(), A.rp, rpl.size(), s);
            for (int32_t r : rows) maxlen = std::max(maxlen, rpl[r + 1] - rpl[r]);
        }
        AIRG_REQUIRE(maxlen <= kLongRowMax, ST_LIMIT,
                     "row of " + std::to_string(maxlen) + " entries exceeds the fixed-sparsity row limit");
        k_poly_long<<<(unsigned)B.count(5), 256, 0, s>>>(B.list(5), B.count(5), A.rp, A.ci, A.v, c, nalpha, out_v);
        AIRG_LAUNCH_CHECK();
    }
}

}  // namespace airg

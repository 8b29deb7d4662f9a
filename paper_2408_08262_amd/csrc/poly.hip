// GMRES-polynomial kernels for gfx950: Box-Muller rhs, column norms, a
// tall-skinny Householder QR tree in LDS, and the row-local fixed-sparsity
// power sum (one lane group per row, M_i staged in LDS).
#include <cmath>

#include "csr.hpp"
#include "group.hpp"
#include "poly.hpp"
#include "spgemm.hpp"

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

// Batch segments: entry k of segment p draws with p's seed at the index k
// takes within the segment.
__global__ void k_gauss_seg(int32_t n, const int32_t *__restrict__ off, int nseg, const uint64_t *__restrict__ seeds,
                            int32_t level, double *__restrict__ b) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int p = seg_of(off, nseg, k);
    const double two53 = 1.0 / 9007199254740992.0;
    uint64_t local = (uint64_t)(k - off[p]);
    uint64_t r1 = splitmix64(rng_counter(seeds[p], 1, (uint32_t)level, local));
    uint64_t r2 = splitmix64(rng_counter(seeds[p], 2, (uint32_t)level, local));
    double u1 = ((double)(r1 >> 11) + 1.0) * two53;
    double u2 = (double)(r2 >> 11) * two53;
    b[k] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// ------------------------------------------------------------ reductions ---
constexpr int kQrThreads = 256;       // column-norm reductions
constexpr int kQrLanes = 64;          // one wavefront per QR panel
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

// -------------------------------------------------------------- TSQR leaf ---
// Householder QR of a panel of `rows` (<= kQrRows) rows x cols (columns
// scaled by `scale` when given) by one wavefront, the panel held in
// registers: lane l owns rows l, l + 64, ... of every column.  The column
// loop is unrolled over the compile-time width NC >= cols, so every register
// index is a constant and step col touches only the columns after it (a
// triangular amount of work; no register shifts).  The reductions are DPP
// wave sums, the independent ones of a step side by side.  Row `col` of R is
// taken after step col (alpha on the diagonal, or x0 when the column below is
// already zero); R (cols x cols, upper triangular) is written column-major at
// out with leading dimension ldo, through Rl (cols * cols doubles of LDS).
template <int NC>
__device__ __forceinline__ void qr_panel(const double *__restrict__ K, int64_t ldk, int64_t r0, int rows, int cols,
                         const double *__restrict__ scale, double *__restrict__ out, int64_t ldo,
                         double *__restrict__ Rl) {
    constexpr int RPL = kQrRows / kQrLanes;
    const int lane = threadIdx.x;
    const double scv = scale && lane < cols ? scale[lane] : 1.0;
    double W[RPL][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double sc = readlane_f64(scv, c);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const int r = lane + j * kQrLanes;
            W[j][c] = c < cols && r < rows ? K[(int64_t)c * ldk + r0 + r] * sc : 0.0;
        }
    }
    for (int idx = lane; idx < cols * cols; idx += kQrLanes) Rl[idx] = 0.0;
    wave_sync();
#pragma clang loop unroll(full)
    for (int col = 0; col < NC; ++col) {
        if (col >= cols) continue;   // uniform
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < RPL; ++j)
            if (lane + j * kQrLanes >= col) part += W[j][col] * W[j][col];
        const double nx2 = wave_sum_f64(part);
        const double x0 = readlane_f64(W[0][col], col);   // row col: lane col (cols <= 64)
        const double nx = sqrt(nx2);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        const double vv = 2.0 * nx * (nx + fabs(x0));
        double diag = x0;
        if (vv > 0.0) {
            double v[RPL];
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
                const int r = lane + j * kQrLanes;
                v[j] = r == col ? x0 - alpha : (r > col ? W[j][col] : 0.0);
            }
            // the dot products of the columns after col, then their wave
            // sums side by side (independent reductions overlap)
            double d[NC];
#pragma unroll
            for (int c = col + 1; c < NC; ++c) {
                d[c] = 0.0;
#pragma unroll
                for (int j = 0; j < RPL; ++j) d[c] += v[j] * W[j][c];
            }
#pragma unroll
            for (int c = col + 1; c < NC; ++c) d[c] = wave_sum_f64(d[c]);
#pragma unroll
            for (int c = col + 1; c < NC; ++c) {
                if (c < cols) {
                    const double f = 2.0 * d[c] / vv;
#pragma unroll
                    for (int j = 0; j < RPL; ++j) W[j][c] -= f * v[j];
                }
            }
            diag = alpha;
        }
        // row col of R: lane t < cols - col takes entry (col, col + t)
        double mine = diag;
#pragma unroll
        for (int c = col + 1; c < NC; ++c) {
            if (c < cols) {
                const double t = readlane_f64(W[0][c], col);
                if (lane == c - col) mine = t;
            }
        }
        if (lane < cols - col) Rl[(col + lane) * cols + col] = mine;
    }
    wave_sync();
    for (int idx = lane; idx < cols * cols; idx += kQrLanes) {
        const int c = idx / cols, r = idx % cols;
        out[(int64_t)c * ldo + r] = Rl[idx];
    }
}
template <int NC>
__global__ void __launch_bounds__(kQrLanes) k_tsqr_leaf(const double *__restrict__ K, int64_t n, int64_t ldk,
                                                        int cols, const double *__restrict__ scale,
                                                        double *__restrict__ Rs, int64_t ldr) {
    __shared__ double Rl[NC * NC];
    int64_t r0 = (int64_t)blockIdx.x * kQrRows;
    int rows = (int)(n - r0 < kQrRows ? n - r0 : kQrRows);
    qr_panel<NC>(K, ldk, r0, rows, cols, scale, Rs + (int64_t)blockIdx.x * cols, ldr, Rl);
}

// Batch form: one leaf per table entry; a leaf with fin >= 0 is the last of
// segment fin and writes that segment's final R (cols x cols, column-major).
struct QrLeaf {
    int64_t r0;      // first row in the source
    int32_t rows;
    int32_t seg;     // scale row (first tree level), else unused
    int64_t out;     // first row in the stacked output
    int32_t fin;
    int32_t pad;
};

template <int NC>
__global__ void __launch_bounds__(kQrLanes) k_tsqr_leaf_tab(const double *__restrict__ K, int64_t ldk, int cols,
                                                              const QrLeaf *__restrict__ leaves,
                                                              const double *__restrict__ scale,
                                                              double *__restrict__ Rs, int64_t ldr,
                                                              double *__restrict__ Rf) {
    __shared__ double Rl[NC * NC];
    QrLeaf L = leaves[blockIdx.x];
    const double *sc = scale ? scale + (int64_t)L.seg * cols : nullptr;
    double *out = L.fin >= 0 ? Rf + (int64_t)L.fin * cols * cols : Rs + L.out;
    qr_panel<NC>(K, ldk, L.r0, L.rows, cols, sc, out, L.fin >= 0 ? (int64_t)cols : ldr, Rl);
}

// partial[leaf * cols + c] = sum over the leaf's rows of K[:, c]^2
__global__ void __launch_bounds__(kQrThreads) k_colsq_tab(const double *__restrict__ K, int64_t ldk, int cols,
                                                          const QrLeaf *__restrict__ leaves,
                                                          double *__restrict__ partial) {
    __shared__ double sh[4 * kMaxPolyCols];
    QrLeaf L = leaves[blockIdx.x];
    double v[kMaxPolyCols];
#pragma unroll
    for (int c = 0; c < kMaxPolyCols; ++c) v[c] = 0.0;
    for (int r = threadIdx.x; r < L.rows; r += kQrThreads) {
#pragma unroll
        for (int c = 0; c < kMaxPolyCols; ++c)
            if (c < cols) {
                double x = K[(int64_t)c * ldk + L.r0 + r];
                v[c] += x * x;
            }
    }
    block_sum_vec<kMaxPolyCols>(v, cols, sh);
    if (threadIdx.x < cols) partial[(int64_t)blockIdx.x * cols + threadIdx.x] = v[threadIdx.x];
}

// Per segment p (leaves first[p] .. first[p+1]-1, summed in order): column
// norms into out[p * cols + c] and their inverses into inv.
__global__ void k_colsq_seg_finish(const double *__restrict__ partial, const int32_t *__restrict__ first, int nseg,
                                   int cols, double *__restrict__ norm, double *__restrict__ inv) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nseg * cols) return;
    int p = (int)(t / cols), c = (int)(t % cols);
    double acc = 0.0;
    for (int q = first[p]; q < first[p + 1]; ++q) acc += partial[(int64_t)q * cols + c];
    double nr = sqrt(acc);
    norm[t] = nr;
    inv[t] = nr > 0.0 ? 1.0 / nr : 1.0;
}

// R of the column-scaled basis K D (D = diag(1 / ||K e_c||)) by a tree of
// Householder panels over K itself: Householder QR is columnwise backward
// stable, so R(K D) = R(K) D up to rounding, and the column norms of K are
// those of R(K).  The scaling is therefore applied to the final R on the host
// and the norms need no pass over K.
static void tsqr_r_x(const double *K, int64_t n, int cols, double *h_R, double *h_colnorm, hipStream_t s,
                     const ExtraReads *extra);
void tsqr_r(const double *K, int64_t n, int cols, double *h_R, double *h_colnorm, hipStream_t s) {
    tsqr_r_x(K, n, cols, h_R, h_colnorm, s, nullptr);
}
static void tsqr_r_x(const double *K, int64_t n, int cols, double *h_R, double *h_colnorm, hipStream_t s,
                     const ExtraReads *extra) {
    AIRG_REQUIRE(cols >= 1 && cols <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order too large");
    const double *src = K;
    int64_t rows = n, ld = n;
    DBuf<double> bufs[2];
    int which = 0;
    for (;;) {
        int64_t nb = (rows + kQrRows - 1) / kQrRows;
        if (nb < 1) nb = 1;
        int64_t out_rows = nb * cols;
        bufs[which].alloc((size_t)out_rows * cols, s);
        if (cols <= 8)
            k_tsqr_leaf<8><<<(unsigned)nb, kQrLanes, 0, s>>>(src, rows, ld, cols, nullptr, bufs[which].p, out_rows);
        else
            k_tsqr_leaf<kMaxPolyCols><<<(unsigned)nb, kQrLanes, 0, s>>>(src, rows, ld, cols, nullptr, bufs[which].p,
                                                                       out_rows);
        AIRG_LAUNCH_CHECK();
        src = bufs[which].p;
        rows = out_rows;
        ld = out_rows;
        which ^= 1;
        if (nb == 1) break;
    }
    std::vector<double> R((size_t)cols * cols);   // column-major
    if (!extra) {
        d2h(R.data(), src, R.size(), s);
    } else {
        // R and the caller's ranges in one readback
        std::vector<const int32_t *> srcs{reinterpret_cast<const int32_t *>(src)};
        std::vector<int32_t> cnts{2 * cols * cols};
        srcs.insert(srcs.end(), extra->src.begin(), extra->src.end());
        cnts.insert(cnts.end(), extra->cnt.begin(), extra->cnt.end());
        int64_t words = 0;
        for (int32_t c : cnts) words += c;
        std::vector<int32_t> h((size_t)words);
        read_ints(srcs, cnts, h.data(), s);
        std::memcpy(R.data(), h.data(), R.size() * sizeof(double));
        std::copy(h.begin() + 2 * cols * cols, h.end(), extra->h);
    }
    for (int c = 0; c < cols; ++c) {
        double ss = 0.0;
        for (int r = 0; r <= c; ++r) ss += R[(size_t)c * cols + r] * R[(size_t)c * cols + r];
        h_colnorm[c] = std::sqrt(ss);
    }
    for (int r = 0; r < cols; ++r)
        for (int c = 0; c < cols; ++c) {
            const double sc = h_colnorm[c] > 0.0 ? 1.0 / h_colnorm[c] : 1.0;
            h_R[r * cols + c] = r <= c ? R[(size_t)c * cols + r] * sc : 0.0;
        }
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

PolyInfo gmres_poly(const CsrView &A, uint64_t seed, int32_t level, int m, hipStream_t s, const ExtraReads *extra) {
    AIRG_REQUIRE(m >= 1 && m + 1 <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order out of range");
    PolyInfo P;
    P.m = m;
    int64_t n = A.nr;
    if (n == 0) {
        if (extra && !extra->src.empty()) read_ints(extra->src, extra->cnt, extra->h, s);
        return P;
    }
    DBuf<double> K((size_t)n * (m + 1), s);
    gauss_rhs(n, seed, level, K.p, s);
    for (int k = 1; k <= m; ++k) spmv(A, K.p + (int64_t)(k - 1) * n, K.p + (int64_t)k * n, nullptr, SPMV_SET, s);
    tsqr_r_x(K.p, n, m + 1, P.R, P.colnorm, s, extra && !extra->src.empty() ? extra : nullptr);
    P.used = poly_coeffs_from_r(P.R, P.colnorm, m, P.alpha);
    return P;
}

void tsqr_r_seg(const double *K, const std::vector<int32_t> &off, int cols, double *h_R, double *h_colnorm,
                hipStream_t s) {
    AIRG_REQUIRE(cols >= 1 && cols <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order too large");
    const int nseg = (int)off.size() - 1;
    const int64_t n = off[nseg];
    // first tree level: the segments' own row blocks
    std::vector<QrLeaf> leaves;
    std::vector<int32_t> first(nseg + 1, 0);
    std::vector<int64_t> rows0(nseg), start0(nseg);
    for (int p = 0; p < nseg; ++p) {
        first[p] = (int32_t)leaves.size();
        int64_t m = off[p + 1] - off[p];
        for (int64_t r = 0; r < m || r == 0; r += kQrRows)
            leaves.push_back(QrLeaf{off[p] + r, (int32_t)std::min<int64_t>(kQrRows, m - r), p, 0, -1, 0});
        rows0[p] = m;
        start0[p] = off[p];
    }
    first[nseg] = (int32_t)leaves.size();
    // column norms per segment
    DBuf<QrLeaf> dl(leaves.size(), s);
    DBuf<int32_t> dfirst(first.size(), s);
    DBuf<double> part(leaves.size() * cols, s), normout((size_t)nseg * cols * (cols + 1), s), inv((size_t)nseg * cols, s);
    h2d(dl.p, leaves.data(), leaves.size(), s);
    h2d(dfirst.p, first.data(), first.size(), s);
    k_colsq_tab<<<(unsigned)leaves.size(), kQrThreads, 0, s>>>(K, n, cols, dl.p, part.p);
    AIRG_LAUNCH_CHECK();
    double *Rf = normout.p;                               // nseg * cols * cols, then the norms
    double *norm = normout.p + (size_t)nseg * cols * cols;
    k_colsq_seg_finish<<<grid_for((int64_t)nseg * cols, 256), 256, 0, s>>>(part.p, dfirst.p, nseg, cols, norm, inv.p);
    AIRG_LAUNCH_CHECK();
    // further tree levels: every unfinished segment's rows -> one R per leaf, stacked
    std::vector<int64_t> rows = rows0, start = start0;
    std::vector<char> done(nseg, 0);
    const double *src = K;
    int64_t ld = n;
    bool scaled = true;
    DBuf<double> bufs[2];
    std::vector<DBuf<QrLeaf>> tables;
    std::vector<std::vector<QrLeaf>> host_tabs;   // sources of the async copies, kept until the final sync
    int which = 0;
    for (;;) {
        host_tabs.emplace_back();
        std::vector<QrLeaf> &tab = host_tabs.back();
        int64_t out_rows = 0;
        std::vector<int64_t> nrows(nseg, 0), nstart(nseg, 0);
        for (int p = 0; p < nseg; ++p) {
            if (done[p]) continue;
            int64_t nb = std::max<int64_t>(1, (rows[p] + kQrRows - 1) / kQrRows);
            if (nb == 1) {
                tab.push_back(QrLeaf{start[p], (int32_t)rows[p], p, 0, p, 0});
                done[p] = 1;
                continue;
            }
            nstart[p] = out_rows;
            for (int64_t b = 0; b < nb; ++b)
                tab.push_back(QrLeaf{start[p] + b * kQrRows, (int32_t)std::min<int64_t>(kQrRows, rows[p] - b * kQrRows),
                                     p, out_rows + b * cols, -1, 0});
            nrows[p] = nb * cols;
            out_rows += nb * cols;
        }
        if (tab.empty()) break;
        tables.emplace_back(tab.size(), s);
        h2d(tables.back().p, tab.data(), tab.size(), s);
        bufs[which].alloc((size_t)std::max<int64_t>(out_rows, 1) * cols, s);
        auto leaf_tab = cols <= 8 ? k_tsqr_leaf_tab<8> : k_tsqr_leaf_tab<kMaxPolyCols>;
        leaf_tab<<<(unsigned)tab.size(), kQrLanes, 0, s>>>(src, ld, cols, tables.back().p, scaled ? inv.p : nullptr,
                                                          bufs[which].p, std::max<int64_t>(out_rows, 1), Rf);
        AIRG_LAUNCH_CHECK();
        src = bufs[which].p;
        ld = std::max<int64_t>(out_rows, 1);
        scaled = false;
        rows = nrows;
        start = nstart;
        which ^= 1;
        if (out_rows == 0) break;
    }
    std::vector<double> h((size_t)nseg * cols * (cols + 1));
    d2h(h.data(), normout.p, h.size(), s);
    for (int p = 0; p < nseg; ++p) {
        const double *R = h.data() + (size_t)p * cols * cols;
        for (int r = 0; r < cols; ++r)
            for (int c = 0; c < cols; ++c) h_R[(size_t)p * cols * cols + r * cols + c] = R[(size_t)c * cols + r];
        for (int c = 0; c < cols; ++c) h_colnorm[(size_t)p * cols + c] = h[(size_t)nseg * cols * cols + p * cols + c];
    }
}

std::vector<PolyInfo> gmres_poly_seg(const CsrView &A, const std::vector<int32_t> &off, const int32_t *d_off,
                                     const uint64_t *d_seeds, int32_t level, int m, hipStream_t s) {
    AIRG_REQUIRE(m >= 1 && m + 1 <= kMaxPolyCols, ST_INVALID_ARG, "polynomial order out of range");
    const int nseg = (int)off.size() - 1;
    std::vector<PolyInfo> P(nseg);
    for (auto &q : P) q.m = m;
    int32_t n = A.nr;
    if (n == 0) return P;
    DBuf<double> K((size_t)n * (m + 1), s);
    k_gauss_seg<<<grid_for(n, 256), 256, 0, s>>>(n, d_off, nseg, d_seeds, level, K.p);
    AIRG_LAUNCH_CHECK();
    for (int k = 1; k <= m; ++k) spmv(A, K.p + (int64_t)(k - 1) * n, K.p + (int64_t)k * n, nullptr, SPMV_SET, s);
    int cols = m + 1;
    std::vector<double> R((size_t)nseg * cols * cols), cn((size_t)nseg * cols);
    tsqr_r_seg(K.p, off, cols, R.data(), cn.data(), s);
    for (int p = 0; p < nseg; ++p) {
        std::copy(R.begin() + (size_t)p * cols * cols, R.begin() + (size_t)(p + 1) * cols * cols, P[p].R);
        std::copy(cn.begin() + (size_t)p * cols, cn.begin() + (size_t)(p + 1) * cols, P[p].colnorm);
        P[p].used = poly_coeffs_from_r(P[p].R, P[p].colnorm, m, P[p].alpha);
    }
    return P;
}

// --------------------------------------------- fixed-sparsity assembly ----
// One G-lane group per row (L = row length <= G).  M_i = A(J_i, J_i) is built
// in LDS: the pairs (column, position) of J_i go into a small LDS hash of
// two-slot buckets (4G slots for groups of 32 lanes, 2G otherwise; a key
// goes to the first bucket from its home with a free slot, so a lookup ends
// at the first bucket that holds it or has a free slot).  The group then
// reads the gathered rows A(J_i[p], :) in batches of rows, lane t taking
// entries t, t + G, ... of each row, and looks every column up.  The lookups
// of a batch probe in step: one round reads the current bucket of every row
// of the batch (independent LDS reads behind one wait), so a batch costs as
// many LDS round trips as its longest probe sequence.  Then
// v_k = v_{k-1} M_i with lane a owning column a of M_i in registers, the sum
// over p ascending; v_{k-1} is broadcast through LDS, two entries per read.
// Over the earlier form (each lane walking its own gathered row, M_i read
// from LDS in the powers, x broadcast by lane reads) this takes the coarsest
// dg_square_512 assembly from 0.67 to 0.47 ms.
template <int NB>
__device__ inline uint32_t poly_hash(int32_t c) {   // multiplicative hash, top bits
    constexpr int kBits = __builtin_ctz(NB);
    static_assert(NB >= 2 && (NB & (NB - 1)) == 0, "a power-of-two bucket count");
    return ((uint32_t)c * 2654435761u) >> (32 - kBits);
}

// MS (<= G): the rows of the launch have at most MS entries, and M_i is
// stored MS x MS, so that a bin of shorter rows holds more of them in LDS.
template <int G, int TPB, int MS>
__global__ void __launch_bounds__(TPB) k_poly_rows(const int32_t *__restrict__ list, int64_t count,
                                                   const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, const int32_t *__restrict__ prp,
                                                   const int32_t *__restrict__ pci, const double *__restrict__ alt,
                                                   const int32_t *__restrict__ soff, int nseg, int nalpha,
                                                   double *__restrict__ out) {
#pragma clang fp contract(off)
    static_assert(MS <= G, "row capacity above the group width");
    constexpr int NG = TPB / G;
    constexpr int NB = G == 32 ? 2 * G : G;   // hash buckets of two slots
    constexpr uint32_t kHM = NB - 1;
    __shared__ __align__(16) double Ms[NG][MS * MS];
    __shared__ __align__(16) double Xs[NG][G];
    __shared__ int4 Hs[NG][NB];   // (column, position) x 2; column -1 marks an empty slot
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t b = prp[row];
    int32_t L = prp[row + 1] - b;
    double *M = Ms[gid];
    double *X = Xs[gid];
    int4 *H = Hs[gid];
    const int32_t myc = lane < L ? pci[b + lane] : -1;
    const int32_t rb = lane < L ? rp[myc] : 0;       // extent of the gathered row J_i[lane]
    const int32_t re = lane < L ? rp[myc + 1] : 0;
    for (int t = lane; t < NB; t += G) H[t] = make_int4(-1, 0, -1, 0);
    static_assert(MS % 2 == 0, "M_i rows of an even length, cleared two entries at a time");
    for (int t = lane; t < MS * MS / 2; t += G) reinterpret_cast<double2 *>(M)[t] = make_double2(0.0, 0.0);
    wave_sync();
    if (lane < L) {   // columns are distinct: each claims its own slot
        uint32_t h = poly_hash<NB>(myc);
        for (;;) {   // L <= G < 2 NB keys: a free slot remains
            if (atomicCAS(&H[h].x, -1, myc) == -1) {
                H[h].y = lane;
                break;
            }
            if (atomicCAS(&H[h].z, -1, myc) == -1) {
                H[h].w = lane;
                break;
            }
            h = (h + 1) & kHM;
        }
    }
    wave_sync();
    // row p of M_i is row J_i[p] of A against J_i; a row's columns are
    // distinct, so its lanes write distinct entries.  Pass q takes entries
    // qG .. qG + G - 1 of every gathered row (as many passes as the group's
    // longest gathered row needs), RB rows loaded before any is looked up.
    // The pad rows p >= L have the empty extent [0, 0).
    constexpr int RB = MS <= 4 ? MS : MS <= 8 ? 4 : MS <= 24 ? 8 : 16;
    static_assert((MS + RB - 1) / RB * RB <= G, "padded row batches exceed the group");
    const int passes = group_max<G>((re - rb + G - 1) / G);
    for (int q = 0; q < passes; ++q)
    for (int p0 = 0; p0 < L; p0 += RB) {
        int32_t cb[RB];
        double vb[RB];
        uint32_t hb[RB];
        int32_t kb[RB], eb[RB];
        uint32_t pend = 0;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            if constexpr (G == 64) {   // one group per wavefront: p0 + u is uniform, a lane read
                kb[u] = __builtin_amdgcn_readlane(rb, p0 + u) + q * G + lane;
                eb[u] = __builtin_amdgcn_readlane(re, p0 + u);
            } else {
                kb[u] = group_bcast<G>(rb, p0 + u) + q * G + lane;
                eb[u] = group_bcast<G>(re, p0 + u);
            }
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const bool ok = kb[u] < eb[u];
            cb[u] = ok ? ci[kb[u]] : -1;
            vb[u] = ok ? v[kb[u]] : 0.0;
            pend |= ok ? 1u << u : 0u;
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) hb[u] = poly_hash<NB>(cb[u]);
        while (pend) {
            int4 kv[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) kv[u] = H[hb[u]];   // every bucket index is in range
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const bool on = (pend >> u) & 1u;
                const bool h0 = kv[u].x == cb[u];
                const bool hit = on && (h0 || kv[u].z == cb[u]);
                const bool stop = hit || kv[u].z < 0;
                if (hit) M[(p0 + u) * MS + (h0 ? kv[u].y : kv[u].w)] = vb[u];
                pend &= on && stop ? ~(1u << u) : ~0u;
                hb[u] = on && !stop ? (hb[u] + 1) & kHM : hb[u];
            }
        }
    }
    wave_sync();
    // Lane a keeps column a of M_i in registers.  Every power sums all MS
    // terms in ascending p: the terms past L are 0 * 0 (rows and columns of
    // M_i past L are zero, and so is x there, which is reset after every
    // power), and adding +0 leaves a sum that starts at +0 unchanged, so the
    // sum equals the one over p < L.
    double Mr[MS];
#pragma unroll
    for (int p = 0; p < MS; ++p) {
        const double m = M[p * MS + min(lane, MS - 1)];   // read on every lane, kept below MS
        Mr[p] = lane < MS ? m : 0.0;
    }
    const double *al = alt + (nseg > 1 ? seg_of(soff, nseg, row) : 0) * kMaxPolyCols;
    double x = (lane < L && myc == row) ? 1.0 : 0.0;
    double acc = al[0] * x;
    for (int k = 1; k < nalpha; ++k) {
        X[lane] = x;
        wave_sync();
        double xn = 0.0;
#pragma unroll
        for (int p = 0; p < MS; p += 2) {
            const double2 xp = *reinterpret_cast<const double2 *>(X + p);   // same address on every lane
            xn += xp.x * Mr[p];
            xn += xp.y * Mr[p + 1];
        }
        wave_sync();
        xn = lane < L ? xn : 0.0;
        x = xn;
        acc += al[k] * x;
    }
    if (lane < L) out[b + lane] = acc;
}

constexpr int kLongRowMax = 2048;

// Rows longer than 64: one block per row, J_i and the vectors in LDS, the
// gathered rows streamed once per power in ascending p.
__global__ void __launch_bounds__(256) k_poly_long(const int32_t *__restrict__ list, int64_t count,
                                                   const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ v, const int32_t *__restrict__ prp,
                                                   const int32_t *__restrict__ pci, const double *__restrict__ alt,
                                                   const int32_t *__restrict__ soff, int nseg, int nalpha,
                                                   double *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ int32_t J[kLongRowMax];
    __shared__ double x[kLongRowMax], xn[kLongRowMax], acc[kLongRowMax];
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t b = prp[row];
    int32_t L = prp[row + 1] - b;
    const double *al = alt + (nseg > 1 ? seg_of(soff, nseg, row) : 0) * kMaxPolyCols;
    for (int a = threadIdx.x; a < L; a += blockDim.x) {
        J[a] = pci[b + a];
        x[a] = J[a] == row ? 1.0 : 0.0;
        acc[a] = al[0] * x[a];
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
            acc[a] += al[k] * x[a];
        }
        __syncthreads();
    }
    for (int a = threadIdx.x; a < L; a += blockDim.x) out[b + a] = acc[a];
}

FixedPlan fixed_sparsity_begin(const CsrView &Pt, hipStream_t s) {
    FixedPlan F;
    const int32_t n = Pt.nr;
    F.bin.alloc((size_t)n + 1, s);
    // bins by row length: <= 4, 8, 16, 24, 32, 48, 64, longer
    const BinRule rule{{4, 8, 16, 24, 32, 48, 64}, 7};
    F.bins = bin_rows_begin_rule(Pt.rp, true, rule, F.bin.p, n, kFixedBins, s);
    return F;
}

// Rows of the pattern by length (bins of fixed_sparsity_begin), and the
// longest of the long ones checked against the LDS capacity of k_poly_long.
static Bins fixed_bins(const CsrView &Pt, FixedPlan &F, const int32_t *h_tot, hipStream_t s) {
    Bins B = bin_rows_end(F.bins, h_tot, s);
    if (B.count(kFixedLongBin)) {
        int32_t maxlen = 0;
        {
            std::vector<int32_t> lr((size_t)B.count(kFixedLongBin)), rpl((size_t)Pt.nr + 1);
            d2h(lr.data(), B.list(kFixedLongBin), lr.size(), s);
            d2h(rpl.data(), Pt.rp, rpl.size(), s);
            for (int32_t r : lr) maxlen = std::max(maxlen, rpl[r + 1] - rpl[r]);
        }
        AIRG_REQUIRE(maxlen <= kLongRowMax, ST_LIMIT,
                     "row of " + std::to_string(maxlen) + " entries exceeds the fixed-sparsity row limit");
    }
    return B;
}

// Coefficient table (kMaxPolyCols per segment) and segment offsets on the
// device; nseg = 1 needs no offsets.
static void fixed_sparsity_binned(const CsrView &A, const CsrView &Pt, const double *alt, const int32_t *soff,
                                  int nseg, int nalpha, double *out_v, const Bins &B, hipStream_t s) {
    auto rows = [&](auto kern, int b, int per_block, unsigned tpb) {
        if (B.count(b))
            kern<<<grid_for(B.count(b), per_block), tpb, 0, s>>>(B.list(b), B.count(b), A.rp, A.ci, A.v, Pt.rp,
                                                                Pt.ci, alt, soff, nseg, nalpha, out_v);
    };
    rows(k_poly_rows<4, 256, 4>, 0, 64, 256);
    rows(k_poly_rows<8, 256, 8>, 1, 32, 256);
    rows(k_poly_rows<16, 256, 16>, 2, 16, 256);
    rows(k_poly_rows<32, 128, 24>, 3, 4, 128);
    rows(k_poly_rows<32, 128, 32>, 4, 4, 128);
    rows(k_poly_rows<64, 64, 48>, 5, 1, 64);
    rows(k_poly_rows<64, 64, 64>, 6, 1, 64);
    AIRG_LAUNCH_CHECK();
    if (B.count(kFixedLongBin)) {
        k_poly_long<<<(unsigned)B.count(kFixedLongBin), 256, 0, s>>>(B.list(kFixedLongBin), B.count(kFixedLongBin),
                                                                     A.rp, A.ci, A.v, Pt.rp, Pt.ci, alt, soff, nseg,
                                                                     nalpha, out_v);
        AIRG_LAUNCH_CHECK();
    }
}

static void fixed_sparsity_run(const CsrView &A, const CsrView &Pt, const double *alt, const int32_t *soff, int nseg,
                               int nalpha, double *out_v, FixedPlan &F, const int32_t *h_tot, hipStream_t s) {
    Bins B = fixed_bins(Pt, F, h_tot, s);
    fixed_sparsity_binned(A, Pt, alt, soff, nseg, nalpha, out_v, B, s);
}

static void fixed_sparsity_tab(const CsrView &A, const CsrView &Pt, const double *alt, const int32_t *soff,
                               int nseg, int nalpha, double *out_v, hipStream_t s) {
    FixedPlan F = fixed_sparsity_begin(Pt, s);
    int32_t h[kFixedBins + 1];
    d2h(h, F.bins.tot.p, (size_t)kFixedBins + 1, s);
    fixed_sparsity_run(A, Pt, alt, soff, nseg, nalpha, out_v, F, h, s);
}

// The single form's coefficients, written to the device by a kernel that
// takes them as arguments (no host staging to outlive).
struct CoefArgs {
    double a[kMaxPolyCols];
};
__global__ void k_set_coefs(CoefArgs c, double *__restrict__ out) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kMaxPolyCols; ++k) out[k] = c.a[k];
    }
}

Bins poly_pattern_bins(const CsrView &Pt, hipStream_t s) {
    FixedPlan F = fixed_sparsity_begin(Pt, s);
    int32_t h[kFixedBins + 1];
    d2h(h, F.bins.tot.p, (size_t)kFixedBins + 1, s);
    return fixed_bins(Pt, F, h, s);
}

void poly_fixed_sparsity_binned(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha, double *out_v,
                                const Bins &B, hipStream_t s) {
    AIRG_REQUIRE(nalpha >= 1 && nalpha <= kMaxPolyCols, ST_INVALID_ARG, "bad number of coefficients");
    AIRG_REQUIRE(Pt.nr == A.nr, ST_INVALID_ARG, "pattern and matrix differ in rows");
    if (A.nr == 0) return;
    CoefArgs c{};
    for (int k = 0; k < nalpha; ++k) c.a[k] = alpha[k];
    DBuf<double> alt(kMaxPolyCols, s);
    k_set_coefs<<<1, 64, 0, s>>>(c, alt.p);
    AIRG_LAUNCH_CHECK();
    fixed_sparsity_binned(A, Pt, alt.p, nullptr, 1, nalpha, out_v, B, s);
}

void poly_fixed_sparsity_planned(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha,
                                 double *out_v, FixedPlan &plan, const int32_t *h_tot, hipStream_t s) {
    AIRG_REQUIRE(nalpha >= 1 && nalpha <= kMaxPolyCols, ST_INVALID_ARG, "bad number of coefficients");
    AIRG_REQUIRE(Pt.nr == A.nr, ST_INVALID_ARG, "pattern and matrix differ in rows");
    if (A.nr == 0) return;
    CoefArgs c{};
    for (int k = 0; k < nalpha; ++k) c.a[k] = alpha[k];
    DBuf<double> alt(kMaxPolyCols, s);
    k_set_coefs<<<1, 64, 0, s>>>(c, alt.p);
    AIRG_LAUNCH_CHECK();
    fixed_sparsity_run(A, Pt, alt.p, nullptr, 1, nalpha, out_v, plan, h_tot, s);
}

void poly_fixed_sparsity(const CsrView &A, const double *alpha, int nalpha, double *out_v, hipStream_t s) {
    poly_fixed_sparsity_pattern(A, A, alpha, nalpha, out_v, s);
}

void poly_fixed_sparsity_pattern(const CsrView &A, const CsrView &Pt, const double *alpha, int nalpha,
                                 double *out_v, hipStream_t s) {
    AIRG_REQUIRE(nalpha >= 1 && nalpha <= kMaxPolyCols, ST_INVALID_ARG, "bad number of coefficients");
    AIRG_REQUIRE(Pt.nr == A.nr, ST_INVALID_ARG, "pattern and matrix differ in rows");
    if (A.nr == 0) return;
    double tab[kMaxPolyCols] = {};
    for (int k = 0; k < nalpha; ++k) tab[k] = alpha[k];
    DBuf<double> alt(kMaxPolyCols, s);
    h2d(alt.p, tab, kMaxPolyCols, s);
    fixed_sparsity_tab(A, Pt, alt.p, nullptr, 1, nalpha, out_v, s);   // synchronises (row binning) before tab dies
}

void poly_fixed_sparsity_seg(const CsrView &A, const CsrView &Pt, const std::vector<int32_t> &off,
                             const std::vector<PolyInfo> &P, double *out_v, hipStream_t s) {
    const int nseg = (int)P.size();
    AIRG_REQUIRE(nseg >= 1 && (int)off.size() == nseg + 1, ST_INVALID_ARG, "bad segment table");
    if (A.nr == 0) return;
    int nalpha = P[0].m;
    AIRG_REQUIRE(nalpha >= 1 && nalpha <= kMaxPolyCols, ST_INVALID_ARG, "bad number of coefficients");
    std::vector<double> tab((size_t)nseg * kMaxPolyCols, 0.0);
    for (int p = 0; p < nseg; ++p) {
        AIRG_REQUIRE(P[p].m == nalpha, ST_INVALID_ARG, "segments differ in polynomial order");
        for (int k = 0; k < nalpha; ++k) tab[(size_t)p * kMaxPolyCols + k] = P[p].alpha[k];
    }
    DBuf<double> alt(tab.size(), s);
    DBuf<int32_t> soff(off.size(), s);
    h2d(alt.p, tab.data(), tab.size(), s);
    h2d(soff.p, off.data(), off.size(), s);
    fixed_sparsity_tab(A, Pt, alt.p, soff.p, nseg, nalpha, out_v, s);   // synchronises before the tables die
}

Csr power_pattern(const CsrView &A, int order, hipStream_t s) {
    AIRG_REQUIRE(order >= 1 && order <= 3, ST_INVALID_ARG, "sparsity order must be 1, 2 or 3");
    Csr P = spgemm(A, A, s);
    if (order == 3) P = spgemm(view(P), A, s);
    return P;
}

}  // namespace airg

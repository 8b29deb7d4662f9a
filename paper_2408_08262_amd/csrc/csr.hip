// Sparse building blocks on gfx950: validation, CSR SpMV/SpMM with G lanes
// per row, CF block extraction, row drop filter, transpose, reductions.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <tuple>

#include <hip/hip_ext.h>

#include "csr.hpp"
#include "group.hpp"

namespace airg {

// ------------------------------------------------------------ validation --
enum : uint32_t { BAD_COL = 1, NO_DIAG = 2, ZERO_DIAG = 4, NONFINITE = 8, BAD_RP = 16 };

// One G-lane group per row: every lane checks its entries; the kept count
// and the diagonal's presence are combined over the group.
template <int G>
__global__ void __launch_bounds__(256) k_validate(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  int32_t *__restrict__ keep, uint32_t *__restrict__ flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / G);
    const int lane = group_lane<G>();
    if (i >= n) return;
    uint32_t f = 0;
    const int32_t b = rp[i], e = rp[i + 1];
    const bool bad_rp = e < b || b < 0 || (int64_t)e > nnz;
    int32_t cnt = 0;
    bool diag = false;
    if (bad_rp) {
        f |= BAD_RP;
    } else {
        for (int32_t k = b + lane; k < e; k += G) {
            int32_t j = ci[k];
            double a = v[k];
            if (j < 0 || j >= n || (k > b && j <= ci[k - 1])) f |= BAD_COL;
            if (!isfinite(a)) f |= NONFINITE;
            if (j == i) {
                diag = true;
                if (a == 0.0) f |= ZERO_DIAG;
            }
            cnt += (j == i || a != 0.0);
        }
    }
    cnt = group_sum<G>(cnt);
    diag = group_any<G>(diag);
    if (lane == 0) {
        keep[i] = cnt;
        if (!bad_rp && !diag) f |= NO_DIAG;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_canonical_fill(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, const int32_t *__restrict__ orp,
                                 int32_t *__restrict__ oci, double *__restrict__ ov) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t w = orp[i];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (ci[k] == i || v[k] != 0.0) {
            oci[w] = ci[k];
            ov[w] = v[k];
            ++w;
        }
    }
}

Csr canonical_copy(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, hipStream_t s) {
    AIRG_REQUIRE(n > 0, ST_INVALID_ARG, "matrix must have at least one row");
    AIRG_REQUIRE(nnz >= n && nnz < ((int64_t)1 << 31), ST_INVALID_ARG, "nnz out of range");
    int32_t ends[2] = {-1, -1};
    read_ints({rp, rp + n}, {1, 1}, ends, s);
    AIRG_REQUIRE(ends[0] == 0 && (int64_t)ends[1] == nnz, ST_BAD_CSR, "row pointers must start at 0 and end at nnz");
    DBuf<int32_t> keep((size_t)n, s);
    DBuf<uint32_t> flags(1, s);
    fill_zero(flags.p, 4, s);
    dispatch_group(lanes_for(nnz, n), [&]<int G>() {
        k_validate<G><<<grid_for((int64_t)n * G, 256), 256, 0, s>>>(n, nnz, rp, ci, v, keep.p, flags.p);
    });
    AIRG_LAUNCH_CHECK();
    Csr A;
    A.nr = A.nc = n;
    A.rp.alloc((size_t)n + 1, s);
    exclusive_scan(keep.p, A.rp.p, n, s, false);
    // the flags and the kept count in one readback
    int32_t fk[2];
    read_ints({reinterpret_cast<const int32_t *>(flags.p), A.rp.p + n}, {1, 1}, fk, s);
    const uint32_t f = (uint32_t)fk[0];
    AIRG_REQUIRE(!(f & (BAD_RP | BAD_COL)), ST_BAD_CSR, "columns must be in range and strictly ascending per row");
    AIRG_REQUIRE(!(f & NONFINITE), ST_NONFINITE, "matrix has a non-finite value");
    AIRG_REQUIRE(!(f & NO_DIAG), ST_BAD_CSR, "every row must store its diagonal");
    AIRG_REQUIRE(!(f & ZERO_DIAG), ST_ZERO_DIAG, "matrix has a zero diagonal entry");
    const int64_t kept = fk[1];
    A.nnz = kept;
    A.ci.alloc((size_t)kept, s);
    A.v.alloc((size_t)kept, s);
    if (kept == nnz) {
        const CopyReq req[2] = {{A.ci.p, ci, (size_t)nnz * sizeof(int32_t)}, {A.v.p, v, (size_t)nnz * sizeof(double)}};
        copy_many(req, 2, s);
    } else {
        k_canonical_fill<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, v, A.rp.p, A.ci.p, A.v.p);
        AIRG_LAUNCH_CHECK();
    }
    return A;
}

Csr copy_csr(const CsrView &A, hipStream_t s) {
    Csr B;
    B.alloc(A.nr, A.nc, A.nnz, s);
    const CopyReq req[3] = {{B.rp.p, A.rp, ((size_t)A.nr + 1) * sizeof(int32_t)},
                            {B.ci.p, A.ci, (size_t)A.nnz * sizeof(int32_t)},
                            {B.v.p, A.v, (size_t)A.nnz * sizeof(double)}};
    copy_many(req, 3, s);
    return B;
}

// ------------------------------------------------------------------ SpMV ---
// G lanes per row; a wavefront covers 64/G consecutive rows so its loads of
// columns and values stay within a contiguous stretch of the arrays.
template <int G, class VT, class XT, int MODE, int TAG = 0>
__global__ void __launch_bounds__(256) k_spmv(int32_t nr, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci, const VT *__restrict__ v,
                                              const XT *__restrict__ x, XT *y, const XT *z) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= nr) return;  // uniform across the group
    int32_t b = rp[row], e = rp[row + 1];
    XT acc = 0;
    for (int32_t k = b + lane; k < e; k += G) acc += (XT)v[k] * x[ci[k]];
    acc = group_sum<G>(acc);
    if (lane == 0) {
        if (MODE == SPMV_SET) y[row] = acc;
        else if (MODE == SPMV_ZMINUS) y[row] = z[row] - acc;
        else y[row] = y[row] + acc;
    }
}

// Rows of up to ~16 entries: CSR-stream.  A workgroup owns kStreamRows
// consecutive rows; its threads stream the rows' nonzeros (values, columns)
// coalesced in chunks of kStreamChunk, park the products in LDS, and then each
// thread sums its own row from LDS in ascending order.  Each thread issues
// all of its column and value loads of a chunk before any gather of x, so a
// chunk costs two dependent trips to memory rather than two per entry.
constexpr int kStreamRows = 256;
constexpr int kStreamChunk = 1536;
constexpr int kStreamUnroll = kStreamChunk / kStreamRows;
constexpr int32_t kStreamMinRows = 32768;   // below this the lane-group kernel has less latency

template <class VT, class XT, int MODE, int TAG>
__global__ void __launch_bounds__(kStreamRows) k_spmv_stream(int32_t nr, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const VT *__restrict__ v, const XT *__restrict__ x,
                                                            XT *y, const XT *z) {
    __shared__ XT prod[kStreamChunk];
    int32_t tile = xcd_tile(blockIdx.x);
    int32_t r0 = tile * kStreamRows;
    if (r0 >= nr) return;
    int32_t r1 = r0 + kStreamRows < nr ? r0 + kStreamRows : nr;
    int32_t row = r0 + threadIdx.x;
    int32_t base = rp[r0], end = rp[r1];
    int32_t mb = 0, me = 0;
    if (row < r1) {
        mb = rp[row];
        me = rp[row + 1];
    }
    XT acc = 0;
    for (int32_t c0 = base; c0 < end; c0 += kStreamChunk) {
        int32_t c1 = c0 + kStreamChunk < end ? c0 + kStreamChunk : end;
        int32_t cc[kStreamUnroll];
        XT vv[kStreamUnroll], xx[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            int32_t k = c0 + u * kStreamRows + threadIdx.x;
            cc[u] = 0;
            vv[u] = 0;
            if (k < c1) {
                cc[u] = __builtin_nontemporal_load(ci + k);   // streamed once: keep L2 for the x gathers
                vv[u] = (XT)__builtin_nontemporal_load(v + k);
            }
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) xx[u] = c0 + u * kStreamRows + (int32_t)threadIdx.x < c1 ? x[cc[u]] : 0;
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            int32_t k = c0 + u * kStreamRows + threadIdx.x;
            if (k < c1) prod[k - c0] = vv[u] * xx[u];
        }
        __syncthreads();
        int32_t lo = mb > c0 ? mb : c0, hi = me < c1 ? me : c1;
        for (int32_t k = lo; k < hi; ++k) acc += prod[k - c0];
        __syncthreads();
    }
    if (row < r1) {
        if (MODE == SPMV_SET) y[row] = acc;
        else if (MODE == SPMV_ZMINUS) y[row] = z[row] - acc;
        else y[row] = y[row] + acc;
    }
}

// Whether spmv_t takes the CSR-stream kernel for this shape.
bool spmv_streams(int32_t nr, int64_t nnz) {
    return nr >= kStreamMinRows && (double)nnz <= 16.0 * (double)nr;
}

// e0/e1 (timed launches): events stamped by the kernel dispatch itself at
// the kernel's start and end, so their interval is the kernel's own duration.
template <int TAG, class VT, class XT>
static void spmv_t(int32_t nr, int64_t nnz, const int32_t *rp, const int32_t *ci, const VT *v, const XT *x, XT *y,
                   const XT *z, int mode, hipStream_t s, int lanes, hipEvent_t e0 = nullptr,
                   hipEvent_t e1 = nullptr) {
    if (nr == 0) return;
    auto launch = [&](auto kern, unsigned grid) {
        if (e0) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, e0, e1, 0, nr, rp, ci, v, x, y, z);
        else kern<<<grid, 256, 0, s>>>(nr, rp, ci, v, x, y, z);
    };
    if (lanes == 0 && spmv_streams(nr, nnz)) {
        static_assert(kStreamRows == 256, "stream SpMV launches 256-thread workgroups");
        unsigned grid = grid_for(xcd_grid((nr + kStreamRows - 1) / kStreamRows), 1);
        if (mode == SPMV_SET) launch(k_spmv_stream<VT, XT, SPMV_SET, TAG>, grid);
        else if (mode == SPMV_ZMINUS) launch(k_spmv_stream<VT, XT, SPMV_ZMINUS, TAG>, grid);
        else launch(k_spmv_stream<VT, XT, SPMV_ADD, TAG>, grid);
        AIRG_LAUNCH_CHECK();
        return;
    }
    int g = lanes > 0 ? lanes : lanes_for(nnz, nr);
    dispatch_group(g, [&]<int G>() {
        unsigned grid = grid_for((int64_t)nr * G, 256);
        if (mode == SPMV_SET) launch(k_spmv<G, VT, XT, SPMV_SET, TAG>, grid);
        else if (mode == SPMV_ZMINUS) launch(k_spmv<G, VT, XT, SPMV_ZMINUS, TAG>, grid);
        else launch(k_spmv<G, VT, XT, SPMV_ADD, TAG>, grid);
    });
    AIRG_LAUNCH_CHECK();
}

void spmv(const CsrView &A, const double *x, double *y, const double *z, int mode, hipStream_t s, int lanes) {
    spmv_t<0, double, double>(A.nr, A.nnz, A.rp, A.ci, A.v, x, y, z, mode, s, lanes);
}
void spmv32(const CsrView &A, const float *x, float *y, const float *z, int mode, hipStream_t s, int lanes) {
    AIRG_REQUIRE(A.vf != nullptr, ST_INVALID_ARG, "matrix has no single-precision copy");
    spmv_t<0, float, float>(A.nr, A.nnz, A.rp, A.ci, A.vf, x, y, z, mode, s, lanes);
}

// ------------------------------------------------------ top-operator SpMV ---
// The outer iterations' products with the finest operator run as their own
// kernel instantiation (TAG 1) so that they can be timed and profiled apart
// from the V-cycle's SpMVs; while timing is on, each plain product launch
// (y = A x, the FGMRES Arnoldi product) is bracketed by events on its stream
// and its algorithmic bytes are accounted.
namespace {
struct TopClock {
    std::mutex mu;
    bool on = false;
    std::vector<std::tuple<hipEvent_t, hipEvent_t, double>> spans;
} g_top;
}  // namespace

void top_timing(bool enable) {
    std::lock_guard<std::mutex> lk(g_top.mu);
    for (auto &t : g_top.spans) {
        (void)hipEventDestroy(std::get<0>(t));
        (void)hipEventDestroy(std::get<1>(t));
    }
    g_top.spans.clear();
    g_top.on = enable;
}

void top_timing_read(int64_t *launches, double *bytes, double *seconds) {
    std::lock_guard<std::mutex> lk(g_top.mu);
    double b = 0.0, t = 0.0;
    for (auto &sp : g_top.spans) {
        AIRG_HIP(hipEventSynchronize(std::get<1>(sp)));
        float ms = 0.f;
        AIRG_HIP(hipEventElapsedTime(&ms, std::get<0>(sp), std::get<1>(sp)));
        t += ms * 1e-3;
        b += std::get<2>(sp);
    }
    *launches = (int64_t)g_top.spans.size();
    *bytes = b;
    *seconds = t;
}

void spmv_top(const CsrView &A, const double *x, double *y, const double *z, int mode, hipStream_t s) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_top.mu);
        on = g_top.on;
    }
    on = on && mode == SPMV_SET;   // the Arnoldi product; residual launches are a different kernel
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (on) {
        AIRG_HIP(hipEventCreate(&e0));
        AIRG_HIP(hipEventCreate(&e1));
    }
    spmv_t<1, double, double>(A.nr, A.nnz, A.rp, A.ci, A.v, x, y, z, mode, s, 0, e0, e1);
    if (on) {
        double bytes = (double)A.nnz * 12.0 + 4.0 * (A.nr + 1) + 8.0 * (A.nc + A.nr + (mode != SPMV_SET ? A.nr : 0));
        std::lock_guard<std::mutex> lk(g_top.mu);
        g_top.spans.emplace_back(e0, e1, bytes);
    }
}

// k right-hand sides, row-major: one group per row, each lane keeps K sums.
template <int G, int K, class VT, class XT, int MODE>
__global__ void __launch_bounds__(256) k_spmm(int32_t nr, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci, const VT *__restrict__ v,
                                              const XT *__restrict__ x, XT *y, const XT *z) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= nr) return;
    XT acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = 0;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) {
        XT a = (XT)v[k];
        const XT *xr = x + (int64_t)ci[k] * K;
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] += a * xr[c];
    }
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = group_sum<G>(acc[c]);
    if (lane == 0) {
        XT *yr = y + (int64_t)row * K;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            if (MODE == SPMV_SET) yr[c] = acc[c];
            else if (MODE == SPMV_ZMINUS) yr[c] = z[(int64_t)row * K + c] - acc[c];
            else yr[c] = yr[c] + acc[c];
        }
    }
}

// CSR-stream for K right-hand sides (row-major n x K): the workgroup parks
// the K products of each nonzero in LDS.  Persistent: the launch walks the
// tiles in xcd_tile order, gridDim.x (a multiple of the XCD count) apart, so
// each workgroup stays on the tiles of its own XCD.
template <int K, class VT, class XT, int MODE, int TAG = 0>
__global__ void __launch_bounds__(kStreamRows) k_spmm_stream(int32_t nr, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const VT *__restrict__ v, const XT *__restrict__ x,
                                                            XT *y, const XT *z) {
    constexpr int CH = 2048 / K;
    constexpr int U = (CH + kStreamRows - 1) / kStreamRows;
    __shared__ XT prod[CH * K];
    int32_t ntiles = (nr + kStreamRows - 1) / kStreamRows;
    int32_t nid = (int32_t)xcd_grid(ntiles);
    for (int32_t id = blockIdx.x; id < nid; id += gridDim.x) {
        int32_t r0 = xcd_tile(id) * kStreamRows;
        if (r0 >= nr) continue;   // uniform across the workgroup
        int32_t r1 = r0 + kStreamRows < nr ? r0 + kStreamRows : nr;
        int32_t row = r0 + threadIdx.x;
        int32_t base = rp[r0], end = rp[r1];
        int32_t mb = 0, me = 0;
        if (row < r1) {
            mb = rp[row];
            me = rp[row + 1];
        }
        XT acc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = 0;
        for (int32_t c0 = base; c0 < end; c0 += CH) {
            int32_t c1 = c0 + CH < end ? c0 + CH : end;
            int32_t cc[U];
            XT vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int32_t k = c0 + u * kStreamRows + threadIdx.x;
                cc[u] = 0;
                vv[u] = 0;
                if (k < c1 && u * kStreamRows + (int)threadIdx.x < CH) {
                    cc[u] = ci[k];
                    vv[u] = (XT)v[k];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int32_t k = c0 + u * kStreamRows + threadIdx.x;
                if (k < c1 && u * kStreamRows + (int)threadIdx.x < CH) {
                    const XT *xr = x + (int64_t)cc[u] * K;
#pragma unroll
                    for (int c = 0; c < K; ++c) prod[(k - c0) * K + c] = vv[u] * xr[c];
                }
            }
            __syncthreads();
            int32_t lo = mb > c0 ? mb : c0, hi = me < c1 ? me : c1;
            for (int32_t k = lo; k < hi; ++k) {
#pragma unroll
                for (int c = 0; c < K; ++c) acc[c] += prod[(k - c0) * K + c];
            }
            __syncthreads();
        }
        if (row < r1) {
            XT *yr = y + (int64_t)row * K;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                if (MODE == SPMV_SET) yr[c] = acc[c];
                else if (MODE == SPMV_ZMINUS) yr[c] = z[(int64_t)row * K + c] - acc[c];
                else yr[c] = yr[c] + acc[c];
            }
        }
    }
}

// Persistent grid size: enough workgroups to fill the chip a few times over,
// a multiple of the XCD count, never more than there are tile ids.
static unsigned persistent_grid(int32_t nr) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    int64_t ids = xcd_grid(((int64_t)nr + kStreamRows - 1) / kStreamRows);
    int64_t cap = std::max<int64_t>(kXcds, (int64_t)cus * 8 / kXcds * kXcds);
    return (unsigned)std::min(ids, cap);
}

// TAG 1: the batched outer product with the finest operators (timed apart);
// e0/e1 as in spmv_t.
template <int K, class VT, class XT, int TAG = 0>
static void spmm_k(const CsrView &A, const VT *v, const XT *x, XT *y, const XT *z, int mode, hipStream_t s,
                   int lanes = -1, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (lanes == 0 || (lanes < 0 && A.nr >= kStreamMinRows && (double)A.nnz <= 16.0 * (double)A.nr)) {
        unsigned grid = persistent_grid(A.nr);
        auto launch = [&](auto kern) {
            if (e0) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kStreamRows), 0, s, e0, e1, 0, A.nr, A.rp, A.ci, v, x,
                                          y, z);
            else kern<<<grid, kStreamRows, 0, s>>>(A.nr, A.rp, A.ci, v, x, y, z);
        };
        if (mode == SPMV_SET) launch(k_spmm_stream<K, VT, XT, SPMV_SET, TAG>);
        else if (mode == SPMV_ZMINUS) launch(k_spmm_stream<K, VT, XT, SPMV_ZMINUS, TAG>);
        else launch(k_spmm_stream<K, VT, XT, SPMV_ADD, TAG>);
        AIRG_LAUNCH_CHECK();
        return;
    }
    AIRG_REQUIRE(e0 == nullptr, ST_INVALID_ARG, "timed products take the stream kernel");
    int g = lanes > 0 ? lanes : lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int G>() {
        unsigned grid = grid_for((int64_t)A.nr * G, 256);
        if (mode == SPMV_SET) k_spmm<G, K, VT, XT, SPMV_SET><<<grid, 256, 0, s>>>(A.nr, A.rp, A.ci, v, x, y, z);
        else if (mode == SPMV_ZMINUS)
            k_spmm<G, K, VT, XT, SPMV_ZMINUS><<<grid, 256, 0, s>>>(A.nr, A.rp, A.ci, v, x, y, z);
        else k_spmm<G, K, VT, XT, SPMV_ADD><<<grid, 256, 0, s>>>(A.nr, A.rp, A.ci, v, x, y, z);
    });
    AIRG_LAUNCH_CHECK();
}

template <class VT, class XT>
static void spmm_t(const CsrView &A, const VT *v, int k, const XT *x, XT *y, const XT *z, int mode, hipStream_t s,
                   int lanes) {
    if (A.nr == 0) return;
    switch (k) {
    case 1: spmm_k<1>(A, v, x, y, z, mode, s, lanes); break;
    case 2: spmm_k<2>(A, v, x, y, z, mode, s, lanes); break;
    case 3: spmm_k<3>(A, v, x, y, z, mode, s, lanes); break;
    case 4: spmm_k<4>(A, v, x, y, z, mode, s, lanes); break;
    case 8: spmm_k<8>(A, v, x, y, z, mode, s, lanes); break;
    default: throw Error(ST_INVALID_ARG, "number of right-hand sides must be 1, 2, 3, 4 or 8");
    }
}

void spmm(const CsrView &A, int k, const double *x, double *y, const double *z, int mode, hipStream_t s, int lanes) {
    spmm_t<double, double>(A, A.v, k, x, y, z, mode, s, lanes);
}
void spmm32(const CsrView &A, int k, const float *x, float *y, const float *z, int mode, hipStream_t s, int lanes) {
    AIRG_REQUIRE(A.vf != nullptr, ST_INVALID_ARG, "matrix has no single-precision copy");
    spmm_t<float, float>(A, A.vf, k, x, y, z, mode, s, lanes);
}

// The batched outer iterations' products with the finest operators: their
// own kernel instantiation (TAG 1), timed like spmv_top while timing is on.
void spmm_top(const CsrView &A, int k, const double *x, double *y, const double *z, int mode, hipStream_t s) {
    if (A.nr == 0) return;
    const bool stream = A.nr >= kStreamMinRows && (double)A.nnz <= 16.0 * (double)A.nr;
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_top.mu);
        on = g_top.on;
    }
    on = on && mode == SPMV_SET && stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (on) {
        AIRG_HIP(hipEventCreate(&e0));
        AIRG_HIP(hipEventCreate(&e1));
    }
    switch (k) {
    case 1: spmm_k<1, double, double, 1>(A, A.v, x, y, z, mode, s, -1, e0, e1); break;
    case 2: spmm_k<2, double, double, 1>(A, A.v, x, y, z, mode, s, -1, e0, e1); break;
    case 3: spmm_k<3, double, double, 1>(A, A.v, x, y, z, mode, s, -1, e0, e1); break;
    case 4: spmm_k<4, double, double, 1>(A, A.v, x, y, z, mode, s, -1, e0, e1); break;
    case 8: spmm_k<8, double, double, 1>(A, A.v, x, y, z, mode, s, -1, e0, e1); break;
    default: throw Error(ST_INVALID_ARG, "number of right-hand sides must be 1, 2, 3, 4 or 8");
    }
    if (on) {
        double bytes = (double)A.nnz * 12.0 + 4.0 * (A.nr + 1) + 8.0 * k * (A.nc + A.nr);
        std::lock_guard<std::mutex> lk(g_top.mu);
        g_top.spans.emplace_back(e0, e1, bytes);
    }
}

// ------------------------------------------------------------- CF ranks ---
__global__ void k_cf_flags(const int8_t *__restrict__ cf, int32_t n, int32_t *__restrict__ fF,
                           int32_t *__restrict__ fC, int32_t *__restrict__ fT) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int8_t c = cf[i];
    fF[i] = c == CF_F;
    fC[i] = c == CF_C;
    fT[i] = c == CF_T;
}
__global__ void k_cf_rank(const int8_t *__restrict__ cf, int32_t n, const int32_t *__restrict__ sF,
                          const int32_t *__restrict__ sC, const int32_t *__restrict__ sT, int32_t *__restrict__ rank,
                          int32_t *__restrict__ tot) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        tot[0] = sF[n];
        tot[1] = sC[n];
        tot[2] = sT[n];
    }
    if (i >= n) return;
    int8_t c = cf[i];
    rank[i] = c == CF_F ? sF[i] : c == CF_C ? sC[i] : sT[i];
}

CfCounts cf_ranks3(const int8_t *cf, int32_t n, int32_t *rank, hipStream_t s,
                   const std::vector<const int32_t *> &extra, int32_t *extra_out, const int32_t *flags3) {
    DBuf<int32_t> fl;
    if (!flags3) {
        fl.alloc((size_t)3 * n, s);
        k_cf_flags<<<grid_for(n, 256), 256, 0, s>>>(cf, n, fl.p, fl.p + n, fl.p + 2 * (size_t)n);
        AIRG_LAUNCH_CHECK();
        flags3 = fl.p;
    }
    DBuf<int32_t> sF((size_t)n + 1, s), sC((size_t)n + 1, s), sT((size_t)n + 1, s), tot(3, s);
    exclusive_scans({flags3, flags3 + n, flags3 + 2 * (size_t)n}, {sF.p, sC.p, sT.p}, {n, n, n}, s);
    k_cf_rank<<<grid_for(n, 256), 256, 0, s>>>(cf, n, sF.p, sC.p, sT.p, rank, tot.p);
    AIRG_LAUNCH_CHECK();
    std::vector<int32_t> h(3 + extra.size());
    if (!extra.empty()) {
        std::vector<const int32_t *> src{tot.p};
        std::vector<int32_t> cnt{3};
        for (const int32_t *e : extra) {
            src.push_back(e);
            cnt.push_back(1);
        }
        read_ints(src, cnt, h.data(), s);
        std::copy(h.begin() + 3, h.end(), extra_out);
    } else {
        d2h(h.data(), tot.p, 3, s);
    }
    return CfCounts{h[0], h[1], h[2]};
}

// out[3 p + {0, 1, 2}] = F, C and terminal rows before row off[p], p = 0..na
__global__ void k_cf_bounds(const int32_t *__restrict__ sF, const int32_t *__restrict__ sC,
                            const int32_t *__restrict__ sT, const int32_t *__restrict__ off, int na,
                            int32_t *__restrict__ out) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > na) return;
    int32_t i = off[p];
    out[3 * p] = sF[i];
    out[3 * p + 1] = sC[i];
    out[3 * p + 2] = sT[i];
}

CfCounts cf_ranks_seg(const int8_t *cf, int32_t n, int32_t *rank, const int32_t *d_off, int na, int32_t *h_bounds,
                      hipStream_t s) {
    DBuf<int32_t> fF((size_t)n, s), fC((size_t)n, s), fT((size_t)n, s);
    DBuf<int32_t> sF((size_t)n + 1, s), sC((size_t)n + 1, s), sT((size_t)n + 1, s), tot(3, s);
    DBuf<int32_t> bnd((size_t)3 * (na + 1), s);
    k_cf_flags<<<grid_for(n, 256), 256, 0, s>>>(cf, n, fF.p, fC.p, fT.p);
    AIRG_LAUNCH_CHECK();
    exclusive_scans({fF.p, fC.p, fT.p}, {sF.p, sC.p, sT.p}, {n, n, n}, s);
    k_cf_rank<<<grid_for(n, 256), 256, 0, s>>>(cf, n, sF.p, sC.p, sT.p, rank, tot.p);
    AIRG_LAUNCH_CHECK();
    k_cf_bounds<<<grid_for(na + 1, 256), 256, 0, s>>>(sF.p, sC.p, sT.p, d_off, na, bnd.p);
    AIRG_LAUNCH_CHECK();
    d2h(h_bounds, bnd.p, (size_t)3 * (na + 1), s);
    return CfCounts{h_bounds[3 * na], h_bounds[3 * na + 1], h_bounds[3 * na + 2]};
}

std::pair<int32_t, int32_t> cf_ranks(const int8_t *cf, int32_t n, int32_t *rank, hipStream_t s) {
    CfCounts c = cf_ranks3(cf, n, rank, s);
    return {c.nF, c.nC};
}

__global__ void k_cf_lists(const int8_t *__restrict__ cf, const int32_t *__restrict__ rank, int32_t n,
                           int32_t *__restrict__ fidx, int32_t *__restrict__ cidx) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == CF_F) {
        if (fidx) fidx[rank[i]] = i;
    } else if (cf[i] == CF_C && cidx) {
        cidx[rank[i]] = i;
    }
}

void cf_index_lists(const int8_t *cf, const int32_t *rank, int32_t n, int32_t *fidx, int32_t *cidx, hipStream_t s) {
    k_cf_lists<<<grid_for(n, 256), 256, 0, s>>>(cf, rank, n, fidx, cidx);
    AIRG_LAUNCH_CHECK();
}

// ------------------------------------------------------------ extraction ---
template <int G>
__global__ void __launch_bounds__(256) k_extract_count(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const int8_t *__restrict__ cf,
                                                       const int32_t *__restrict__ rank, int8_t rowsel,
                                                       int8_t colsel, int32_t *__restrict__ cnt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n || cf[row] != rowsel) return;
    int32_t c = 0;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) c += cf[ci[k]] == colsel;
    c = group_sum<G>(c);
    if (lane == 0) cnt[rank[row]] = c;
}

template <int G>
__global__ void __launch_bounds__(256) k_extract_fill(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                      const int8_t *__restrict__ cf,
                                                      const int32_t *__restrict__ rank, int8_t rowsel, int8_t colsel,
                                                      const int32_t *__restrict__ orp, int32_t *__restrict__ oci,
                                                      double *__restrict__ ov) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n || cf[row] != rowsel) return;
    int32_t w = orp[rank[row]];
    int32_t e = rp[row + 1];
    for (int32_t base = rp[row]; base < e; base += G) {
        int32_t k = base + lane;
        bool keep = false;
        int32_t j = 0;
        if (k < e) {
            j = ci[k];
            keep = cf[j] == colsel;
        }
        int tot;
        int pre = group_prefix<G>(keep, &tot);
        if (keep) {
            oci[w + pre] = rank[j];
            ov[w + pre] = v[k];
        }
        w += tot;
    }
}

// The three blocks of the splitting in one pass: F rows give A_ff and A_fc,
// C rows give A_cf (terminal rows give nothing).  The counts are kept per
// original row (zero where a row gives no entries to a block), so that their
// scans, and the block sizes, need only cf: ranks order the rows of each
// class as the original order does, so row i's offset is its rank's.
template <int G>
__global__ void __launch_bounds__(256) k_extract3_count(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci, const int8_t *__restrict__ cf,
                                                        int32_t *__restrict__ cff, int32_t *__restrict__ cfc,
                                                        int32_t *__restrict__ ccf) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    const int8_t me = cf[row];
    int32_t nf = 0, nc = 0;
    if (me == CF_F || me == CF_C) {
        for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) {
            int8_t c = cf[ci[k]];
            nf += c == CF_F;
            nc += c == CF_C;
        }
        nf = group_sum<G>(nf);
        nc = group_sum<G>(nc);
    }
    if (lane == 0) {
        cff[row] = me == CF_F ? nf : 0;
        cfc[row] = me == CF_F ? nc : 0;
        ccf[row] = me == CF_C ? nf : 0;
    }
}

// off: the three scans of the counts (n + 1 entries each: A_ff, A_fc, A_cf);
// each row also writes its block row pointers (thread 0 their ends) and,
// when fidx / cidx are given, its entry in the F or C index list.
template <int G>
__global__ void __launch_bounds__(256) k_extract3_fill(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                       const int8_t *__restrict__ cf, const int32_t *__restrict__ rank,
                                                       const int32_t *__restrict__ off, int32_t nF, int32_t nC,
                                                       int32_t *__restrict__ ffrp, int32_t *__restrict__ ffci,
                                                       double *__restrict__ ffv, int32_t *__restrict__ fcrp,
                                                       int32_t *__restrict__ fcci, double *__restrict__ fcv,
                                                       int32_t *__restrict__ cfrp, int32_t *__restrict__ cfci,
                                                       double *__restrict__ cfv, int32_t *__restrict__ fidx,
                                                       int32_t *__restrict__ cidx) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    const int64_t n1 = (int64_t)n + 1;
    if (t == 0) {
        ffrp[nF] = off[n];
        fcrp[nF] = off[n1 + n];
        cfrp[nC] = off[2 * n1 + n];
    }
    if (row >= n) return;
    int8_t me = cf[row];
    if (me != CF_F && me != CF_C) return;
    const bool frow = me == CF_F;
    const int32_t r = rank[row];
    int32_t wf = frow ? off[row] : off[2 * n1 + row];
    int32_t wc = frow ? off[n1 + row] : 0;
    if (lane == 0) {
        if (frow) {
            ffrp[r] = wf;
            fcrp[r] = wc;
            if (fidx) fidx[r] = row;
        } else {
            cfrp[r] = wf;
            if (cidx) cidx[r] = row;
        }
    }
    int32_t *oci_f = frow ? ffci : cfci;
    double *ov_f = frow ? ffv : cfv;
    int32_t e = rp[row + 1];
    for (int32_t base = rp[row]; base < e; base += G) {
        int32_t k = base + lane;
        int8_t c = CF_U;
        int32_t j = 0;
        if (k < e) {
            j = ci[k];
            c = cf[j];
        }
        int tf, tc;
        int pf = group_prefix<G>(c == CF_F, &tf);
        int pc = group_prefix<G>(frow && c == CF_C, &tc);
        if (c == CF_F) {
            oci_f[wf + pf] = rank[j];
            ov_f[wf + pf] = v[k];
        } else if (frow && c == CF_C) {
            fcci[wc + pc] = rank[j];
            fcv[wc + pc] = v[k];
        }
        wf += tf;
        wc += tc;
    }
}

ExtractPlan extract_begin(const CsrView &A, const int8_t *cf, hipStream_t s) {
    ExtractPlan P;
    const int32_t n = A.nr;
    P.n = n;
    P.off.alloc((size_t)3 * ((size_t)n + 1), s);
    DBuf<int32_t> cnt((size_t)3 * std::max<int32_t>(n, 1), s);
    int32_t *off = P.off.p;
    if (n > 0) {
        dispatch_group(lanes_for(A.nnz, n), [&]<int G>() {
            k_extract3_count<G><<<grid_for((int64_t)n * G, 256), 256, 0, s>>>(n, A.rp, A.ci, cf, cnt.p, cnt.p + n,
                                                                              cnt.p + 2 * (size_t)n);
        });
        AIRG_LAUNCH_CHECK();
    }
    exclusive_scans({cnt.p, cnt.p + n, cnt.p + 2 * (size_t)n}, {off, off + (n + 1), off + 2 * ((size_t)n + 1)},
                    {n, n, n}, s);
    return P;
}

std::vector<const int32_t *> ExtractPlan::totals() const {
    const size_t n1 = (size_t)n + 1;
    return {off.p + n, off.p + n1 + n, off.p + 2 * n1 + n};
}

void extract_finish(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                    const int32_t *tot, ExtractPlan &P, Csr &Aff, Csr &Afc, Csr &Acf, hipStream_t s, int32_t *fidx,
                    int32_t *cidx) {
    AIRG_REQUIRE(P.n == A.nr, ST_INVALID_ARG, "extraction plan does not match");
    for (int k = 0; k < 3; ++k) AIRG_REQUIRE(tot[k] >= 0, ST_LIMIT, "prefix sum exceeds the int32 index range");
    Aff.alloc(nF, nF, tot[0], s);
    Afc.alloc(nF, nC, tot[1], s);
    Acf.alloc(nC, nF, tot[2], s);
    if (A.nr == 0) return;
    dispatch_group(lanes_for(A.nnz, A.nr), [&]<int G>() {
        k_extract3_fill<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(
            A.nr, A.rp, A.ci, A.v, cf, rank, P.off.p, nF, nC, Aff.rp.p, Aff.ci.p, Aff.v.p, Afc.rp.p, Afc.ci.p,
            Afc.v.p, Acf.rp.p, Acf.ci.p, Acf.v.p, fidx, cidx);
    });
    AIRG_LAUNCH_CHECK();
}

void extract_refill(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC,
                    const ExtractPlan &P, Csr &Aff, Csr &Afc, Csr &Acf, hipStream_t s) {
    AIRG_REQUIRE(P.n == A.nr && Aff.nr == nF && Acf.nr == nC, ST_INVALID_ARG, "extraction plan does not match");
    if (A.nr == 0) return;
    dispatch_group(lanes_for(A.nnz, A.nr), [&]<int G>() {
        k_extract3_fill<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(
            A.nr, A.rp, A.ci, A.v, cf, rank, P.off.p, nF, nC, Aff.rp.p, Aff.ci.p, Aff.v.p, Afc.rp.p, Afc.ci.p,
            Afc.v.p, Acf.rp.p, Acf.ci.p, Acf.v.p, nullptr, nullptr);
    });
    AIRG_LAUNCH_CHECK();
}

void extract_fc_blocks(const CsrView &A, const int8_t *cf, const int32_t *rank, int32_t nF, int32_t nC, Csr &Aff,
                       Csr &Afc, Csr &Acf, hipStream_t s) {
    ExtractPlan P = extract_begin(A, cf, s);
    int32_t tot[3];
    read_ints(P.totals(), {1, 1, 1}, tot, s);
    extract_finish(A, cf, rank, nF, nC, tot, P, Aff, Afc, Acf, s);
}

Csr extract_block(const CsrView &A, const int8_t *cf, const int32_t *rank, int8_t rowsel, int8_t colsel,
                  int32_t nrows_out, int32_t ncols_out, hipStream_t s) {
    Csr B;
    B.nr = nrows_out;
    B.nc = ncols_out;
    B.rp.alloc((size_t)nrows_out + 1, s);
    DBuf<int32_t> cnt((size_t)nrows_out + 1, s);
    int g = lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int G>() {
        k_extract_count<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(A.nr, A.rp, A.ci, cf, rank, rowsel,
                                                                            colsel, cnt.p);
    });
    AIRG_LAUNCH_CHECK();
    B.nnz = exclusive_scan(cnt.p, B.rp.p, nrows_out, s);
    B.ci.alloc((size_t)B.nnz, s);
    B.v.alloc((size_t)B.nnz, s);
    dispatch_group(g, [&]<int G>() {
        k_extract_fill<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(
            A.nr, A.rp, A.ci, A.v, cf, rank, rowsel, colsel, B.rp.p, B.ci.p, B.v.p);
    });
    AIRG_LAUNCH_CHECK();
    return B;
}

// ------------------------------------------------------------------ drop ---
template <int G>
__device__ inline double row_absmax(const int32_t *rp, const double *v, int32_t row, int lane) {
    double m = 0.0;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) m = fmax(m, fabs(v[k]));
    return group_max<G>(m);
}

template <int G>
__global__ void __launch_bounds__(256) k_drop_count(int32_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                    double tau, int keep_diag, int32_t *__restrict__ cnt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    double thr = tau * row_absmax<G>(rp, v, row, lane);
    int32_t c = 0;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G)
        c += (keep_diag && ci[k] == row) || fabs(v[k]) >= thr;
    c = group_sum<G>(c);
    if (lane == 0) cnt[row] = c;
}

template <int G>
__global__ void __launch_bounds__(256) k_drop_fill(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   double tau, int keep_diag, double sign,
                                                   const int32_t *__restrict__ orp, int32_t *__restrict__ oci,
                                                   double *__restrict__ ov) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    double thr = tau * row_absmax<G>(rp, v, row, lane);
    int32_t w = orp[row];
    int32_t e = rp[row + 1];
    for (int32_t base = rp[row]; base < e; base += G) {
        int32_t k = base + lane;
        bool keep = false;
        if (k < e) keep = (keep_diag && ci[k] == row) || fabs(v[k]) >= thr;
        int tot;
        int pre = group_prefix<G>(keep, &tot);
        if (keep) {
            oci[w + pre] = ci[k];
            ov[w + pre] = sign * v[k];
        }
        w += tot;
    }
}

static Csr drop_rows_x(const CsrView &A, double tau, bool keep_diag, bool negate, bool bound, hipStream_t s) {
    Csr B;
    B.nr = A.nr;
    B.nc = A.nc;
    B.rp.alloc((size_t)A.nr + 1, s);
    DBuf<int32_t> cnt((size_t)A.nr + 1, s);
    int g = lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int G>() {
        k_drop_count<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(A.nr, A.rp, A.ci, A.v, tau, keep_diag,
                                                                         cnt.p);
    });
    AIRG_LAUNCH_CHECK();
    if (bound) {
        exclusive_scan(cnt.p, B.rp.p, A.nr, s, false);
        B.nnz = A.nnz;
    } else {
        B.nnz = exclusive_scan(cnt.p, B.rp.p, A.nr, s);
    }
    B.ci.alloc((size_t)B.nnz, s);
    B.v.alloc((size_t)B.nnz, s);
    dispatch_group(g, [&]<int G>() {
        k_drop_fill<G><<<grid_for((int64_t)A.nr * G, 256), 256, 0, s>>>(
            A.nr, A.rp, A.ci, A.v, tau, keep_diag, negate ? -1.0 : 1.0, B.rp.p, B.ci.p, B.v.p);
    });
    AIRG_LAUNCH_CHECK();
    return B;
}

Csr drop_rows(const CsrView &A, double tau, bool keep_diag, bool negate, hipStream_t s) {
    return drop_rows_x(A, tau, keep_diag, negate, false, s);
}

Csr drop_rows_bound(const CsrView &A, double tau, bool keep_diag, bool negate, hipStream_t s) {
    return drop_rows_x(A, tau, keep_diag, negate, true, s);
}

// ------------------------------------------------------------- transpose ---
__global__ void k_col_count(int64_t nnz, const int32_t *__restrict__ ci, int32_t *__restrict__ cnt) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[ci[k]], 1);
}
__global__ void k_transpose_fill(int32_t nr, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, const int32_t *__restrict__ trp,
                                 int32_t *__restrict__ cursor, int32_t *__restrict__ tci, double *__restrict__ tv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        int32_t j = ci[k];
        int32_t p = trp[j] + atomicAdd(&cursor[j], 1);
        tci[p] = i;
        tv[p] = v[k];
    }
}
// Insertion sort of each row by column: makes the scatter order irrelevant.
__global__ void k_row_sort(int32_t nr, const int32_t *__restrict__ rp, int32_t *__restrict__ ci,
                           double *__restrict__ v) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    int32_t b = rp[i], e = rp[i + 1];
    for (int32_t k = b + 1; k < e; ++k) {
        int32_t c = ci[k];
        double x = v ? v[k] : 0.0;
        int32_t q = k - 1;
        while (q >= b && ci[q] > c) {
            ci[q + 1] = ci[q];
            if (v) v[q + 1] = v[q];
            --q;
        }
        ci[q + 1] = c;
        if (v) v[q + 1] = x;
    }
}

Csr transpose(const CsrView &A, hipStream_t s) {
    Csr T;
    T.alloc(A.nc, A.nr, A.nnz, s);
    DBuf<int32_t> cnt((size_t)A.nc + 1, s), cursor((size_t)A.nc, s);
    fill_zero(cnt.p, ((size_t)A.nc + 1) * 4, s);
    fill_zero(cursor.p, (size_t)A.nc * 4, s);
    k_col_count<<<grid_for(A.nnz, 256), 256, 0, s>>>(A.nnz, A.ci, cnt.p);
    AIRG_LAUNCH_CHECK();
    exclusive_scan(cnt.p, T.rp.p, A.nc, s, false);
    k_transpose_fill<<<grid_for(A.nr, 256), 256, 0, s>>>(A.nr, A.rp, A.ci, A.v, T.rp.p, cursor.p, T.ci.p, T.v.p);
    AIRG_LAUNCH_CHECK();
    k_row_sort<<<grid_for(A.nc, 256), 256, 0, s>>>(A.nc, T.rp.p, T.ci.p, T.v.p);
    AIRG_LAUNCH_CHECK();
    return T;
}

// ------------------------------------------------------------ elementwise ---
__global__ void k_d2f(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}
__global__ void k_f2d(const float *__restrict__ x, double *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}
void cast_d2f(const double *x, float *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_d2f<<<grid_for(n, 256), 256, 0, s>>>(x, y, n);
    AIRG_LAUNCH_CHECK();
}
void cast_f2d(const float *x, double *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_f2d<<<grid_for(n, 256), 256, 0, s>>>(x, y, n);
    AIRG_LAUNCH_CHECK();
}
// y[i] = (float) x[idx[i]] and y[idx[i]] = (double) x[i]: the casts into and
// out of a level-ordered FP32 cycle from natural-order FP64 vectors.
__global__ void k_gather_d2f(const double *__restrict__ x, const int32_t *__restrict__ idx, float *__restrict__ y,
                             int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[idx[i]];
}
__global__ void k_scatter_f2d(const float *__restrict__ x, const int32_t *__restrict__ idx, double *__restrict__ y,
                              int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[idx[i]] = (double)x[i];
}
void gather_d2f(const double *x, const int32_t *idx, float *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_gather_d2f<<<grid_for(n, 256), 256, 0, s>>>(x, idx, y, n);
    AIRG_LAUNCH_CHECK();
}
void scatter_f2d(const float *x, const int32_t *idx, double *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_scatter_f2d<<<grid_for(n, 256), 256, 0, s>>>(x, idx, y, n);
    AIRG_LAUNCH_CHECK();
}
void make_f32(Csr &A, hipStream_t s) {
    A.vf.alloc((size_t)A.nnz, s);
    cast_d2f(A.v.p, A.vf.p, A.nnz, s);
}

__global__ void k_axpy(double a, const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}
__global__ void k_scal_copy(double a, const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}
void axpy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_axpy<<<grid_for(n, 256), 256, 0, s>>>(a, x, y, n);
    AIRG_LAUNCH_CHECK();
}
void scal_copy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_scal_copy<<<grid_for(n, 256), 256, 0, s>>>(a, x, y, n);
    AIRG_LAUNCH_CHECK();
}

__global__ void k_gather(const double *__restrict__ x, const int32_t *__restrict__ idx, double *__restrict__ y,
                         int64_t n, int k, int64_t ldx, int64_t ldy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t src = idx[i];
    for (int c = 0; c < k; ++c) y[i * ldy + c] = x[src * ldx + c];
}
__global__ void k_scatter(const double *__restrict__ x, const int32_t *__restrict__ idx, double *__restrict__ y,
                          int64_t n, int k, int64_t ldx, int64_t ldy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t dst = idx[i];
    for (int c = 0; c < k; ++c) y[dst * ldy + c] = x[i * ldx + c];
}
void gather(const double *x, const int32_t *idx, double *y, int64_t n, hipStream_t s) {
    gather_k(x, idx, y, n, 1, 1, 1, s);
}
void scatter(const double *x, const int32_t *idx, double *y, int64_t n, hipStream_t s) {
    scatter_k(x, idx, y, n, 1, 1, 1, s);
}
void gather_k(const double *x, const int32_t *idx, double *y, int64_t n, int k, int64_t ldx, int64_t ldy,
              hipStream_t s) {
    if (n <= 0) return;
    k_gather<<<grid_for(n, 256), 256, 0, s>>>(x, idx, y, n, k, ldx, ldy);
    AIRG_LAUNCH_CHECK();
}
void scatter_k(const double *x, const int32_t *idx, double *y, int64_t n, int k, int64_t ldx, int64_t ldy,
               hipStream_t s) {
    if (n <= 0) return;
    k_scatter<<<grid_for(n, 256), 256, 0, s>>>(x, idx, y, n, k, ldx, ldy);
    AIRG_LAUNCH_CHECK();
}

// ------------------------------------------------------------ reductions ---
// Fixed grid (depends only on n) and fixed in-block tree: bitwise
// reproducible for a given n.
constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 1024;

__device__ inline double block_sum(double v) {
    __shared__ double part[kRedThreads / kWave];
    v = group_sum<kWave>(v);
    int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / kWave; ++w) t += part[w];
    __syncthreads();
    return t;
}

static int red_blocks(int64_t n) {
    int64_t b = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kRedMaxBlocks));
}

// partial[j * nb + b] = block b's share of dot(V_j, w) for j < nvec.
__global__ void __launch_bounds__(kRedThreads) k_multi_dot(const double *__restrict__ V, int64_t ldv, int nvec,
                                                           const double *__restrict__ w, int64_t n,
                                                           double *__restrict__ partial) {
    int nb = gridDim.x;
    for (int j = 0; j < nvec; ++j) {
        const double *vj = V + (int64_t)j * ldv;
        double s = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)nb * kRedThreads)
            s += vj[i] * w[i];
        s = block_sum(s);
        if (threadIdx.x == 0) partial[(int64_t)j * nb + blockIdx.x] = s;
    }
}
__global__ void k_finish_dots(const double *__restrict__ partial, int nb, int nvec, double *__restrict__ out) {
    int j = blockIdx.x;
    if (j >= nvec) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partial[(int64_t)j * nb + b];
    s = block_sum(s);
    if (threadIdx.x == 0) out[j] = s;
}

// Gram-Schmidt pass fused with the next one's products: w -= V h, then
// out[j] = dot(V_j, w) on the updated w, or (NORM) out[0] = dot(w, w).  V is
// read once for both; the entries are visited as in k_multi_dot (the same
// per-thread order and block tree; k_finish_dots adds the block partials), so
// the sums are those of a separate update and product.  NV >= nvec bounds the unrolled vector loops: each thread keeps
// the NV entries of a row of V in registers, two rows of the stride in flight.
template <int NV, bool NORM>
__global__ void __launch_bounds__(kRedThreads) k_gemv_fused(const double *__restrict__ V, int64_t ldv, int nvec,
                                                            const double *__restrict__ h, double *__restrict__ w,
                                                            int64_t n, double *__restrict__ partial) {
    constexpr int NA = NORM ? 1 : NV;
    const int nb = gridDim.x;
    const int64_t step = (int64_t)nb * kRedThreads;
    double hh[NV], acc[NA];
#pragma unroll
    for (int j = 0; j < NV; ++j) hh[j] = j < nvec ? h[j] : 0.0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = 0.0;
    auto row = [&](int64_t i, const double (&v)[NV]) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < nvec) s += v[j] * hh[j];
        const double wi = w[i] + -1.0 * s;
        w[i] = wi;
        if constexpr (NORM) {
            acc[0] += wi * wi;
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < nvec) acc[j] += v[j] * wi;
        }
    };
    int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    for (; i + step < n; i += 2 * step) {
        double a[NV], b[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            a[j] = j < nvec ? V[(int64_t)j * ldv + i] : 0.0;
            b[j] = j < nvec ? V[(int64_t)j * ldv + i + step] : 0.0;
        }
        row(i, a);
        row(i + step, b);
    }
    if (i < n) {
        double a[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) a[j] = j < nvec ? V[(int64_t)j * ldv + i] : 0.0;
        row(i, a);
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        if (j < (NORM ? 1 : nvec)) {
            const double t = block_sum(acc[j]);
            if (threadIdx.x == 0) partial[(int64_t)j * nb + blockIdx.x] = t;
        }
    }
}

constexpr int kMaxGsVectors = 32;
template <bool NORM>
static void gemv_fused(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n,
                       double *d_out, hipStream_t s) {
    AIRG_REQUIRE(nvec >= 1 && nvec <= kMaxGsVectors, ST_INVALID_ARG, "too many basis vectors");
    const int nb = red_blocks(n);
    const int nd = NORM ? 1 : nvec;
    DBuf<double> part((size_t)nb * nd, s);
    auto go = [&](auto kern) { kern<<<nb, kRedThreads, 0, s>>>(V, ldv, nvec, h_dev, w, n, part.p); };
    if (nvec <= 4) go(k_gemv_fused<4, NORM>);
    else if (nvec <= 8) go(k_gemv_fused<8, NORM>);
    else if (nvec <= 16) go(k_gemv_fused<16, NORM>);
    else go(k_gemv_fused<32, NORM>);
    AIRG_LAUNCH_CHECK();
    k_finish_dots<<<nd, kRedThreads, 0, s>>>(part.p, nb, nd, d_out);
    AIRG_LAUNCH_CHECK();
}

void multi_dot_dev(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *d_out,
                   hipStream_t s) {
    int nb = red_blocks(n);
    DBuf<double> part((size_t)nb * nvec, s);
    k_multi_dot<<<nb, kRedThreads, 0, s>>>(V, ldv, nvec, w, n, part.p);
    AIRG_LAUNCH_CHECK();
    k_finish_dots<<<nvec, kRedThreads, 0, s>>>(part.p, nb, nvec, d_out);
    AIRG_LAUNCH_CHECK();
}

void gemv_sub_dots(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, double *d_out,
                   hipStream_t s) {
    gemv_fused<false>(V, ldv, nvec, h_dev, w, n, d_out, s);
}

void gemv_sub_norm(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, double *d_nn,
                   hipStream_t s) {
    gemv_fused<true>(V, ldv, nvec, h_dev, w, n, d_nn, s);
}

void multi_dot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *h_out, hipStream_t s) {
    DBuf<double> out((size_t)nvec, s);
    multi_dot_dev(V, ldv, nvec, w, n, out.p, s);
    d2h(h_out, out.p, (size_t)nvec, s);
}

double dot(const double *x, const double *y, int64_t n, hipStream_t s) {
    double r;
    multi_dot(x, n, 1, y, n, &r, s);
    return r;
}

double nrm2(const double *x, int64_t n, hipStream_t s) { return std::sqrt(dot(x, x, n, s)); }

__global__ void k_gemv(const double *__restrict__ V, int64_t ldv, int nvec, const double *__restrict__ h,
                       double *__restrict__ w, int64_t n, double sign) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < nvec; ++j) s += V[(int64_t)j * ldv + i] * h[j];
    w[i] += sign * s;
}
// w *= 1 / sqrt(nn[0]) when nn[0] > 0 (the norm squared stays on the device)
__global__ void k_normalize(double *__restrict__ w, const double *__restrict__ nn, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double q = nn[0];
    if (i >= n || !(q > 0.0)) return;
    w[i] = (1.0 / sqrt(q)) * w[i];
}
void normalize_dev(double *w, const double *nn_dev, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_normalize<<<grid_for(n, 256), 256, 0, s>>>(w, nn_dev, n);
    AIRG_LAUNCH_CHECK();
}

void gemv_sub(const double *V, int64_t ldv, int nvec, const double *h_dev, double *w, int64_t n, hipStream_t s) {
    if (n <= 0 || nvec <= 0) return;
    k_gemv<<<grid_for(n, 256), 256, 0, s>>>(V, ldv, nvec, h_dev, w, n, -1.0);
    AIRG_LAUNCH_CHECK();
}
void gemv_add(const double *V, int64_t ldv, int nvec, const double *h_dev, double *x, int64_t n, hipStream_t s) {
    if (n <= 0 || nvec <= 0) return;
    k_gemv<<<grid_for(n, 256), 256, 0, s>>>(V, ldv, nvec, h_dev, x, n, 1.0);
    AIRG_LAUNCH_CHECK();
}

// -------------------------------------------------------------- binning ---
// Row binning.  Rows are listed bin by bin, in ascending row order within a
// bin.  One wavefront takes kBinSpan consecutive rows: pass 1 counts its rows
// per bin, an exclusive scan over the (bin, wavefront) counts gives every
// wavefront its write offset in each bin, and pass 2 places the rows at those
// offsets plus their ballot ranks.
constexpr int kBinItems = 8;                     // rows per lane
constexpr int32_t kBinSpan = 64 * kBinItems;

// The wavefront's rows per bin (b: each lane's bins, -1 past the end).
template <int NB>
__device__ inline void bin_count_store(const int (&b)[kBinItems], int32_t w, int32_t nw, int32_t *__restrict__ bc) {
    const int lane = threadIdx.x;
    int32_t c[NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) {
        c[v] = 0;
#pragma unroll
        for (int u = 0; u < kBinItems; ++u) c[v] += __popcll(__ballot(b[u] == v));
    }
#pragma unroll
    for (int v = 0; v < NB; ++v)
        if (lane == v) bc[(int64_t)v * nw + w] = c[v];
}

template <int NB>
__global__ void __launch_bounds__(64) k_bin_count(const int8_t *__restrict__ bin, int32_t n, int32_t nw,
                                                  int32_t *__restrict__ bc) {
    const int32_t w = blockIdx.x;
    const int32_t r0 = w * kBinSpan;
    int b[kBinItems];
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
        int32_t i = r0 + u * 64 + (int)threadIdx.x;
        b[u] = i < n ? bin[i] : -1;
    }
    bin_count_store<NB>(b, w, nw, bc);
}

template <int NB>
__global__ void __launch_bounds__(64) k_bin_count_rule(const int32_t *__restrict__ val, int diff, BinRule rule,
                                                       int32_t n, int32_t nw, int8_t *__restrict__ bin,
                                                       int32_t *__restrict__ bc) {
    const int32_t w = blockIdx.x;
    const int32_t r0 = w * kBinSpan;
    int b[kBinItems];
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
        int32_t i = r0 + u * 64 + (int)threadIdx.x;
        b[u] = -1;
        if (i < n) {
            const int32_t x = diff ? val[i + 1] - val[i] : val[i];
            int c = 0;
            for (int t = 0; t < rule.nthr; ++t) c += x > rule.thr[t];
            b[u] = c;
            bin[i] = (int8_t)c;
        }
    }
    bin_count_store<NB>(b, w, nw, bc);
}

template <int NB>
__global__ void __launch_bounds__(64) k_bin_scatter(const int8_t *__restrict__ bin, int32_t n, int32_t nw,
                                                    const int32_t *__restrict__ boff, int32_t *__restrict__ rows) {
    const int32_t w = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t r0 = w * kBinSpan;
    const uint64_t below = (1ull << lane) - 1ull;
    int b[kBinItems];
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
        int32_t i = r0 + u * 64 + lane;
        b[u] = i < n ? bin[i] : -1;
    }
    int32_t base[NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) base[v] = boff[(int64_t)v * nw + w];
#pragma unroll
    for (int u = 0; u < kBinItems; ++u) {
        int32_t i = r0 + u * 64 + lane;
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            uint64_t m = __ballot(b[u] == v);
            if (b[u] == v) rows[base[v] + __popcll(m & below)] = i;
            base[v] += __popcll(m);
        }
    }
}

struct RuleSrc {
    const int32_t *val;
    bool diff;
    BinRule rule;
    int8_t *out;
};

template <int NB>
static void bin_begin_t(BinPlan &P, const RuleSrc *src, hipStream_t s) {
    const int64_t m = (int64_t)NB * P.nw;
    DBuf<int32_t> bc((size_t)m + 1, s);
    P.boff.alloc((size_t)m + 1, s);
    P.tot.alloc(NB + 1, s);
    if (src)
        k_bin_count_rule<NB><<<P.nw, 64, 0, s>>>(src->val, src->diff ? 1 : 0, src->rule, P.n, P.nw, src->out, bc.p);
    else
        k_bin_count<NB><<<P.nw, 64, 0, s>>>(P.bin, P.n, P.nw, bc.p);
    AIRG_LAUNCH_CHECK();
    // tot[b] = boff[b * nw]: bin b's first offset; tot[NB] = boff[m], the total
    ScanSample smp;
    smp.out = P.tot.p;
    smp.stride = P.nw;
    smp.count = NB + 1;
    exclusive_scan_sampled(bc.p, P.boff.p, m, smp, s);
}

template <int NB>
static void bin_end_t(BinPlan &P, Bins &B, hipStream_t s) {
    k_bin_scatter<NB><<<P.nw, 64, 0, s>>>(P.bin, P.n, P.nw, P.boff.p, B.rows.p);
    AIRG_LAUNCH_CHECK();
}

template <class F>
static void with_nbins(int nbins, F &&f) {
    switch (nbins) {
    case 6: f.template operator()<6>(); break;
    case 8: f.template operator()<8>(); break;
    case 9: f.template operator()<9>(); break;
    case 10: f.template operator()<10>(); break;
    default: throw Error(ST_INVALID_ARG, "unsupported number of bins");
    }
}

static BinPlan bin_begin(const int8_t *bin, const RuleSrc *src, int32_t n, int nbins, hipStream_t s) {
    BinPlan P;
    P.bin = bin;
    P.n = n;
    P.nbins = nbins;
    P.nw = n > 0 ? (n + kBinSpan - 1) / kBinSpan : 0;
    if (n <= 0) {
        P.tot.alloc((size_t)nbins + 1, s);
        fill_zero(P.tot.p, ((size_t)nbins + 1) * 4, s);
        return P;
    }
    with_nbins(nbins, [&]<int NB>() { bin_begin_t<NB>(P, src, s); });
    return P;
}

BinPlan bin_rows_begin(const int8_t *bin, int32_t n, int nbins, hipStream_t s) {
    return bin_begin(bin, nullptr, n, nbins, s);
}

BinPlan bin_rows_begin_rule(const int32_t *val, bool diff, const BinRule &rule, int8_t *bin_out, int32_t n, int nbins,
                            hipStream_t s) {
    AIRG_REQUIRE(rule.nthr >= 0 && rule.nthr < nbins && rule.nthr <= BinRule::kMax, ST_INVALID_ARG,
                 "bin rule does not match the number of bins");
    const RuleSrc src{val, diff, rule, bin_out};
    return bin_begin(bin_out, &src, n, nbins, s);
}

Bins bin_rows_end(BinPlan &P, const int32_t *h_tot, hipStream_t s) {
    Bins B;
    B.off.assign(P.nbins + 1, 0);
    for (int b = 0; b <= P.nbins; ++b) B.off[b] = h_tot[b];
    B.rows.alloc((size_t)std::max<int32_t>(h_tot[P.nbins], 1), s);
    if (P.n > 0) with_nbins(P.nbins, [&]<int NB>() { bin_end_t<NB>(P, B, s); });
    return B;
}

Bins bin_rows(const int8_t *bin, int32_t n, int nbins, hipStream_t s) {
    BinPlan P = bin_rows_begin(bin, n, nbins, s);
    std::vector<int32_t> h(nbins + 1);
    d2h(h.data(), P.tot.p, h.size(), s);
    return bin_rows_end(P, h.data(), s);
}

}  // namespace airg

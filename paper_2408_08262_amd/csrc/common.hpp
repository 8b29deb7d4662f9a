// Shared infrastructure of the AIRG HIP library: errors, device buffers with
// a stream-keyed caching allocator, CSR containers, launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace airg {

// Status values mirror airg_status in include/airg.h.
enum Status : int {
    ST_OK = 0,
    ST_NOT_CONVERGED = 1,
    ST_INVALID_ARG = -1,
    ST_BAD_CSR = -2,
    ST_ZERO_DIAG = -3,
    ST_NONFINITE = -4,
    ST_OOM = -5,
    ST_HIP = -6,
    ST_STALL = -7,
    ST_LIMIT = -8,
};

struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string &m) : std::runtime_error(m), status(st) {}
};

#define AIRG_HIP(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            throw ::airg::Error(e_ == hipErrorOutOfMemory ? ::airg::ST_OOM : ::airg::ST_HIP,        \
                                std::string(#call) + ": " + hipGetErrorString(e_) + " at " __FILE__ \
                                ":" + std::to_string(__LINE__));                                    \
    } while (0)

#define AIRG_REQUIRE(cond, st, msg)                         \
    do {                                                    \
        if (!(cond)) throw ::airg::Error((st), (msg));      \
    } while (0)

#define AIRG_LAUNCH_CHECK() AIRG_HIP(hipGetLastError())

// ---------------------------------------------------------------- memory --
// Device memory is cached per (stream, size class) so that repeated setups
// and solves do not pay hipMalloc/hipFree; a block is only handed back on the
// stream it was released on, which keeps reuse stream-ordered.
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_release(void *p, hipStream_t s);
void dev_trim();                 // frees every cached block (synchronises the device)
size_t dev_bytes_in_use();
void set_device_cap(int64_t bytes);

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DBuf() = default;
    DBuf(size_t count, hipStream_t st) { alloc(count, st); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept { *this = std::move(o); }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p = o.p; n = o.n; s = o.s;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DBuf() { reset(); }
    void alloc(size_t count, hipStream_t st) {
        reset();
        s = st;
        n = count;
        p = static_cast<T *>(dev_alloc((count ? count : 1) * sizeof(T), st));
    }
    void reset() {
        if (p) dev_release(p, s);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
};

// Device CSR matrix: int32 row pointers and columns (ascending per row).
struct Csr {
    int32_t nr = 0, nc = 0;
    int64_t nnz = 0;
    DBuf<int32_t> rp, ci;
    DBuf<double> v;
    DBuf<float> vf;          // optional single-precision copy of v
    void alloc(int32_t rows, int32_t cols, int64_t nz, hipStream_t s) {
        nr = rows; nc = cols; nnz = nz;
        rp.alloc((size_t)rows + 1, s);
        ci.alloc((size_t)nz, s);
        v.alloc((size_t)nz, s);
    }
    size_t bytes(int vbytes = 8) const { return (size_t)(nr + 1) * 4 + (size_t)nnz * (4 + vbytes); }
};

// Non-owning view of a device CSR.
struct CsrView {
    int32_t nr, nc;
    int64_t nnz;
    const int32_t *rp, *ci;
    const double *v;
    const float *vf;
};
inline CsrView view(const Csr &A) { return {A.nr, A.nc, A.nnz, A.rp.p, A.ci.p, A.v.p, A.vf.p}; }

// Two-phase CSR builds: the row pointers are scanned first; resolve_sizes
// then reads nnz = rp[nr] of every listed matrix with one host
// synchronisation and allocates their columns and values.
void resolve_sizes(const std::vector<Csr *> &ms, hipStream_t s);

// ------------------------------------------------------------- launching --
constexpr int kWave = 64;
inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    AIRG_REQUIRE(g < (int64_t)1 << 31, ST_LIMIT, "grid too large");
    return (unsigned)g;
}

// Workgroups are handed to the chip's 8 XCDs round-robin by id, and each XCD
// has its own L2.  xcd_tile renumbers launch ids so that every XCD receives
// runs of kXcdRun consecutive tiles: neighbouring tiles, whose gathers touch
// the same lines of x, then share one L2.  The launch must cover
// xcd_grid(tiles) ids; ids mapped past the last tile do nothing.
constexpr int kXcds = 8;
constexpr int kXcdRun = 16;
__device__ inline int32_t xcd_tile(int32_t id) {
    int32_t x = id % kXcds, r = id / kXcds;
    return (r / kXcdRun) * (kXcds * kXcdRun) + x * kXcdRun + r % kXcdRun;
}
__host__ __device__ inline int64_t xcd_grid(int64_t tiles) {
    const int64_t g = (int64_t)kXcds * kXcdRun;
    return (tiles + g - 1) / g * g;
}

// Group width (lanes per row) for row-parallel kernels: the largest power of
// two not above the mean row length, between 1 and 64 (rows a little longer
// than the group take a second pass rather than leave most lanes idle).
inline int lanes_for(int64_t nnz, int64_t rows) {
    double avg = rows > 0 ? (double)nnz / (double)rows : 1.0;
    int g = 1;
    while (g < 64 && 2 * g <= avg) g <<= 1;
    return g;
}

// Device-to-host read of `bytes` with one stream synchronisation: small
// word-aligned reads go through pinned host memory that a kernel writes
// directly, larger or unaligned ones through a copy.
void read_bytes(void *h, const void *d, size_t bytes, hipStream_t s);
template <class T>
inline void d2h(T *h, const T *d, size_t count, hipStream_t s) {
    if (!count) return;
    read_bytes(h, d, count * sizeof(T), s);
}
template <class T>
inline T d2h_one(const T *d, hipStream_t s) {
    T h;
    d2h(&h, d, 1, s);
    return h;
}
template <class T>
inline void h2d(T *d, const T *h, size_t count, hipStream_t s) {
    if (!count) return;
    AIRG_HIP(hipMemcpyAsync(d, h, count * sizeof(T), hipMemcpyHostToDevice, s));
}
// Device-to-device copy by a copy kernel (no blit or memset node, so also
// safe inside captured graphs).
void copy_bytes(void *d, const void *src, size_t bytes, hipStream_t s);
// Several device-to-device copies in one launch.
constexpr int kMaxCopies = 4;
struct CopyReq {
    void *dst;
    const void *src;
    size_t bytes;
};
void copy_many(const CopyReq *req, int n, hipStream_t s);
template <class T>
inline void d2d(T *d, const T *src, size_t count, hipStream_t s) {
    copy_bytes(d, src, count * sizeof(T), s);
}
// Timing events of the current device, created once and reused: setups record
// a few hundred per call, and creating and destroying them cost more host
// time than the records.
hipEvent_t pooled_event();
void release_event(hipEvent_t e);
void fill_zero(void *d, size_t bytes, hipStream_t s);
void fill_i32(int32_t *d, int32_t value, size_t count, hipStream_t s);

// Several small device int32 ranges (src[i], counts[i] values each) copied to
// h back to back with one host synchronisation (one gather launch per 16
// ranges, its table in the kernel arguments, writing pinned host memory).
void read_ints(const std::vector<const int32_t *> &src, const std::vector<int32_t> &counts, int32_t *h,
               hipStream_t s);

// --------------------------------------------------------------- scans ----
// out[0..n] = exclusive prefix sum of in[0..n-1]; out[n] = total.  Returns
// the total (synchronising) when want_total is set.
int64_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, bool want_total = true);
// The same scan, also writing smp.out[q] = out[q * smp.stride] for
// q < smp.count (all sampled positions <= n); no synchronisation.
struct ScanSample {
    int32_t *out = nullptr;
    int64_t stride = 1, count = 0;
};
void exclusive_scan_sampled(const int32_t *in, int32_t *out, int64_t n, const ScanSample &smp, hipStream_t s);
// Up to four independent exclusive scans (out[r] of n[r] + 1 entries) in the
// same launches; no synchronisation.
void exclusive_scans(const std::vector<const int32_t *> &in, const std::vector<int32_t *> &out,
                     const std::vector<int64_t> &n, hipStream_t s);

// Counter-based generator shared by the PMISR keys and the Box-Muller rhs:
// the SplitMix64 output function (Steele, Lea & Flood 2014) of a counter
// keyed by (seed, stream, level, index).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t rng_counter(uint64_t seed, uint32_t stream, uint32_t level, uint64_t i) {
    return seed ^ ((uint64_t)(stream & 0xffu) << 56) ^ ((uint64_t)(level & 0xffffu) << 40) ^ i;
}

// Segment of row i given the ascending segment row offsets off[0..nseg]
// (the last p with off[p] <= i).
__host__ __device__ inline int seg_of(const int32_t *off, int nseg, int32_t i) {
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// CF markers; CF_T marks the rows of a batch segment whose hierarchy ends at
// this level (they take neither an F nor a C role).
constexpr int8_t CF_U = 0, CF_F = 1, CF_C = 2, CF_T = 3;

}  // namespace airg

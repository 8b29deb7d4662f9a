// Runtime pieces of the AIRG library: the caching device allocator, fills,
// and the device-wide exclusive scan used to build every CSR row pointer.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace airg {

// ------------------------------------------------------------- allocator --
namespace {
struct Block {
    size_t bytes;
    hipStream_t s;
};
struct Key {
    uintptr_t s;
    size_t bytes;
    bool operator==(const Key &o) const { return s == o.s && bytes == o.bytes; }
};
struct KeyHash {
    size_t operator()(const Key &k) const { return std::hash<uintptr_t>()(k.s) * 31u ^ std::hash<size_t>()(k.bytes); }
};
std::mutex g_mu;
std::unordered_map<Key, std::vector<void *>, KeyHash> g_free;
std::unordered_map<void *, Block> g_live;
size_t g_in_use = 0, g_cached = 0;
int64_t g_cap = 0;

size_t size_class(size_t b) {
    if (b <= 256) return 256;
    size_t p = 256;
    while (p < b && p < ((size_t)1 << 20)) p <<= 1;
    if (p >= b) return p;
    // above 1 MiB: multiples of 1/8 of the power of two below
    size_t q = (size_t)1 << 20;
    while ((q << 1) <= b) q <<= 1;
    size_t step = q >> 3;
    return (b + step - 1) / step * step;
}

void trim_locked() {
    for (auto &kv : g_free)
        for (void *p : kv.second) (void)hipFree(p);
    g_free.clear();
    g_cached = 0;
}
}  // namespace

void set_device_cap(int64_t bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cap = bytes;
}

void *dev_alloc(size_t bytes, hipStream_t s) {
    size_t b = size_class(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    Key k{(uintptr_t)s, b};
    auto it = g_free.find(k);
    void *p = nullptr;
    if (g_cap > 0 && (int64_t)(g_in_use + b) > g_cap)
        throw Error(ST_OOM, "device byte cap exceeded (" + std::to_string(g_in_use + b) + " > " +
                                std::to_string(g_cap) + ")");
    if (it != g_free.end() && !it->second.empty()) {
        p = it->second.back();
        it->second.pop_back();
        g_cached -= b;
    } else {
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim_locked();
            e = hipMalloc(&p, b);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(ST_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
            }
        }
    }
    g_live[p] = Block{b, s};
    g_in_use += b;
    return p;
}

void dev_release(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    size_t b = it->second.bytes;
    g_live.erase(it);
    g_in_use -= b;
    g_free[Key{(uintptr_t)s, b}].push_back(p);
    g_cached += b;
}

void dev_trim() {
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipDeviceSynchronize();
    trim_locked();
}

size_t dev_bytes_in_use() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_in_use;
}

// ------------------------------------------------------------------ fills --
__global__ void k_fill_u32(uint32_t *d, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = v;
}
__global__ void k_fill_u8(uint8_t *d, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = 0;
}

// Zero fill by a kernel (rather than a memset node) so that the same code is
// safe inside captured graphs.
void fill_zero(void *d, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if (bytes % 4 == 0 && ((uintptr_t)d % 4) == 0) {
        size_t n = bytes / 4;
        unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
        k_fill_u32<<<g, 256, 0, s>>>((uint32_t *)d, 0u, n);
    } else {
        unsigned g = (unsigned)std::min<size_t>((bytes + 255) / 256, 8192);
        k_fill_u8<<<g, 256, 0, s>>>((uint8_t *)d, bytes);
    }
    AIRG_LAUNCH_CHECK();
}

void fill_i32(int32_t *d, int32_t value, size_t count, hipStream_t s) {
    if (!count) return;
    unsigned g = (unsigned)std::min<size_t>((count + 255) / 256, 8192);
    k_fill_u32<<<g, 256, 0, s>>>((uint32_t *)d, (uint32_t)value, count);
    AIRG_LAUNCH_CHECK();
}

namespace {
std::mutex g_event_mu;
std::map<int, std::vector<hipEvent_t>> g_events;   // per device; never destroyed (the pool lives as long as the process)
}  // namespace

hipEvent_t pooled_event() {
    int dev = 0;
    AIRG_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_event_mu);
        auto &v = g_events[dev];
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e;
    AIRG_HIP(hipEventCreate(&e));
    return e;
}

void release_event(hipEvent_t e) {
    if (!e) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_event_mu);
    g_events[dev].push_back(e);
}

// Device-to-device copies by one kernel launch for up to kMaxCopies buffers.
// Each copy owns a contiguous range of workgroups; where both ends are
// 16-byte aligned its body moves as 16-byte vectors and the last (< 16) bytes
// as 4-byte words, else all of it as words (every element type here is 4 or 8
// bytes).  Grid-stride loops, at most 4096 workgroups in all.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct CopyItem {
    const char *src;
    char *dst;
    size_t vecs;       // 16-byte vectors from the start
    size_t words;      // 4-byte words after them
    unsigned block0, blocks;
};
struct CopySet {
    CopyItem it[kMaxCopies];
    int n;
};
__global__ void __launch_bounds__(256) k_copy_set(CopySet c) {
    int k = 0;
    while (k + 1 < c.n && blockIdx.x >= c.it[k + 1].block0) ++k;
    const CopyItem &t = c.it[k];
    const size_t first = (size_t)(blockIdx.x - t.block0) * 256 + threadIdx.x;
    const size_t stride = (size_t)t.blocks * 256;
    const u32x4 *sv = reinterpret_cast<const u32x4 *>(t.src);
    u32x4 *dv = reinterpret_cast<u32x4 *>(t.dst);
    for (size_t i = first; i < t.vecs; i += stride) dv[i] = __builtin_nontemporal_load(sv + i);
    const uint32_t *sw = reinterpret_cast<const uint32_t *>(t.src + t.vecs * 16);
    uint32_t *dw = reinterpret_cast<uint32_t *>(t.dst + t.vecs * 16);
    for (size_t i = first; i < t.words; i += stride) dw[i] = sw[i];
}

void copy_many(const CopyReq *req, int n, hipStream_t s) {
    AIRG_REQUIRE(n >= 0 && n <= kMaxCopies, ST_INVALID_ARG, "too many copies in one launch");
    CopySet c{};
    size_t work[kMaxCopies] = {};
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const CopyReq &r = req[i];
        if (!r.bytes) continue;
        const uintptr_t a = (uintptr_t)r.dst, b = (uintptr_t)r.src;
        if (r.bytes % 4 || a % 4 || b % 4) {   // not met by any element type here
            AIRG_HIP(hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToDevice, s));
            continue;
        }
        CopyItem &t = c.it[c.n];
        t.src = static_cast<const char *>(r.src);
        t.dst = static_cast<char *>(r.dst);
        t.vecs = (a % 16 == 0 && b % 16 == 0) ? r.bytes / 16 : 0;
        t.words = (r.bytes - t.vecs * 16) / 4;
        work[c.n] = std::max(t.vecs, t.words);
        total += work[c.n];
        ++c.n;
    }
    if (!c.n) return;
    // workgroups in proportion to each copy's work, at least one each
    const size_t budget = std::max<size_t>(std::min<size_t>((total + 255) / 256, 4096), (size_t)c.n);
    unsigned next = 0;
    for (int i = 0; i < c.n; ++i) {
        const size_t want = (work[i] + 255) / 256;
        const size_t share = std::max<size_t>(1, std::min(want, budget * work[i] / std::max<size_t>(total, 1)));
        c.it[i].block0 = next;
        c.it[i].blocks = (unsigned)share;
        next += (unsigned)share;
    }
    k_copy_set<<<next, 256, 0, s>>>(c);
    AIRG_LAUNCH_CHECK();
}

void copy_bytes(void *d, const void *src, size_t bytes, hipStream_t s) {
    const CopyReq r{d, src, bytes};
    copy_many(&r, 1, s);
}

// ------------------------------------------------------------------ scan ---
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int64_t kScanFusedBlocks = 1024;   // up to this many tiles the final pass reduces the block sums itself

// Exclusive scan of one value per thread across the block; returns the
// block total through *total.
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    int lane = threadIdx.x & (kWave - 1);
    int wid = threadIdx.x / kWave;
    int64_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// Up to kScanArrays independent arrays are scanned by the same launches,
// blockIdx.y selecting the array.
constexpr int kScanArrays = 4;
struct ScanSet {
    const int32_t *in[kScanArrays];
    int32_t *out[kScanArrays];
    int64_t n[kScanArrays];
    int64_t *bsum[kScanArrays];   // nb + 1 block sums per array (tiled path); [0] the total (small path)
    // optional samples: samp[q] = out[q * sstride] for q < nsamp (0: none)
    int32_t *samp[kScanArrays];
    int64_t sstride[kScanArrays];
    int64_t nsamp[kScanArrays];
};

// The sample taken at the total out[n], if n is a sampled position.
__device__ inline void sample_total(const ScanSet &S, int r, int64_t n, int64_t total) {
    const int64_t st = S.sstride[r];
    if (S.nsamp[r] > 0 && n % st == 0 && n / st < S.nsamp[r]) S.samp[r][n / st] = (int32_t)total;
}

__host__ __device__ inline int64_t scan_tiles(int64_t n) {
    return n > 0 ? (n + kScanTile - 1) / kScanTile : 1;
}

__global__ void k_scan_reduce(ScanSet S) {
    const int r = blockIdx.y;
    const int32_t *in = S.in[r];
    const int64_t n = S.n[r];
    if ((int64_t)blockIdx.x >= scan_tiles(n)) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) S.bsum[r][blockIdx.x] = tot;
}

// Single block per array: exclusive scan of the nb block sums in place,
// total at bsum[nb].
__global__ void k_scan_bsums(ScanSet S) {
    const int r = blockIdx.y;
    int64_t *bsum = S.bsum[r];
    const int64_t nb = scan_tiles(S.n[r]);
    int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    int64_t lo = (int64_t)threadIdx.x * per;
    int64_t hi = lo + per < nb ? lo + per : nb;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += bsum[i];
    int64_t tot;
    int64_t off = block_exclusive_scan(s, &tot);
    for (int64_t i = lo; i < hi; ++i) {
        int64_t v = bsum[i];
        bsum[i] = off;
        off += v;
    }
    if (threadIdx.x == 0) bsum[nb] = tot;
}

__device__ inline int scan_slot(int p) { return p + (p >> 5); }   // pads out LDS bank conflicts

// Block b scans its tile and adds the sums of the blocks before it: with
// SUMS_SCANNED bsum[b] already holds them (k_scan_bsums ran); otherwise the
// block reduces bsum[0..b) itself (few, L2-resident values), which saves the
// separate pass.  The tile moves through LDS both ways, so that the loads and
// stores are coalesced while each thread scans kScanItems consecutive
// entries.  The last block writes out[n] and the total at bsum[nb].
template <bool SUMS_SCANNED>
__global__ void __launch_bounds__(kScanThreads) k_scan_final(ScanSet S) {
    __shared__ int32_t buf[kScanTile + kScanTile / 32];
    const int r = blockIdx.y;
    const int32_t *in = S.in[r];
    int32_t *out = S.out[r];
    const int64_t n = S.n[r];
    int64_t *bsum = S.bsum[r];
    const int64_t nb = scan_tiles(n);
    if ((int64_t)blockIdx.x >= nb) return;
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int p = j * kScanThreads + tid;
        buf[scan_slot(p)] = t0 + p < n ? in[t0 + p] : 0;
    }
    int64_t before;
    if (SUMS_SCANNED) {
        before = bsum[blockIdx.x];
    } else {
        int64_t part = 0;
        for (int64_t i = tid; i < (int64_t)blockIdx.x; i += kScanThreads) part += bsum[i];
        block_exclusive_scan(part, &before);   // its barriers also complete the tile's LDS stores
    }
    __syncthreads();
    int32_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = buf[scan_slot(tid * kScanItems + k)];
        s += v[k];
    }
    int64_t tot;
    int64_t off = block_exclusive_scan(s, &tot) + before;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        buf[scan_slot(tid * kScanItems + k)] = (int32_t)off;
        off += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int p = j * kScanThreads + tid;
        if (t0 + p < n) out[t0 + p] = buf[scan_slot(p)];
    }
    if (S.nsamp[r] > 0) {   // sampled positions inside [t0, min(t0 + tile, n))
        const int64_t st = S.sstride[r], hi = t0 + kScanTile < n ? t0 + kScanTile : n;
        for (int64_t q = (t0 + st - 1) / st + tid; q < S.nsamp[r] && q * st < hi; q += kScanThreads)
            S.samp[r][q] = buf[scan_slot((int)(q * st - t0))];
    }
    if ((int64_t)blockIdx.x == nb - 1 && tid == 0) {
        out[n] = (int32_t)(before + tot);
        sample_total(S, r, n, before + tot);
        if (!SUMS_SCANNED) bsum[nb] = before + tot;
    }
}

// Small inputs: one workgroup per array scans everything, a tile of
// kSmallScanTile entries at a time: coalesced loads into LDS, each thread
// scans kSmallScanItems consecutive entries there, a workgroup scan of the
// per-thread sums, coalesced stores, and a carry into the next tile.
constexpr int kSmallScanThreads = 1024;
constexpr int kSmallScanItems = 8;
constexpr int64_t kSmallScan = 16384;
constexpr int64_t kTinyScan = 2048;   // up to this size a 256-thread workgroup

template <int TH>
__global__ void __launch_bounds__(TH) k_scan_small(ScanSet S) {
    constexpr int kSmallScanTile = TH * kSmallScanItems;
    __shared__ int32_t buf[kSmallScanTile + kSmallScanTile / 32];
    __shared__ int64_t wsum[TH / kWave];
    const int r = blockIdx.y;
    const int32_t *in = S.in[r];
    int32_t *out = S.out[r];
    const int64_t n = S.n[r];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kSmallScanTile) {
#pragma unroll
        for (int j = 0; j < kSmallScanItems; ++j) {
            int p = j * TH + tid;
            buf[scan_slot(p)] = t0 + p < n ? in[t0 + p] : 0;
        }
        __syncthreads();
        int32_t v[kSmallScanItems];
        int64_t s = 0;
#pragma unroll
        for (int u = 0; u < kSmallScanItems; ++u) {
            v[u] = buf[scan_slot(tid * kSmallScanItems + u)];
            s += v[u];
        }
        int64_t x = s;
        for (int o = 1; o < kWave; o <<= 1) {
            int64_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[wid] = x;
        __syncthreads();
        int64_t off = carry + x - s, tot = 0;
        for (int w = 0; w < TH / kWave; ++w) {
            if (w < wid) off += wsum[w];
            tot += wsum[w];
        }
#pragma unroll
        for (int u = 0; u < kSmallScanItems; ++u) {
            buf[scan_slot(tid * kSmallScanItems + u)] = (int32_t)off;
            off += v[u];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSmallScanItems; ++j) {
            int p = j * TH + tid;
            if (t0 + p < n) out[t0 + p] = buf[scan_slot(p)];
        }
        if (S.nsamp[r] > 0) {   // sampled positions inside [t0, min(t0 + tile, n))
            const int64_t st = S.sstride[r], hi = t0 + kSmallScanTile < n ? t0 + kSmallScanTile : n;
            for (int64_t q = (t0 + st - 1) / st + tid; q < S.nsamp[r] && q * st < hi; q += TH)
                S.samp[r][q] = buf[scan_slot((int)(q * st - t0))];
        }
        carry += tot;
        __syncthreads();
    }
    if (tid == 0) {
        out[n] = (int32_t)carry;
        sample_total(S, r, n, carry);
        S.bsum[r][0] = carry;
    }
}

// ------------------------------------------------------ batched readback --
// Readbacks land in pinned host memory mapped into the device address
// space: the gather kernel stores into it directly, so a readback costs one
// launch and one stream synchronisation, with no staging copy through
// pageable memory and no upload of the gather table.
namespace {
constexpr int kReadRanges = 16;
constexpr int kReadChunk = 1024;                      // words per block and range
constexpr size_t kReadStageMax = (size_t)1 << 22;     // bytes read through the pinned buffer

struct ReadArgs {
    const int32_t *src[kReadRanges];
    int32_t cnt[kReadRanges];
    int64_t off[kReadRanges];
};

// Small readbacks (all ranges in one table, at most kReadSignalWords words):
// one workgroup copies them and then writes `seq` into the stage's flag,
// after every lane's copies have completed at system scope, so that the host
// can watch the flag instead of waiting for the stream's completion signal
// (about 12 us a round trip on an idle MI355X against about 6.6 us).
constexpr int64_t kReadSignalWords = 4096;
__global__ void __launch_bounds__(256) k_read_words_signal(ReadArgs a, int nranges, int32_t *__restrict__ out,
                                                           int32_t *flag, int32_t seq) {
    for (int r = 0; r < nranges; ++r) {
        const int32_t *p = a.src[r];
        int32_t *o = out + a.off[r];
        for (int64_t i = threadIdx.x; i < a.cnt[r]; i += 256)
            __hip_atomic_store(o + i, p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // the copies are system-coherent stores; every wave waits for its own to
    // complete before the barrier, and the flag is stored after it
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Block (x, r) copies words [x * kReadChunk, (x + 1) * kReadChunk) of range r.
__global__ void __launch_bounds__(256) k_read_words(ReadArgs a, int32_t *__restrict__ out) {
    const int r = blockIdx.y;
    const int64_t end = (int64_t)a.cnt[r] < ((int64_t)blockIdx.x + 1) * kReadChunk ? (int64_t)a.cnt[r]
                                                                                   : ((int64_t)blockIdx.x + 1) * kReadChunk;
    const int32_t *p = a.src[r];
    int32_t *o = out + a.off[r];
    for (int64_t i = (int64_t)blockIdx.x * kReadChunk + threadIdx.x; i < end; i += 256) o[i] = p[i];
}

// A few pinned buffers, so that host threads driving different streams do
// not wait on each other's synchronisations; a readback takes the first free
// one (or waits for the first).
struct ReadStage {
    std::mutex mu;
    int32_t *host = nullptr;   // host view of the pinned buffer
    int32_t *dev = nullptr;    // its device address
    size_t words = 0;
    int32_t *flag_host = nullptr, *flag_dev = nullptr;   // completion flag of signalled readbacks
    uint32_t seq = 0;

    int32_t *flag() {
        if (!flag_host) {
            AIRG_HIP(hipHostMalloc((void **)&flag_host, 64,
                                   hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent));
            AIRG_HIP(hipHostGetDevicePointer((void **)&flag_dev, flag_host, 0));
            *reinterpret_cast<volatile int32_t *>(flag_host) = 0;
        }
        return flag_dev;
    }

    // Room for `words` (mu held; every earlier use has been synchronised, so
    // the old buffer can go).
    int32_t *reserve(size_t w) {
        if (w > words) {
            if (host) (void)hipHostFree(host);
            host = dev = nullptr;
            words = 0;
            size_t n = std::max<size_t>(w, (size_t)1 << 14);
            AIRG_HIP(hipHostMalloc((void **)&host, n * sizeof(int32_t),
                                   hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent));
            AIRG_HIP(hipHostGetDevicePointer((void **)&dev, host, 0));
            words = n;
        }
        return dev;
    }
};
constexpr int kReadStages = 4;
ReadStage g_stage[kReadStages];

std::unique_lock<std::mutex> take_stage(ReadStage **out) {
    for (auto &st : g_stage) {
        std::unique_lock<std::mutex> lk(st.mu, std::try_to_lock);
        if (lk.owns_lock()) {
            *out = &st;
            return lk;
        }
    }
    *out = &g_stage[0];
    return std::unique_lock<std::mutex>(g_stage[0].mu);
}

// Waits for a signalled readback: watches the stage's flag for a while (the
// copy is normally the last work queued), then falls back to a stream
// synchronisation, which also reports any error of the stream.
void wait_signal(ReadStage *st, int32_t seq, hipStream_t s) {
    const volatile int32_t *f = st->flag_host;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0; *f != seq; ++spin) {
        if ((spin & 255u) == 255u && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(500)) {
            AIRG_HIP(hipStreamSynchronize(s));
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

// Reads ranges [0, m) into the stage's pinned buffer and waits for them:
// small reads through the signalled kernel, others through the gather
// kernels and a stream synchronisation.
void read_ranges(const int32_t *const *src, const int32_t *cnt, const int64_t *off, size_t m, int64_t total,
                 ReadStage *st, hipStream_t s);

// Launches the gathers of ranges [0, m) into dev (offsets in words).
void launch_reads(const int32_t *const *src, const int32_t *cnt, const int64_t *off, size_t m, int32_t *dev,
                  hipStream_t s) {
    for (size_t b = 0; b < m; b += kReadRanges) {
        ReadArgs a{};
        const int k = (int)std::min<size_t>(kReadRanges, m - b);
        int64_t maxc = 0;
        for (int j = 0; j < k; ++j) {
            a.src[j] = src[b + j];
            a.cnt[j] = cnt[b + j];
            a.off[j] = off[b + j];
            maxc = std::max<int64_t>(maxc, cnt[b + j]);
        }
        if (maxc == 0) continue;
        dim3 grid((unsigned)((maxc + kReadChunk - 1) / kReadChunk), (unsigned)k);
        k_read_words<<<grid, 256, 0, s>>>(a, dev);
        AIRG_LAUNCH_CHECK();
    }
}

void read_ranges(const int32_t *const *src, const int32_t *cnt, const int64_t *off, size_t m, int64_t total,
                 ReadStage *st, hipStream_t s) {
    int32_t *dev = st->reserve((size_t)total);
    if (m <= (size_t)kReadRanges && total <= kReadSignalWords) {
        ReadArgs a{};
        for (size_t j = 0; j < m; ++j) {
            a.src[j] = src[j];
            a.cnt[j] = cnt[j];
            a.off[j] = off[j];
        }
        int32_t *flag = st->flag();
        const int32_t seq = (int32_t)++st->seq;
        k_read_words_signal<<<1, 256, 0, s>>>(a, (int)m, dev, flag, seq);
        AIRG_LAUNCH_CHECK();
        wait_signal(st, seq, s);
        return;
    }
    launch_reads(src, cnt, off, m, dev, s);
    AIRG_HIP(hipStreamSynchronize(s));
}
}  // namespace

void read_ints(const std::vector<const int32_t *> &src, const std::vector<int32_t> &counts, int32_t *h,
               hipStream_t s) {
    const size_t m = src.size();
    if (m == 0) return;
    std::vector<int64_t> off(m);
    int64_t total = 0;
    for (size_t i = 0; i < m; ++i) {
        AIRG_REQUIRE(counts[i] >= 0, ST_INVALID_ARG, "negative readback count");
        off[i] = total;
        total += counts[i];
    }
    if (total == 0) return;
    ReadStage *st;
    auto lk = take_stage(&st);
    read_ranges(src.data(), counts.data(), off.data(), m, total, st, s);
    std::memcpy(h, st->host, (size_t)total * sizeof(int32_t));
}

void read_bytes(void *h, const void *d, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if (bytes % 4 != 0 || (uintptr_t)d % 4 != 0 || bytes > kReadStageMax) {
        AIRG_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
        AIRG_HIP(hipStreamSynchronize(s));
        return;
    }
    const int32_t *src = static_cast<const int32_t *>(d);
    const int32_t cnt = (int32_t)(bytes / 4);
    const int64_t off = 0;
    ReadStage *st;
    auto lk = take_stage(&st);
    read_ranges(&src, &cnt, &off, 1, (int64_t)cnt, st, s);
    std::memcpy(h, st->host, bytes);
}

void resolve_sizes(const std::vector<Csr *> &ms, hipStream_t s) {
    std::vector<const int32_t *> src;
    std::vector<int32_t> cnt;
    for (Csr *M : ms) {
        src.push_back(M->rp.p + M->nr);
        cnt.push_back(1);
    }
    std::vector<int32_t> nz(ms.size());
    read_ints(src, cnt, nz.data(), s);
    for (size_t i = 0; i < ms.size(); ++i) {
        AIRG_REQUIRE(nz[i] >= 0, ST_LIMIT, "prefix sum exceeds the int32 index range");
        Csr &M = *ms[i];
        M.nnz = nz[i];
        M.ci.alloc((size_t)M.nnz, s);
        M.v.alloc((size_t)M.nnz, s);
    }
}

// Blocked layout: thread t of block b owns items [b*tile + t*items, +items).
// The reduce kernel above strides differently, but only block totals are
// taken from it, and those do not depend on the layout inside the tile.
// Returns where each array's total lands on the device.
static std::vector<const int64_t *> scan_set(const int32_t *const *in, int32_t *const *out, const int64_t *n, int k,
                                             DBuf<int64_t> &sums, hipStream_t s, const ScanSample *smp = nullptr) {
    AIRG_REQUIRE(k >= 1 && k <= kScanArrays, ST_INVALID_ARG, "bad number of scans");
    ScanSet S{};
    bool small = true;
    int64_t maxnb = 1, slots = 0;
    for (int r = 0; r < k; ++r) {
        small = small && n[r] <= kSmallScan;
        maxnb = std::max(maxnb, scan_tiles(n[r]));
        slots += scan_tiles(n[r]) + 1;
    }
    sums.alloc((size_t)slots, s);
    std::vector<const int64_t *> tot((size_t)k);
    int64_t o = 0;
    for (int r = 0; r < k; ++r) {
        S.in[r] = in[r];
        S.out[r] = out[r];
        S.n[r] = n[r];
        S.bsum[r] = sums.p + o;
        if (smp && smp[r].count > 0) {
            AIRG_REQUIRE(smp[r].stride >= 1 && (smp[r].count - 1) * smp[r].stride <= n[r], ST_INVALID_ARG,
                         "scan samples beyond the output");
            S.samp[r] = smp[r].out;
            S.sstride[r] = smp[r].stride;
            S.nsamp[r] = smp[r].count;
        }
        tot[r] = small ? sums.p + o : sums.p + o + scan_tiles(n[r]);
        o += scan_tiles(n[r]) + 1;
    }
    if (small) {
        bool tiny = true;
        for (int r = 0; r < k; ++r) tiny = tiny && n[r] <= kTinyScan;
        if (tiny) k_scan_small<256><<<dim3(1, k), 256, 0, s>>>(S);
        else k_scan_small<kSmallScanThreads><<<dim3(1, k), kSmallScanThreads, 0, s>>>(S);
    } else {
        k_scan_reduce<<<dim3((unsigned)maxnb, k), kScanThreads, 0, s>>>(S);
        AIRG_LAUNCH_CHECK();
        if (maxnb <= kScanFusedBlocks) {
            k_scan_final<false><<<dim3((unsigned)maxnb, k), kScanThreads, 0, s>>>(S);
        } else {
            k_scan_bsums<<<dim3(1, k), kScanThreads, 0, s>>>(S);
            AIRG_LAUNCH_CHECK();
            k_scan_final<true><<<dim3((unsigned)maxnb, k), kScanThreads, 0, s>>>(S);
        }
    }
    AIRG_LAUNCH_CHECK();
    return tot;
}

void exclusive_scans(const std::vector<const int32_t *> &in, const std::vector<int32_t *> &out,
                     const std::vector<int64_t> &n, hipStream_t s) {
    DBuf<int64_t> sums;
    scan_set(in.data(), out.data(), n.data(), (int)in.size(), sums, s);
}

void exclusive_scan_sampled(const int32_t *in, int32_t *out, int64_t n, const ScanSample &smp, hipStream_t s) {
    DBuf<int64_t> sums;
    scan_set(&in, &out, &n, 1, sums, s, &smp);
}

int64_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, bool want_total) {
    DBuf<int64_t> sums;
    auto tot = scan_set(&in, &out, &n, 1, sums, s);
    if (!want_total) return -1;
    int64_t t = d2h_one(tot[0], s);
    AIRG_REQUIRE(t < ((int64_t)1 << 31), ST_LIMIT, "prefix sum exceeds the int32 index range");
    return t;
}

}  // namespace airg

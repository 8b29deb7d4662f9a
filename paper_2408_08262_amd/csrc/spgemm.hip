// Two-phase sparse matrix product C = A B for gfx950 with LDS hash rows.
//
// Rows are binned by their product-count upper bound ub_i = sum_k |B_k|.
// Short A rows with few products: one thread per row merging the sorted B
// rows.  Other small rows: one G-lane group per row with a private hash table
// in LDS.
// Larger rows: one workgroup per row (table in LDS up to 8192 slots, in
// global scratch beyond).  The symbolic pass counts distinct columns, the
// numeric pass accumulates.  Accumulation is deterministic: the entries of
// the A row are taken one at a time in ascending order and the lanes spread
// over the B row, whose columns are distinct, so every output entry receives
// its products in ascending k order, without contraction -- the same order
// and rounding as a sequential row-wise (Gustavson) product.
#include "csr.hpp"
#include "group.hpp"
#include "spgemm.hpp"

namespace airg {

constexpr int32_t kEmpty = -1;
constexpr int kMergeLists = 16;

__device__ inline uint32_t hash_slot(int32_t c, uint32_t mask) { return ((uint32_t)c * 2654435761u) & mask; }

// Returns the slot holding key c, inserting it if absent; *fresh tells
// whether this call inserted it.
__device__ inline uint32_t hash_insert(int32_t *keys, uint32_t mask, int32_t c, bool *fresh) {
    uint32_t s = hash_slot(c, mask);
    for (;;) {
        int32_t k = keys[s];
        if (k == c) { *fresh = false; return s; }
        if (k == kEmpty) {
            int32_t old = atomicCAS(&keys[s], kEmpty, c);
            if (old == kEmpty) { *fresh = true; return s; }
            if (old == c) { *fresh = false; return s; }
        }
        s = (s + 1) & mask;
    }
}

__global__ void k_spgemm_ub(int32_t m, const int32_t *__restrict__ arp, const int32_t *__restrict__ aci,
                            const int32_t *__restrict__ brp, int32_t *__restrict__ ub, int8_t *__restrict__ bin) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t u = 0;
    for (int32_t k = arp[i]; k < arp[i + 1]; ++k) {
        int32_t j = aci[k];
        u += brp[j + 1] - brp[j];
    }
    int32_t uc = u > 0x7fffffff ? 0x7fffffff : (int32_t)u;
    ub[i] = uc;
    int32_t L = arp[i + 1] - arp[i];
    bin[i] = uc == 0                            ? 0
             : (L <= kMergeLists && uc <= 256) ? 7
             : uc <= 8                         ? 1
             : uc <= 32                        ? 2
             : uc <= 128                       ? 3
             : uc <= 1024                      ? 4
             : uc <= 4096                      ? 5
                                               : 6;
}

// ---------------------------------------------------------- merged rows ---
// Short A rows: one thread per row merges the (sorted) B rows of its
// entries; the smallest head column is emitted with the products of every
// list holding it summed in list (= ascending k) order.
template <bool NUMERIC>
__global__ void __launch_bounds__(256) k_spgemm_merge(const int32_t *__restrict__ list, int64_t count,
                                                      const int32_t *__restrict__ arp,
                                                      const int32_t *__restrict__ aci,
                                                      const double *__restrict__ av,
                                                      const int32_t *__restrict__ brp,
                                                      const int32_t *__restrict__ bci,
                                                      const double *__restrict__ bv, int32_t *__restrict__ cnt,
                                                      const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                                      double *__restrict__ cv) {
#pragma clang fp contract(off)
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t a0 = arp[row], L = arp[row + 1] - a0;
    int32_t pos[kMergeLists], end[kMergeLists], head[kMergeLists];
    double aval[kMergeLists];
#pragma unroll
    for (int q = 0; q < kMergeLists; ++q) {
        pos[q] = end[q] = 0;
        head[q] = 0x7fffffff;
        aval[q] = 0.0;
        if (q < L) {
            int32_t k = aci[a0 + q];
            pos[q] = brp[k];
            end[q] = brp[k + 1];
            if (NUMERIC) aval[q] = av[a0 + q];
            if (pos[q] < end[q]) head[q] = bci[pos[q]];
        }
    }
    int32_t w = NUMERIC ? crp[row] : 0;
    int32_t emitted = 0;
    for (;;) {
        int32_t c = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < kMergeLists; ++q) c = head[q] < c ? head[q] : c;
        if (c == 0x7fffffff) break;
        double acc = 0.0;
        bool first = true;
#pragma unroll
        for (int q = 0; q < kMergeLists; ++q) {
            if (head[q] == c) {
                if (NUMERIC) {
                    double p = aval[q] * bv[pos[q]];
                    acc = first ? p : acc + p;
                }
                first = false;
                ++pos[q];
                head[q] = pos[q] < end[q] ? bci[pos[q]] : 0x7fffffff;
            }
        }
        if (NUMERIC) {
            cci[w] = c;
            cv[w] = acc;
            ++w;
        }
        ++emitted;
    }
    if (!NUMERIC) cnt[row] = emitted;
}

// ---------------------------------------------------------- group rows ----
// One G-lane group per row, T-slot table per group.  NUMERIC = false counts
// the distinct columns into cnt[row]; NUMERIC = true writes the sorted row.
template <int G, int T, int TPB, bool NUMERIC>
__global__ void __launch_bounds__(TPB) k_spgemm_group(const int32_t *__restrict__ list, int64_t count,
                                                      const int32_t *__restrict__ arp,
                                                      const int32_t *__restrict__ aci,
                                                      const double *__restrict__ av,
                                                      const int32_t *__restrict__ brp,
                                                      const int32_t *__restrict__ bci,
                                                      const double *__restrict__ bv, int32_t *__restrict__ cnt,
                                                      const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                                      double *__restrict__ cv) {
#pragma clang fp contract(off)
    constexpr int NG = TPB / G;
    __shared__ int32_t Ks[NG][T];
    __shared__ double Vs[NG][NUMERIC ? T : 1];
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t *keys = Ks[gid];
    double *vals = Vs[gid];
    for (int t = lane; t < T; t += G) {
        keys[t] = kEmpty;
        if (NUMERIC) vals[t] = 0.0;
    }
    wave_sync();
    int fresh_cnt = 0;
    for (int32_t ka = arp[row]; ka < arp[row + 1]; ++ka) {
        int32_t k = aci[ka];
        double a = NUMERIC ? av[ka] : 0.0;
        for (int32_t kb = brp[k] + lane; kb < brp[k + 1]; kb += G) {
            bool fresh;
            uint32_t s = hash_insert(keys, T - 1, bci[kb], &fresh);
            fresh_cnt += fresh;
            if (NUMERIC) vals[s] = vals[s] + a * bv[kb];
        }
        wave_sync();
    }
    if (!NUMERIC) {
        fresh_cnt = group_sum<G>(fresh_cnt);
        if (lane == 0) cnt[row] = fresh_cnt;
        return;
    }
    // rank each occupied slot among the occupied keys; ranks give the
    // ascending column order of the output row
    int32_t base = crp[row];
    for (int t = lane; t < T; t += G) {
        int32_t key = keys[t];
        if (key == kEmpty) continue;
        int r = 0;
        for (int u = 0; u < T; ++u) {
            int32_t o = keys[u];
            r += (o != kEmpty) & (o < key);
        }
        cci[base + r] = key;
        cv[base + r] = vals[t];
    }
}

// ----------------------------------------------------------- block rows ---
// One workgroup per row with a table of T slots at (keys, vals): T = 2048 /
// 8192 in LDS or the row's slice of global scratch.  After accumulation the
// occupied slots are compacted to the front and bitonic-sorted by column.
constexpr int kBlk = 256;

__device__ inline int block_exclusive_count(int v, int *total, int *sh) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kBlk / 64; ++w) {
        if (w < wid) off += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

template <bool NUMERIC>
__device__ void spgemm_block_row(int32_t row, int32_t *keys, double *vals, uint32_t T,
                                 const int32_t *__restrict__ arp, const int32_t *__restrict__ aci,
                                 const double *__restrict__ av, const int32_t *__restrict__ brp,
                                 const int32_t *__restrict__ bci, const double *__restrict__ bv,
                                 int32_t *__restrict__ cnt, const int32_t *__restrict__ crp,
                                 int32_t *__restrict__ cci, double *__restrict__ cv) {
#pragma clang fp contract(off)
    __shared__ int sh[kBlk / 64];
    for (uint32_t t = threadIdx.x; t < T; t += kBlk) {
        keys[t] = kEmpty;
        if (NUMERIC) vals[t] = 0.0;
    }
    __syncthreads();
    int fresh_cnt = 0;
    for (int32_t ka = arp[row]; ka < arp[row + 1]; ++ka) {
        int32_t k = aci[ka];
        double a = NUMERIC ? av[ka] : 0.0;
        for (int32_t kb = brp[k] + threadIdx.x; kb < brp[k + 1]; kb += kBlk) {
            bool fresh;
            uint32_t s = hash_insert(keys, T - 1, bci[kb], &fresh);
            fresh_cnt += fresh;
            if (NUMERIC) vals[s] = vals[s] + a * bv[kb];
        }
        __syncthreads();
    }
    if (!NUMERIC) {
        int tot;
        block_exclusive_count(fresh_cnt, &tot, sh);
        if (threadIdx.x == 0) cnt[row] = tot;
        return;
    }
    // compact the occupied slots into the output row (unsorted): thread t
    // owns a contiguous chunk of slots and writes after the chunks before it
    uint32_t per = (T + kBlk - 1) / kBlk;
    uint32_t lo = threadIdx.x * per, hi = lo + per < T ? lo + per : T;
    int mine = 0;
    for (uint32_t t = lo; t < hi; ++t) mine += keys[t] != kEmpty;
    int nz;
    int off = block_exclusive_count(mine, &nz, sh);
    int32_t base = crp[row];
    for (uint32_t t = lo; t < hi; ++t) {
        int32_t kk = keys[t];
        if (kk != kEmpty) {
            cci[base + off] = kk;
            cv[base + off] = vals[t];
            ++off;
        }
    }
    __syncthreads();
    // bitonic sort of the nz entries (padded to a power of two) in the table
    uint32_t P = 1;
    while ((int)P < nz) P <<= 1;
    for (uint32_t t = threadIdx.x; t < P; t += kBlk) {
        if ((int)t < nz) {
            keys[t] = cci[base + t];
            vals[t] = cv[base + t];
        } else {
            keys[t] = 0x7fffffff;
            vals[t] = 0.0;
        }
    }
    __syncthreads();
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < P; t += kBlk) {
                uint32_t q = t ^ j;
                if (q > t) {
                    bool up = (t & kk) == 0;
                    int32_t a = keys[t], b = keys[q];
                    if ((a > b) == up) {
                        keys[t] = b;
                        keys[q] = a;
                        double va = vals[t];
                        vals[t] = vals[q];
                        vals[q] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < nz; t += kBlk) {
        cci[base + t] = keys[t];
        cv[base + t] = vals[t];
    }
}

template <int T, bool NUMERIC>
__global__ void __launch_bounds__(kBlk) k_spgemm_block_lds(const int32_t *__restrict__ list, int64_t count,
                                                           const int32_t *__restrict__ arp,
                                                           const int32_t *__restrict__ aci,
                                                           const double *__restrict__ av,
                                                           const int32_t *__restrict__ brp,
                                                           const int32_t *__restrict__ bci,
                                                           const double *__restrict__ bv, int32_t *__restrict__ cnt,
                                                           const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                                           double *__restrict__ cv) {
    __shared__ int32_t keys[T];
    __shared__ double vals[NUMERIC ? T : 1];
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    spgemm_block_row<NUMERIC>(list[idx], keys, vals, T, arp, aci, av, brp, bci, bv, cnt, crp, cci, cv);
}

template <bool NUMERIC>
__global__ void __launch_bounds__(kBlk) k_spgemm_block_global(const int32_t *__restrict__ list, int64_t count,
                                                              const int64_t *__restrict__ toff,
                                                              int32_t *__restrict__ gkeys,
                                                              double *__restrict__ gvals,
                                                              const int32_t *__restrict__ arp,
                                                              const int32_t *__restrict__ aci,
                                                              const double *__restrict__ av,
                                                              const int32_t *__restrict__ brp,
                                                              const int32_t *__restrict__ bci,
                                                              const double *__restrict__ bv,
                                                              int32_t *__restrict__ cnt,
                                                              const int32_t *__restrict__ crp,
                                                              int32_t *__restrict__ cci, double *__restrict__ cv) {
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    int64_t o = toff[idx];
    uint32_t T = (uint32_t)(toff[idx + 1] - o);
    spgemm_block_row<NUMERIC>(list[idx], gkeys + o, NUMERIC ? gvals + o : nullptr, T, arp, aci, av, brp, bci, bv,
                              cnt, crp, cci, cv);
}

// ------------------------------------------------------------------ host --
static uint32_t pow2_at_least(int64_t v) {
    uint32_t p = 1;
    while ((int64_t)p < v) p <<= 1;
    return p;
}

template <bool NUMERIC>
static void run_bins(const Bins &B, const CsrView &A, const CsrView &Bm, int32_t *cnt, const int32_t *crp,
                     int32_t *cci, double *cv, const std::vector<int32_t> &ub6, hipStream_t s) {
    auto args = [&](auto kern, unsigned grid, unsigned tpb, int b) {
        kern<<<grid, tpb, 0, s>>>(B.list(b), B.count(b), A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv);
    };
    if (B.count(7)) args(k_spgemm_merge<NUMERIC>, grid_for(B.count(7), 256), 256, 7);
    if (B.count(1)) args(k_spgemm_group<4, 16, 256, NUMERIC>, grid_for(B.count(1), 64), 256, 1);
    if (B.count(2)) args(k_spgemm_group<8, 64, 256, NUMERIC>, grid_for(B.count(2), 32), 256, 2);
    if (B.count(3)) args(k_spgemm_group<16, 256, 256, NUMERIC>, grid_for(B.count(3), 16), 256, 3);
    if (B.count(4)) args(k_spgemm_block_lds<2048, NUMERIC>, (unsigned)B.count(4), kBlk, 4);
    if (B.count(5)) args(k_spgemm_block_lds<8192, NUMERIC>, (unsigned)B.count(5), kBlk, 5);
    AIRG_LAUNCH_CHECK();
    if (B.count(6)) {
        // global tables: 2 ub rounded up to a power of two per row
        std::vector<int64_t> off(ub6.size() + 1, 0);
        for (size_t r = 0; r < ub6.size(); ++r) off[r + 1] = off[r] + pow2_at_least(2 * (int64_t)ub6[r]);
        DBuf<int64_t> toff(off.size(), s);
        h2d(toff.p, off.data(), off.size(), s);
        DBuf<int32_t> gk((size_t)off.back(), s);
        DBuf<double> gv(NUMERIC ? (size_t)off.back() : 1, s);
        k_spgemm_block_global<NUMERIC><<<(unsigned)B.count(6), kBlk, 0, s>>>(
            B.list(6), B.count(6), toff.p, gk.p, gv.p, A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv);
        AIRG_LAUNCH_CHECK();
    }
}

Csr spgemm(const CsrView &A, const CsrView &Bm, hipStream_t s) {
    AIRG_REQUIRE(A.nc == Bm.nr, ST_INVALID_ARG, "inner dimensions differ");
    Csr C;
    C.nr = A.nr;
    C.nc = Bm.nc;
    C.rp.alloc((size_t)A.nr + 1, s);
    int32_t m = A.nr;
    DBuf<int32_t> ub((size_t)m + 1, s), cnt((size_t)m + 1, s);
    DBuf<int8_t> bin((size_t)m + 1, s);
    fill_zero(cnt.p, ((size_t)m + 1) * 4, s);
    if (m > 0) {
        k_spgemm_ub<<<grid_for(m, 256), 256, 0, s>>>(m, A.rp, A.ci, Bm.rp, ub.p, bin.p);
        AIRG_LAUNCH_CHECK();
    }
    Bins B = bin_rows(bin.p, m, 8, s);
    std::vector<int32_t> ub6;
    if (B.count(6)) {
        std::vector<int32_t> rows((size_t)B.count(6)), ubh((size_t)m);
        d2h(rows.data(), B.list(6), rows.size(), s);
        d2h(ubh.data(), ub.p, (size_t)m, s);
        ub6.resize(rows.size());
        for (size_t r = 0; r < rows.size(); ++r) ub6[r] = ubh[rows[r]];
    }
    run_bins<false>(B, A, Bm, cnt.p, nullptr, nullptr, nullptr, ub6, s);
    C.nnz = exclusive_scan(cnt.p, C.rp.p, m, s);
    C.ci.alloc((size_t)C.nnz, s);
    C.v.alloc((size_t)C.nnz, s);
    run_bins<true>(B, A, Bm, cnt.p, C.rp.p, C.ci.p, C.v.p, ub6, s);
    return C;
}

}  // namespace airg

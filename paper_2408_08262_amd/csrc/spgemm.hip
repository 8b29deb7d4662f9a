// Two-phase sparse matrix product C = A B for gfx950 with LDS hash rows
// (dense LDS accumulator rows when B has at most 4096 columns).
//
// Symbolic pass: rows are binned by their product-count upper bound
// ub_i = sum_k |B_k| and their distinct columns counted by a G-lane group (or
// a whole workgroup) inserting columns into a hash table of at least 2 ub
// slots in LDS (global scratch beyond 8192 products).
// Numeric pass: rows are binned again by their exact length cnt_i, so the
// value table needs only 2 cnt slots however many products collide in it:
// the group accumulates, compacts the occupied slots in place and
// bitonic-sorts them by column.  Accumulation is deterministic: the entries of
// the A row are taken one at a time in ascending order and the lanes spread
// over the B row, whose columns are distinct, so every output entry receives
// its products in ascending k order, without contraction -- the same order
// and rounding as a sequential row-wise (Gustavson) product.  The additions
// into LDS tables are the LDS unit's double add (one correctly rounded add,
// as in registers, with no read back into the wavefront): a wavefront's LDS
// operations complete in program order, so the order per slot is unchanged.
#include "csr.hpp"
#include "group.hpp"
#include "spgemm.hpp"

namespace airg {

constexpr int32_t kEmpty = -1;

__device__ inline uint32_t hash_slot(int32_t c, uint32_t mask) { return ((uint32_t)c * 2654435761u) & mask; }

// Returns the slot holding key c, inserting it if absent; *fresh tells
// whether this call inserted it.  Each probe is one compare-and-swap, which
// returns the slot's key: empty (now c, inserted), c (present) or another.
__device__ inline uint32_t hash_insert(int32_t *keys, uint32_t mask, int32_t c, bool *fresh) {
    uint32_t s = hash_slot(c, mask);
    for (;;) {
        const int32_t old = atomicCAS(&keys[s], kEmpty, c);
        if (old == kEmpty || old == c) {
            *fresh = old == kEmpty;
            return s;
        }
        s = (s + 1) & mask;
    }
}

// Symbolic bins by ub.
enum : int8_t { SB_EMPTY = 0, SB_G4, SB_G8, SB_G16, SB_G32S, SB_G32, SB_G64S, SB_G64, SB_BLOCK, SB_GLOBAL, SB_N };
// Numeric bins by the exact row length.
enum : int8_t { NB_EMPTY = 0, NB_G4, NB_G8, NB_G16S, NB_G16, NB_G64S, NB_G64, NB_BLOCK4K, NB_BLOCK8K, NB_GLOBAL, NB_N };

// Visits the products of row `row` of A with B: for each A entry in
// ascending order, f(column, a_ik * b_kj) on the lanes holding the entries of
// B row k.  The A entries are loaded G at a time and broadcast by shuffles.
// The first lane-stride of the B rows of QB consecutive A entries is loaded
// in one batch, all loads in flight together, before any of them is visited,
// and the rest of a B row kChunks lane-strides at a time, so that a row costs
// a few memory latencies rather than one per A entry.  ORDERED puts a
// wave-scope barrier between A entries, so that the updates of one table slot
// happen in ascending k order.
constexpr int kChunks = 4;
template <int G, bool ORDERED, bool VALUES, class F>
__device__ inline void for_products(int32_t row, const int32_t *__restrict__ arp, const int32_t *__restrict__ aci,
                                    const double *__restrict__ av, const int32_t *__restrict__ brp,
                                    const int32_t *__restrict__ bci, const double *__restrict__ bv, F &&f) {
#pragma clang fp contract(off)
    constexpr int QB = 4;
    const int lane = group_lane<G>();
    const int32_t a0 = arp[row], a1 = arp[row + 1];
    for (int32_t kc = a0; kc < a1; kc += G) {
        const int32_t my = kc + lane;
        const bool in = my < a1;
        const int32_t kk = in ? aci[my] : 0;
        const double aa = VALUES && in ? av[my] : 0.0;
        const int32_t bb0 = in ? brp[kk] : 0, bb1 = in ? brp[kk + 1] : 0;
        const int nA = a1 - kc < G ? (int)(a1 - kc) : G;
        for (int q0 = 0; q0 < nA; q0 += QB) {
            int32_t kb[QB], b1[QB], cc[QB];
            double a[QB], vv[QB];
#pragma unroll
            for (int j = 0; j < QB; ++j) {
                const int q = q0 + j < nA ? q0 + j : nA - 1;
                b1[j] = __shfl(bb1, q, G);
                kb[j] = __shfl(bb0, q, G) + lane;
                a[j] = VALUES ? __shfl(aa, q, G) : 0.0;
                const bool ok = q0 + j < nA && kb[j] < b1[j];
                cc[j] = ok ? bci[kb[j]] : -1;
                vv[j] = VALUES && ok ? bv[kb[j]] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < QB; ++j) {
                if (q0 + j < nA) {
                    if (cc[j] >= 0) f(cc[j], a[j] * vv[j]);
                    // the rest of the B row, kChunks lane-strides at a time
                    for (int32_t k2 = kb[j] + G; k2 < b1[j]; k2 += kChunks * G) {
                        int32_t c2[kChunks];
                        double v2[kChunks];
#pragma unroll
                        for (int t = 0; t < kChunks; ++t) {
                            const int32_t e = k2 + t * G;
                            c2[t] = e < b1[j] ? bci[e] : -1;
                            v2[t] = VALUES && e < b1[j] ? bv[e] : 0.0;
                        }
#pragma unroll
                        for (int t = 0; t < kChunks; ++t)
                            if (c2[t] >= 0) f(c2[t], VALUES ? a[j] * v2[t] : 0.0);
                    }
                }
                if (ORDERED) lds_issue_order();
            }
        }
    }
}

// Staged visit for one wavefront per row (G = 64): the products of up to 64
// A entries at a time (at most kStage of them) are loaded into LDS first, all
// their loads in flight together, and then visited from LDS -- A entry by A
// entry, with a wave barrier between entries, when ORDERED.  An A entry whose
// B row alone exceeds the stage is visited straight from global memory.  The
// products and their order per table slot are those of for_products.
constexpr int kStage = 256;
template <bool VALUES>
struct ProdStage {
    int32_t c[kStage];
    double v[VALUES ? kStage : 1];
    int32_t off[65], b0[64];
    double a[64];
};

// Fills a product stage: product p < tot of the nq staged A entries is
// entry b0[j] + (p - off[j]) of B, with j the last entry whose off[j] <= p
// (off ascending from 0), scaled by a[j].  Each lane locates four of its
// products (a fixed six-step search) before issuing their loads together.
template <bool VALUES>
__device__ inline void stage_products(int lane, int nq, int32_t tot, const int32_t *off, const int32_t *b0,
                                      const double *a, const int32_t *__restrict__ bci,
                                      const double *__restrict__ bv, int32_t *sc, double *sv) {
#pragma clang fp contract(off)
    for (int32_t p0 = lane; p0 < tot; p0 += 4 * 64) {
        int32_t e[4], j4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t p = p0 + u * 64;
            int lo = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
                if (lo + step < nq && off[lo + step] <= p) lo += step;
            j4[u] = lo;
            e[u] = p < tot ? b0[lo] + (p - off[lo]) : -1;
        }
        int32_t c[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = e[u] >= 0 ? bci[e[u]] : 0;
            v[u] = VALUES && e[u] >= 0 ? bv[e[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t p = p0 + u * 64;
            if (p < tot) {
                sc[p] = c[u];
                if (VALUES) sv[p] = a[j4[u]] * v[u];
            }
        }
    }
}

template <bool ORDERED, bool VALUES, class F>
__device__ inline void for_products_staged(int32_t row, const int32_t *__restrict__ arp,
                                           const int32_t *__restrict__ aci, const double *__restrict__ av,
                                           const int32_t *__restrict__ brp, const int32_t *__restrict__ bci,
                                           const double *__restrict__ bv, ProdStage<VALUES> &S, F &&f) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int32_t a1 = arp[row + 1];
    for (int32_t q0 = arp[row]; q0 < a1;) {
        const int32_t q = q0 + lane;
        int32_t b0 = 0, len = 0;
        double a = 0.0;
        if (q < a1) {
            const int32_t k = aci[q];
            b0 = brp[k];
            len = brp[k + 1] - b0;
            if (VALUES) a = av[q];
        }
        int32_t x = len;   // inclusive scan of the B row lengths
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        const int nq = __popcll(__ballot(q < a1 && x <= kStage));   // a prefix of the lanes
        if (nq == 0) {
            const int32_t kb0 = __shfl(b0, 0, 64), kl = __shfl(len, 0, 64);
            const double ka = VALUES ? __shfl(a, 0, 64) : 0.0;
            for (int32_t t = lane; t < kl; t += 64) f(bci[kb0 + t], VALUES ? ka * bv[kb0 + t] : 0.0);
            wave_sync();
            q0 += 1;
            continue;
        }
        if (lane < nq) {
            S.off[lane] = x - len;
            S.b0[lane] = b0;
            if (VALUES) S.a[lane] = a;
        }
        const int32_t tot = __shfl(x, nq - 1, 64);
        if (lane == 0) S.off[nq] = tot;
        wave_sync();
        stage_products<VALUES>(lane, nq, tot, S.off, S.b0, S.a, bci, bv, S.c, S.v);
        wave_sync();
        if (ORDERED) {
            for (int j = 0; j < nq; ++j) {
                const int32_t o1 = S.off[j + 1];
                for (int32_t p = S.off[j] + lane; p < o1; p += 64) f(S.c[p], VALUES ? S.v[p] : 0.0);
                lds_issue_order();
            }
            wave_sync();
        } else {
            for (int32_t p = lane; p < tot; p += 64) f(S.c[p], VALUES ? S.v[p] : 0.0);
            wave_sync();
        }
        q0 += nq;
    }
}

// ub_i = sum over the A row of |B_k| by a G-lane group per row, and the
// row's symbolic bin.
template <int G>
__global__ void __launch_bounds__(256) k_spgemm_ub(int32_t m, const int32_t *__restrict__ arp,
                                                   const int32_t *__restrict__ aci,
                                                   const int32_t *__restrict__ brp, int32_t *__restrict__ ub,
                                                   int8_t *__restrict__ bin, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ kcnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(t / G);
    const int lane = group_lane<G>();
    if (i >= m) return;
    int64_t u = 0;
    for (int32_t k = arp[i] + lane; k < arp[i + 1]; k += G) {
        int32_t j = aci[k];
        u += brp[j + 1] - brp[j];
    }
    u = group_sum<G>(u);
    if (lane != 0) return;
    int32_t uc = u > 0x7fffffff ? 0x7fffffff : (int32_t)u;
    ub[i] = uc;
    cnt[i] = 0;    // the symbolic pass counts into it
    kcnt[i] = 0;   // a fused drop counts into it (rows with no product keep 0)
    bin[i] = uc == 0                            ? SB_EMPTY
             : uc <= 8                         ? SB_G4
             : uc <= 32                        ? SB_G8
             : uc <= 128                       ? SB_G16
             : uc <= 256                       ? SB_G32S
             : uc <= 512                       ? SB_G32
             : uc <= 1024                      ? SB_G64S
             : uc <= 2048                      ? SB_G64
             : uc <= 8192                      ? SB_BLOCK
                                               : SB_GLOBAL;
}

// Numeric bins by entry count, bin = number of thresholds below it: 0 (empty),
// <= 8, 32, 64, 128, 256, 512, 2048, 4096, longer (NB_EMPTY .. NB_GLOBAL).
static const BinRule kNumericBins{{0, 8, 32, 64, 128, 256, 512, 2048, 4096}, 9};

// ---------------------------------------------------------- group rows ----
// Symbolic: one G-lane group per row, T-slot key table per group; counts the
// distinct columns into cnt[row].
template <int G, int T, int TPB>
__global__ void __launch_bounds__(TPB) k_spgemm_count(const int32_t *__restrict__ list, int64_t count,
                                                      const int32_t *__restrict__ arp,
                                                      const int32_t *__restrict__ aci,
                                                      const int32_t *__restrict__ brp,
                                                      const int32_t *__restrict__ bci, int32_t *__restrict__ cnt) {
    constexpr int NG = TPB / G;
    __shared__ int32_t Ks[NG][T];
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t *keys = Ks[gid];
    for (int t = lane; t < T; t += G) keys[t] = kEmpty;
    wave_sync();
    int fresh_cnt = 0;
    auto ins = [&](int32_t c, double) {
        bool fresh;
        hash_insert(keys, T - 1, c, &fresh);
        fresh_cnt += fresh;
    };
    if constexpr (G == 64) {
        __shared__ ProdStage<false> St[NG];
        for_products_staged<false, false>(row, arp, aci, nullptr, brp, bci, nullptr, St[gid], ins);
    } else {
        for_products<G, false, false>(row, arp, aci, nullptr, brp, bci, nullptr, ins);
    }
    fresh_cnt = group_sum<G>(fresh_cnt);
    if (lane == 0) cnt[row] = fresh_cnt;
}

// Bitonic sort of a group's w entries (keys distinct) held in registers: lane
// l owns entries l*E .. l*E+E-1; exchanges within a lane are register
// compare-swaps, between lanes shuffles.  Pads (keys INT_MAX) sort last.
template <int E, int J>
__device__ inline void sort_in_lane(int32_t (&k)[E], double (&v)[E], int lane, int kk) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if ((e ^ J) > e) {
            const int p = e ^ J;
            bool up = ((lane * E + e) & kk) == 0;
            if ((k[e] > k[p]) == up) {
                int32_t tk = k[e];
                k[e] = k[p];
                k[p] = tk;
                double tv = v[e];
                v[e] = v[p];
                v[p] = tv;
            }
        }
    }
}

template <int G, int E>
__device__ inline void group_sort_store(const int32_t *keys, const double *vals, int w, int32_t *__restrict__ oci,
                                        double *__restrict__ ov, int32_t row, const DropArgs &D) {
    const int lane = group_lane<G>();
    int32_t k[E];
    double v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int i = lane * E + e;
        k[e] = i < w ? keys[i] : 0x7fffffff;
        v[e] = i < w ? vals[i] : 0.0;
    }
    constexpr int N = G * E;
    for (int kk = 2; kk <= N; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j < E) {
                if (j == 1) sort_in_lane<E, 1>(k, v, lane, kk);
                else if (j == 2) sort_in_lane<E, 2>(k, v, lane, kk);
                else sort_in_lane<E, 4>(k, v, lane, kk);
            } else {
                const int m = j / E;
                const bool lower = (lane & m) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    bool up = ((lane * E + e) & kk) == 0;
                    int32_t ok = __shfl_xor(k[e], m, G);
                    double oval = __shfl_xor(v[e], m, G);
                    bool take = lower == up ? ok < k[e] : ok > k[e];
                    if (take) {
                        k[e] = ok;
                        v[e] = oval;
                    }
                }
            }
        }
    }
    if (D.kcnt) {
        // lane l holds sorted entries l*E .. l*E+E-1: the kept ones, lane by
        // lane, are the row's kept entries in column order
        double mx = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (lane * E + e < w) mx = fmax(mx, fabs(v[e]));
        const double thr = D.tau * group_max<G>(mx);
        bool keep[E];
        int mine = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            keep[e] = lane * E + e < w && ((D.keep_diag && k[e] == row) || fabs(v[e]) >= thr);
            mine += keep[e];
        }
        int x = mine;   // inclusive scan of the kept counts over the group's lanes
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const int y = __shfl_up(x, o, G);
            if (lane >= o) x += y;
        }
        int pos = x - mine;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (keep[e]) {
                oci[pos] = k[e];
                ov[pos] = D.sign * v[e];
                ++pos;
            }
        }
        if (lane == G - 1) D.kcnt[row] = x;
        return;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int i = lane * E + e;
        if (i < w) {
            oci[i] = k[e];
            ov[i] = v[e];
        }
    }
}

// Sorts and stores with the least E (entries per lane) that holds w entries,
// among the widths up to EMAX.
template <int G, int EMAX>
__device__ inline void group_sort_store_upto(const int32_t *keys, const double *vals, int w,
                                             int32_t *__restrict__ oci, double *__restrict__ ov, int32_t row,
                                             const DropArgs &D) {
    if constexpr (EMAX > 1) {
        if (w > G * (EMAX / 2)) {
            group_sort_store<G, EMAX>(keys, vals, w, oci, ov, row, D);
            return;
        }
        group_sort_store_upto<G, EMAX / 2>(keys, vals, w, oci, ov, row, D);
    } else {
        group_sort_store<G, 1>(keys, vals, w, oci, ov, row, D);
    }
}

// Numeric: one G-lane group per row of known length w <= T/2.  The products
// are accumulated in a T-slot table; the occupied slots are then moved to the
// front of the table (in place, G slots at a time: a slot never moves to a
// higher index), sorted by column in registers, and the row is written out.
template <int G, int T, int TPB>
__global__ void __launch_bounds__(TPB) k_spgemm_fill(const int32_t *__restrict__ list, int64_t count,
                                                     const int32_t *__restrict__ arp,
                                                     const int32_t *__restrict__ aci,
                                                     const double *__restrict__ av,
                                                     const int32_t *__restrict__ brp,
                                                     const int32_t *__restrict__ bci,
                                                     const double *__restrict__ bv, const int32_t *__restrict__ crp,
                                                     int32_t *__restrict__ cci, double *__restrict__ cv, DropArgs D) {
#pragma clang fp contract(off)
    constexpr int NG = TPB / G;
    __shared__ int32_t Ks[NG][T];
    __shared__ double Vs[NG][T];
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t *keys = Ks[gid];
    double *vals = Vs[gid];
    for (int t = lane; t < T; t += G) {
        keys[t] = kEmpty;
        vals[t] = 0.0;
    }
    wave_sync();
    auto acc = [&](int32_t c, double p) {
        bool fresh;
        uint32_t s = hash_insert(keys, T - 1, c, &fresh);
        unsafeAtomicAdd(&vals[s], p);
    };
    if constexpr (G == 64) {
        __shared__ ProdStage<true> St[NG];
        for_products_staged<true, true>(row, arp, aci, av, brp, bci, bv, St[gid], acc);
    } else {
        for_products<G, true, true>(row, arp, aci, av, brp, bci, bv, acc);
    }
    wave_sync();
    int w = 0;
    for (int t0 = 0; t0 < T; t0 += G) {
        int32_t key = keys[t0 + lane];
        double val = vals[t0 + lane];
        bool occ = key != kEmpty;
        int tot;
        int pos = w + group_prefix<G>(occ, &tot);
        wave_sync();
        if (occ) {
            keys[pos] = key;
            vals[pos] = val;
        }
        wave_sync();
        w += tot;
    }
    int32_t base = crp[row];
    constexpr int EMAX = T / 2 / G < 1 ? 1 : T / 2 / G > 8 ? 8 : T / 2 / G;   // w <= T / 2
    group_sort_store_upto<G, EMAX>(keys, vals, w, cci + base, cv + base, row, D);
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
                                 int32_t *__restrict__ cci, double *__restrict__ cv, const DropArgs &D) {
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
    if (D.kcnt) {
        // the row's largest magnitude, then its kept entries packed in
        // column order: thread t takes a contiguous chunk of the sorted row
        __shared__ double shm[kBlk / 64];
        double mx = 0.0;
        for (int t = threadIdx.x; t < nz; t += kBlk) mx = fmax(mx, fabs(vals[t]));
        mx = group_max<64>(mx);
        if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = mx;
        __syncthreads();
        double m = 0.0;
        for (int q = 0; q < kBlk / 64; ++q) m = fmax(m, shm[q]);
        const double thr = D.tau * m;
        const int per2 = (nz + kBlk - 1) / kBlk;
        const int lo2 = (int)threadIdx.x * per2, hi2 = lo2 + per2 < nz ? lo2 + per2 : nz;
        int mine2 = 0;
        for (int t = lo2; t < hi2; ++t) mine2 += (D.keep_diag && keys[t] == row) || fabs(vals[t]) >= thr;
        int kept;
        int o2 = block_exclusive_count(mine2, &kept, sh);
        for (int t = lo2; t < hi2; ++t) {
            if ((D.keep_diag && keys[t] == row) || fabs(vals[t]) >= thr) {
                cci[base + o2] = keys[t];
                cv[base + o2] = D.sign * vals[t];
                ++o2;
            }
        }
        if (threadIdx.x == 0) D.kcnt[row] = kept;
        return;
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
                                                           double *__restrict__ cv, DropArgs D) {
    __shared__ int32_t keys[T];
    __shared__ double vals[NUMERIC ? T : 1];
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    spgemm_block_row<NUMERIC>(list[idx], keys, vals, T, arp, aci, av, brp, bci, bv, cnt, crp, cci, cv, D);
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
                                                              int32_t *__restrict__ cci, double *__restrict__ cv,
                                                              DropArgs D) {
    int64_t idx = blockIdx.x;
    if (idx >= count) return;
    int64_t o = toff[idx];
    uint32_t T = (uint32_t)(toff[idx + 1] - o);
    spgemm_block_row<NUMERIC>(list[idx], gkeys + o, NUMERIC ? gvals + o : nullptr, T, arp, aci, av, brp, bci, bv,
                              cnt, crp, cci, cv, D);
}

// -------------------------------------------------------- narrow rows ----
// When B has at most NC <= 4096 columns (the coarse levels), one wavefront
// builds a row of C in a dense accumulator of NC values and NC marks in LDS:
// no hashing, no sort (the marks are read out in ascending column order) and
// no row binning, so a product costs a count pass, a scan and a fill pass.
// The products of up to 64 A entries at a time are staged in LDS first, so
// that all their loads are in flight together; the fill pass then adds them
// in ascending k (one A entry per step, the lanes over its B row, whose
// columns are distinct) from 0.0 without contraction -- the same order and
// rounding as the hash-table kernels.
constexpr int kNarrowStage = 1024;

template <int NC, bool NUMERIC>
__global__ void __launch_bounds__(64) k_spgemm_narrow(int32_t m, const int32_t *__restrict__ arp,
                                                      const int32_t *__restrict__ aci,
                                                      const double *__restrict__ av,
                                                      const int32_t *__restrict__ brp,
                                                      const int32_t *__restrict__ bci,
                                                      const double *__restrict__ bv, int32_t *__restrict__ cnt,
                                                      const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                                      double *__restrict__ cv, DropArgs D) {
#pragma clang fp contract(off)
    __shared__ double acc[NUMERIC ? NC : 1];
    __shared__ uint8_t mark[NC];
    __shared__ int32_t sc[kNarrowStage];
    __shared__ double sv[NUMERIC ? kNarrowStage : 1];
    __shared__ int32_t qoff[65], qb0[64];
    __shared__ double qa[64];
    const int lane = threadIdx.x;
    const int32_t row = blockIdx.x;
    if (row >= m) return;
    for (int c = lane; c < NC; c += 64) {
        mark[c] = 0;
        if (NUMERIC) acc[c] = 0.0;
    }
    wave_sync();
    const int32_t a1 = arp[row + 1];
    for (int32_t q0 = arp[row]; q0 < a1;) {
        const int32_t q = q0 + lane;
        int32_t b0 = 0, len = 0;
        double a = 0.0;
        if (q < a1) {
            const int32_t k = aci[q];
            b0 = brp[k];
            len = brp[k + 1] - b0;
            if (NUMERIC) a = av[q];
        }
        int32_t x = len;   // inclusive scan of the B row lengths over the lanes
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        // entries taken now: the prefix whose products fit the stage (x is
        // nondecreasing, so the ballot is a prefix of the lanes)
        const int nq = __popcll(__ballot(q < a1 && x <= kNarrowStage));
        if (nq == 0) {
            // the first entry's B row alone exceeds the stage: read it directly
            const int32_t kb0 = __shfl(b0, 0, 64), kl = __shfl(len, 0, 64);
            const double ka = __shfl(a, 0, 64);
            for (int32_t t = lane; t < kl; t += 64) {
                const int32_t c = bci[kb0 + t];
                if ((uint32_t)c >= (uint32_t)NC) continue;   // columns beyond B's width are not stored
                mark[c] = 1;
                if (NUMERIC) unsafeAtomicAdd(&acc[c], ka * bv[kb0 + t]);
            }
            wave_sync();
            q0 += 1;
            continue;
        }
        if (lane < nq) {
            qoff[lane] = x - len;
            qb0[lane] = b0;
            if (NUMERIC) qa[lane] = a;
        }
        const int32_t tot = __shfl(x, nq - 1, 64);
        if (lane == 0) qoff[nq] = tot;
        wave_sync();
        stage_products<NUMERIC>(lane, nq, tot, qoff, qb0, qa, bci, bv, sc, sv);
        wave_sync();
        if (NUMERIC) {
            for (int j = 0; j < nq; ++j) {
                const int32_t o1 = qoff[j + 1];
                for (int32_t p = qoff[j] + lane; p < o1; p += 64) {
                    const int32_t c = sc[p];
                    if ((uint32_t)c >= (uint32_t)NC) continue;
                    mark[c] = 1;
                    unsafeAtomicAdd(&acc[c], sv[p]);
                }
                lds_issue_order();
            }
            wave_sync();
        } else {
            for (int32_t p = lane; p < tot; p += 64)
                if ((uint32_t)sc[p] < (uint32_t)NC) mark[sc[p]] = 1;
            wave_sync();
        }
        q0 += nq;
    }
    const int32_t base = NUMERIC ? crp[row] : 0;
    double thr = 0.0;
    if (NUMERIC && D.kcnt) {   // the row's largest magnitude, for the fused drop
        double mx = 0.0;
        for (int c = lane; c < NC; c += 64)
            if (mark[c]) mx = fmax(mx, fabs(acc[c]));
        thr = D.tau * group_max<64>(mx);
    }
    int32_t w = 0;
    for (int c0 = 0; c0 < NC; c0 += 64) {
        const int c = c0 + lane;
        bool occ = mark[c] != 0;
        if (NUMERIC && D.kcnt) occ = occ && ((D.keep_diag && c == row) || fabs(acc[c]) >= thr);
        const uint64_t bm = __ballot(occ);
        if (NUMERIC && occ) {
            const int32_t pos = w + __popcll(bm & ((1ull << lane) - 1ull));
            cci[base + pos] = c;
            cv[base + pos] = D.kcnt ? D.sign * acc[c] : acc[c];
        }
        w += __popcll(bm);
    }
    if (!NUMERIC && lane == 0) cnt[row] = w;
    if (NUMERIC && D.kcnt && lane == 0) D.kcnt[row] = w;
}

constexpr int32_t kNarrowMaxCols = 4096;
constexpr int64_t kNarrowMaxWork = (int64_t)1 << 24;   // rows x NC: the accumulator sweeps per product

template <int NC>
static Csr spgemm_narrow(const CsrView &A, const CsrView &Bm, hipStream_t s, const DropArgs &D) {
    Csr C;
    C.nr = A.nr;
    C.nc = Bm.nc;
    const int32_t m = A.nr;
    C.rp.alloc((size_t)m + 1, s);
    DBuf<int32_t> cnt((size_t)m + 1, s);
    if (m > 0) {
        k_spgemm_narrow<NC, false><<<(unsigned)m, 64, 0, s>>>(m, A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt.p,
                                                                nullptr, nullptr, nullptr, DropArgs{});
        AIRG_LAUNCH_CHECK();
    }
    C.nnz = exclusive_scan(cnt.p, C.rp.p, m, s);
    C.ci.alloc((size_t)C.nnz, s);
    C.v.alloc((size_t)C.nnz, s);
    if (C.nnz > 0) {
        k_spgemm_narrow<NC, true><<<(unsigned)m, 64, 0, s>>>(m, A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, nullptr,
                                                               C.rp.p, C.ci.p, C.v.p, D);
        AIRG_LAUNCH_CHECK();
    } else if (D.kcnt && m > 0) {
        fill_zero(D.kcnt, (size_t)m * sizeof(int32_t), s);   // no fill pass to count the kept entries
    }
    return C;
}

// ------------------------------------------------------------------ host --
static uint32_t pow2_at_least(int64_t v) {
    uint32_t p = 1;
    while ((int64_t)p < v) p <<= 1;
    return p;
}

// ------------------------------------------------------- fixed pattern ---
// Values of sign * (A B) on a given pattern: out[e] for each stored (i, j) of
// row i of the pattern.  One G-lane group per row stages the pattern row in
// LDS; every product finds its column there by binary search (products off
// the pattern are skipped) and is accumulated in ascending k from 0.0 without
// contraction -- the same order and rounding as the two-pass product, so the
// values equal those of the full product at the pattern's positions.
template <int G, int L, int TPB>
__global__ void __launch_bounds__(TPB) k_spgemm_on_pattern(const int32_t *__restrict__ list, int64_t count,
                                                           const int32_t *__restrict__ arp,
                                                           const int32_t *__restrict__ aci,
                                                           const double *__restrict__ av,
                                                           const int32_t *__restrict__ brp,
                                                           const int32_t *__restrict__ bci,
                                                           const double *__restrict__ bv,
                                                           const int32_t *__restrict__ prp,
                                                           const int32_t *__restrict__ pci, double sign,
                                                           double *__restrict__ out) {
#pragma clang fp contract(off)
    constexpr int NG = TPB / G;
    __shared__ int32_t Cs[NG][L];
    __shared__ double Vs[NG][L];
    int gid = threadIdx.x / G;
    int lane = group_lane<G>();
    int64_t idx = (int64_t)blockIdx.x * NG + gid;
    if (idx >= count) return;
    int32_t row = list[idx];
    int32_t *cols = Cs[gid];
    double *vals = Vs[gid];
    const int32_t p0 = prp[row];
    const int len = prp[row + 1] - p0;
    for (int t = lane; t < len; t += G) {
        cols[t] = pci[p0 + t];
        vals[t] = 0.0;
    }
    wave_sync();
    auto acc = [&](int32_t c, double p) {
        int lo = 0, hi = len;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (cols[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        if (lo < len && cols[lo] == c) unsafeAtomicAdd(&vals[lo], p);
    };
    if constexpr (G == 64) {
        __shared__ ProdStage<true> St[NG];
        for_products_staged<true, true>(row, arp, aci, av, brp, bci, bv, St[gid], acc);
    } else {
        for_products<G, true, true>(row, arp, aci, av, brp, bci, bv, acc);
    }
    wave_sync();
    for (int t = lane; t < len; t += G) out[p0 + t] = sign * vals[t];
}

__global__ void k_pattern_bin(int32_t m, const int32_t *__restrict__ prp, int8_t *__restrict__ bin) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t L = prp[i + 1] - prp[i];
    bin[i] = L == 0 ? 0 : L <= 16 ? 1 : L <= 64 ? 2 : L <= 256 ? 3 : L <= 1024 ? 4 : L <= 4096 ? 5 : 6;
}

Bins pattern_bins(const Csr &Pt, hipStream_t s) {
    const int32_t m = Pt.nr;
    DBuf<int8_t> bin((size_t)std::max<int32_t>(m, 1), s);
    if (m > 0) {
        k_pattern_bin<<<grid_for(m, 256), 256, 0, s>>>(m, Pt.rp.p, bin.p);
        AIRG_LAUNCH_CHECK();
    }
    Bins B = bin_rows(bin.p, m, 8, s);
    AIRG_REQUIRE(B.count(6) == 0, ST_LIMIT, "pattern row longer than 4096 entries");
    return B;
}

void spgemm_on_pattern_binned(const CsrView &A, const CsrView &Bm, const CsrView &Pt, const Bins &B, double sign,
                              double *out_v, hipStream_t s) {
    AIRG_REQUIRE(A.nc == Bm.nr && Pt.nr == A.nr, ST_INVALID_ARG, "pattern product dimensions differ");
    if (A.nr == 0 || Pt.nnz == 0) return;
    auto grp = [&](auto kern, int b, int rows_per_block, unsigned tpb) {
        if (B.count(b))
            kern<<<grid_for(B.count(b), rows_per_block), tpb, 0, s>>>(B.list(b), B.count(b), A.rp, A.ci, A.v, Bm.rp,
                                                                      Bm.ci, Bm.v, Pt.rp, Pt.ci, sign, out_v);
    };
    grp(k_spgemm_on_pattern<4, 16, 256>, 1, 64, 256);
    grp(k_spgemm_on_pattern<8, 64, 256>, 2, 32, 256);
    grp(k_spgemm_on_pattern<16, 256, 128>, 3, 8, 128);
    grp(k_spgemm_on_pattern<64, 1024, 64>, 4, 1, 64);
    grp(k_spgemm_on_pattern<64, 4096, 64>, 5, 1, 64);
    AIRG_LAUNCH_CHECK();
}

void spgemm_on_pattern(const CsrView &A, const CsrView &Bm, const Csr &Pt, double sign, double *out_v,
                       hipStream_t s) {
    AIRG_REQUIRE(A.nc == Bm.nr && Pt.nr == A.nr, ST_INVALID_ARG, "pattern product dimensions differ");
    if (A.nr == 0 || Pt.nnz == 0) return;
    Bins B = pattern_bins(Pt, s);
    spgemm_on_pattern_binned(A, Bm, view(Pt), B, sign, out_v, s);
}

static void run_global(bool numeric, const Bins &B, int b, const std::vector<int32_t> &per_row, const CsrView &A,
                       const CsrView &Bm, int32_t *cnt, const int32_t *crp, int32_t *cci, double *cv, hipStream_t s,
                       const DropArgs &D = DropArgs{}) {
    // one table of 2 x per_row[r] slots (rounded up to a power of two) per row
    std::vector<int64_t> off(per_row.size() + 1, 0);
    for (size_t r = 0; r < per_row.size(); ++r) off[r + 1] = off[r] + pow2_at_least(2 * (int64_t)per_row[r]);
    DBuf<int64_t> toff(off.size(), s);
    h2d(toff.p, off.data(), off.size(), s);
    DBuf<int32_t> gk((size_t)off.back(), s);
    DBuf<double> gv(numeric ? (size_t)off.back() : 1, s);
    if (numeric)
        k_spgemm_block_global<true><<<(unsigned)B.count(b), kBlk, 0, s>>>(
            B.list(b), B.count(b), toff.p, gk.p, gv.p, A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv, D);
    else
        k_spgemm_block_global<false><<<(unsigned)B.count(b), kBlk, 0, s>>>(
            B.list(b), B.count(b), toff.p, gk.p, gv.p, A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv,
            DropArgs{});
    AIRG_LAUNCH_CHECK();
}

// per-row values of v at the rows of bin b (host copy)
static std::vector<int32_t> gather_bin(const Bins &B, int b, const int32_t *v, int32_t m, hipStream_t s) {
    std::vector<int32_t> rows((size_t)B.count(b)), h((size_t)m), out(rows.size());
    d2h(rows.data(), B.list(b), rows.size(), s);
    d2h(h.data(), v, (size_t)m, s);
    for (size_t r = 0; r < rows.size(); ++r) out[r] = h[rows[r]];
    return out;
}

static void run_symbolic(const Bins &B, const CsrView &A, const CsrView &Bm, int32_t *cnt, const int32_t *ub,
                         int32_t m, hipStream_t s) {
    auto grp = [&](auto kern, int b, int rows_per_block, unsigned tpb) {
        if (B.count(b))
            kern<<<grid_for(B.count(b), rows_per_block), tpb, 0, s>>>(B.list(b), B.count(b), A.rp, A.ci, Bm.rp,
                                                                      Bm.ci, cnt);
    };
    grp(k_spgemm_count<4, 16, 256>, SB_G4, 64, 256);
    grp(k_spgemm_count<8, 64, 256>, SB_G8, 32, 256);
    grp(k_spgemm_count<16, 256, 256>, SB_G16, 16, 256);
    grp(k_spgemm_count<32, 512, 256>, SB_G32S, 8, 256);
    grp(k_spgemm_count<32, 1024, 256>, SB_G32, 8, 256);
    grp(k_spgemm_count<64, 2048, 128>, SB_G64S, 2, 128);
    grp(k_spgemm_count<64, 4096, 128>, SB_G64, 2, 128);
    if (B.count(SB_BLOCK))
        k_spgemm_block_lds<16384, false><<<(unsigned)B.count(SB_BLOCK), kBlk, 0, s>>>(
            B.list(SB_BLOCK), B.count(SB_BLOCK), A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, nullptr, nullptr, nullptr,
            DropArgs{});
    AIRG_LAUNCH_CHECK();
    if (B.count(SB_GLOBAL))
        run_global(false, B, SB_GLOBAL, gather_bin(B, SB_GLOBAL, ub, m, s), A, Bm, cnt, nullptr, nullptr, nullptr, s);
}

static void run_numeric(const Bins &B, const CsrView &A, const CsrView &Bm, int32_t *cnt, const int32_t *crp,
                        int32_t *cci, double *cv, int32_t m, hipStream_t s, const DropArgs &D) {
    auto grp = [&](auto kern, int b, int rows_per_block, unsigned tpb) {
        if (B.count(b))
            kern<<<grid_for(B.count(b), rows_per_block), tpb, 0, s>>>(B.list(b), B.count(b), A.rp, A.ci, A.v,
                                                                      Bm.rp, Bm.ci, Bm.v, crp, cci, cv, D);
    };
    grp(k_spgemm_fill<4, 16, 256>, NB_G4, 64, 256);
    grp(k_spgemm_fill<8, 64, 256>, NB_G8, 32, 256);
    grp(k_spgemm_fill<16, 128, 128>, NB_G16S, 8, 128);
    grp(k_spgemm_fill<16, 256, 128>, NB_G16, 8, 128);
    grp(k_spgemm_fill<64, 512, 64>, NB_G64S, 1, 64);
    grp(k_spgemm_fill<64, 1024, 64>, NB_G64, 1, 64);
    if (B.count(NB_BLOCK4K))
        k_spgemm_block_lds<4096, true><<<(unsigned)B.count(NB_BLOCK4K), kBlk, 0, s>>>(
            B.list(NB_BLOCK4K), B.count(NB_BLOCK4K), A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv, D);
    if (B.count(NB_BLOCK8K))
        k_spgemm_block_lds<8192, true><<<(unsigned)B.count(NB_BLOCK8K), kBlk, 0, s>>>(
            B.list(NB_BLOCK8K), B.count(NB_BLOCK8K), A.rp, A.ci, A.v, Bm.rp, Bm.ci, Bm.v, cnt, crp, cci, cv, D);
    AIRG_LAUNCH_CHECK();
    if (B.count(NB_GLOBAL))
        run_global(true, B, NB_GLOBAL, gather_bin(B, NB_GLOBAL, cnt, m, s), A, Bm, cnt, crp, cci, cv, s, D);
}

static bool narrow_shape(int32_t m, int32_t bnc, int *nc) {
    if (bnc > kNarrowMaxCols) return false;
    *nc = bnc <= 1024 ? 1024 : bnc <= 2048 ? 2048 : 4096;
    return (int64_t)m * *nc <= kNarrowMaxWork;
}

std::pair<const int32_t *, int32_t> SpgemmPlan::totals() const {
    if (narrow) return {nullptr, 0};
    return {bins.tot.p, SB_N + 1};
}

SpgemmPlan spgemm_begin(const CsrView &A, const int32_t *b_rp, int32_t b_nc, hipStream_t s) {
    SpgemmPlan P;
    P.m = A.nr;
    P.bnc = b_nc;
    int nc;
    P.narrow = narrow_shape(A.nr, b_nc, &nc);
    if (P.narrow) return P;
    const int32_t m = A.nr;
    P.ub.alloc((size_t)m + 1, s);
    P.sbin.alloc((size_t)m + 1, s);
    P.cnt.alloc((size_t)m + 1, s);
    P.kcnt.alloc((size_t)m + 1, s);
    if (m > 0) {
        dispatch_group(lanes_for(A.nnz, m), [&]<int G>() {
            k_spgemm_ub<G><<<grid_for((int64_t)m * G, 256), 256, 0, s>>>(m, A.rp, A.ci, b_rp, P.ub.p, P.sbin.p, P.cnt.p,
                                                                        P.kcnt.p);
        });
        AIRG_LAUNCH_CHECK();
    }
    P.bins = bin_rows_begin(P.sbin.p, m, SB_N, s);
    return P;
}

Csr spgemm_finish(const CsrView &A, const CsrView &Bm, SpgemmPlan &P, const int32_t *h_tot, hipStream_t s,
                  const DropArgs *drop) {
    AIRG_REQUIRE(A.nc == Bm.nr && P.m == A.nr && P.bnc == Bm.nc, ST_INVALID_ARG, "product plan does not match");
    DropArgs D;
    if (drop) {
        D = *drop;
        if (!P.kcnt.p) P.kcnt.alloc((size_t)A.nr + 1, s);   // narrow plans: every row is filled, no clearing
        D.kcnt = P.kcnt.p;
    }
    if (P.narrow) {
        int nc;
        narrow_shape(A.nr, Bm.nc, &nc);
        if (nc == 1024) return spgemm_narrow<1024>(A, Bm, s, D);
        if (nc == 2048) return spgemm_narrow<2048>(A, Bm, s, D);
        return spgemm_narrow<4096>(A, Bm, s, D);
    }
    Csr C;
    C.nr = A.nr;
    C.nc = Bm.nc;
    C.rp.alloc((size_t)A.nr + 1, s);
    int32_t m = A.nr;
    DBuf<int32_t> &cnt = P.cnt;   // zeroed by the plan's bound pass
    DBuf<int8_t> nbin((size_t)m + 1, s);
    Bins SB = bin_rows_end(P.bins, h_tot, s);
    run_symbolic(SB, A, Bm, cnt.p, P.ub.p, m, s);
    exclusive_scan(cnt.p, C.rp.p, m, s, false);
    // nnz and the numeric bin starts come back in one readback
    BinPlan NP = bin_rows_begin_rule(cnt.p, false, kNumericBins, nbin.p, m, NB_N, s);
    std::vector<int32_t> h(NB_N + 2);
    read_ints({C.rp.p + m, NP.tot.p}, {1, NB_N + 1}, h.data(), s);
    AIRG_REQUIRE(h[0] >= 0, ST_LIMIT, "product exceeds the int32 index range");
    C.nnz = h[0];
    C.ci.alloc((size_t)C.nnz, s);
    C.v.alloc((size_t)C.nnz, s);
    if (C.nnz == 0) return C;
    Bins NB = bin_rows_end(NP, h.data() + 1, s);
    run_numeric(NB, A, Bm, cnt.p, C.rp.p, C.ci.p, C.v.p, m, s, D);
    return C;
}

// Row r's first kcnt[r] entries of C moved to its place in the packed matrix.
template <int G>
__global__ void __launch_bounds__(256) k_drop_pack(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   const int32_t *__restrict__ orp, int32_t *__restrict__ oci,
                                                   double *__restrict__ ov) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t row = (int32_t)(t / G);
    const int lane = group_lane<G>();
    if (row >= n) return;
    const int32_t b = rp[row], w = orp[row], kept = orp[row + 1] - w;
    for (int32_t k = lane; k < kept; k += G) {
        oci[w + k] = ci[b + k];
        ov[w + k] = v[b + k];
    }
}

Csr drop_compact(const Csr &C, const int32_t *kcnt, bool bound, hipStream_t s) {
    Csr B;
    B.nr = C.nr;
    B.nc = C.nc;
    B.rp.alloc((size_t)C.nr + 1, s);
    if (bound) {
        exclusive_scan(kcnt, B.rp.p, C.nr, s, false);
        B.nnz = C.nnz;
    } else {
        B.nnz = exclusive_scan(kcnt, B.rp.p, C.nr, s);
    }
    B.ci.alloc((size_t)B.nnz, s);
    B.v.alloc((size_t)B.nnz, s);
    if (C.nr > 0 && C.nnz > 0) {
        dispatch_group(lanes_for(C.nnz, C.nr), [&]<int G>() {
            k_drop_pack<G><<<grid_for((int64_t)C.nr * G, 256), 256, 0, s>>>(C.nr, C.rp.p, C.ci.p, C.v.p, B.rp.p,
                                                                            B.ci.p, B.v.p);
        });
        AIRG_LAUNCH_CHECK();
    }
    return B;
}

Csr spgemm_drop(const CsrView &A, const CsrView &Bm, const DropArgs &drop, hipStream_t s, int64_t *product_nnz) {
    AIRG_REQUIRE(A.nc == Bm.nr, ST_INVALID_ARG, "inner dimensions differ");
    SpgemmPlan P = spgemm_begin(A, Bm.rp, Bm.nc, s);
    auto [src, cnt] = P.totals();
    std::vector<int32_t> h((size_t)std::max(cnt, 1));
    if (cnt > 0) d2h(h.data(), src, (size_t)cnt, s);
    Csr C = spgemm_finish(A, Bm, P, h.data(), s, &drop);
    if (product_nnz) *product_nnz = C.nnz;
    return drop_compact(C, P.kcnt.p, false, s);
}

Csr spgemm(const CsrView &A, const CsrView &Bm, hipStream_t s) {
    AIRG_REQUIRE(A.nc == Bm.nr, ST_INVALID_ARG, "inner dimensions differ");
    SpgemmPlan P = spgemm_begin(A, Bm.rp, Bm.nc, s);
    auto [src, cnt] = P.totals();
    std::vector<int32_t> h((size_t)std::max(cnt, 1));
    if (cnt > 0) d2h(h.data(), src, (size_t)cnt, s);
    return spgemm_finish(A, Bm, P, h.data(), s);
}

}  // namespace airg

// CF splitting kernels for gfx950: strength of connection and degrees in
// S u S^T, PMISR rounds decided with wavefront ballots (push/pull over the
// rows of S), and the DDC diagonal-dominance scan with a fixed summation
// order.
#include <cmath>
#include <mutex>

#include "cfsplit.hpp"
#include "csr.hpp"
#include "group.hpp"

namespace airg {

// ------------------------------------------------------------- strength ---
// Marks the strong entries, counts them per row, and clears the row's S^T
// count for the pass after it.
template <int G>
__global__ void __launch_bounds__(256) k_strength(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  double alpha, uint8_t *__restrict__ strong,
                                                  int32_t *__restrict__ cntS, int32_t *__restrict__ cntT) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    int32_t b = rp[row], e = rp[row + 1];
    double M = 0.0;
    for (int32_t k = b + lane; k < e; k += G)
        if (ci[k] != row) M = fmax(M, fabs(v[k]));
    M = group_max<G>(M);          // order-free, exact
    double thr = alpha * M;       // one correctly rounded product
    int32_t c = 0;
    for (int32_t k = b + lane; k < e; k += G) {
        double a = fabs(v[k]);
        bool st = ci[k] != row && a > 0.0 && a >= thr;
        strong[k] = st;
        c += st;
    }
    c = group_sum<G>(c);
    if (lane == 0) {
        cntS[row] = c;
        cntT[row] = 0;
    }
}

// Per strong entry (i, j): write it to row i of S's own CSR, count it for
// S^T_j, and find whether i in S_j to count mutual pairs: a row j of up to
// kMutualScan entries is read whole (its loads issued together, one trip to
// memory), a longer one is searched by bisection (its columns ascend).
constexpr int kMutualScan = 8;
template <int G>
__global__ void __launch_bounds__(256) k_strength_mutual(int32_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const uint8_t *__restrict__ strong,
                                                         const int32_t *__restrict__ srp, int32_t *__restrict__ sci,
                                                         int32_t *__restrict__ cntT, int32_t *__restrict__ mutual) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    int32_t mu = 0;
    const int32_t b = rp[row], e = rp[row + 1];
    int32_t w = srp[row];
    for (int32_t base = b; base < e; base += G) {
        const int32_t k = base + lane;
        const bool st = k < e && strong[k];
        const uint64_t m = group_ballot<G>(st);
        if (st) {
            const int32_t j = ci[k];
            sci[w + __popcll(m & ((1ull << lane) - 1ull))] = j;
            atomicAdd(&cntT[j], 1);
            const int32_t jb = rp[j], je = rp[j + 1];
            int32_t pos = -1;
            if (je - jb <= kMutualScan) {
                int32_t c[kMutualScan];
#pragma unroll
                for (int u = 0; u < kMutualScan; ++u) c[u] = jb + u < je ? ci[jb + u] : -1;
#pragma unroll
                for (int u = 0; u < kMutualScan; ++u) pos = c[u] == row ? jb + u : pos;
            } else {
                int32_t lo = jb, hi = je;
                while (lo < hi) {
                    int32_t mid = (lo + hi) >> 1;
                    if (ci[mid] < row) lo = mid + 1;
                    else hi = mid;
                }
                pos = lo < je && ci[lo] == row ? lo : -1;
            }
            if (pos >= 0 && strong[pos]) ++mu;
        }
        w += __popcll(m);
    }
    mu = group_sum<G>(mu);
    if (lane == 0) mutual[row] = mu;
}

// |S_i u S_i^T| = |S_i| + |S_i^T| - |S_i n S_i^T|
__device__ inline int32_t strength_degree_of(const int32_t *__restrict__ srp, const int32_t *__restrict__ cntT,
                                             const int32_t *__restrict__ mutual, int32_t i) {
    return srp[i + 1] - srp[i] + cntT[i] - mutual[i];
}

__global__ void k_degree(int32_t n, const int32_t *__restrict__ srp, const int32_t *__restrict__ cntT,
                         const int32_t *__restrict__ mutual, int32_t *__restrict__ deg) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) deg[i] = strength_degree_of(srp, cntT, mutual, i);
}

void strength_degree(const StrengthGraph &G, int32_t *deg, hipStream_t s) {
    if (G.n <= 0) return;
    k_degree<<<grid_for(G.n, 256), 256, 0, s>>>(G.n, G.srp.p, G.cntT.p, G.mutual.p, deg);
    AIRG_LAUNCH_CHECK();
}

StrengthGraph strength_graph(const CsrView &A, double alpha, hipStream_t s) {
    StrengthGraph G;
    int32_t n = A.nr;
    G.n = n;
    G.strong.alloc((size_t)A.nnz, s);
    G.srp.alloc((size_t)n + 1, s);
    G.sci.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);   // S's size is not read back: room for all of A
    G.cntT.alloc((size_t)n, s);
    G.mutual.alloc((size_t)n, s);
    DBuf<int32_t> cntS((size_t)n, s);
    int32_t *cntT = G.cntT.p, *mutual = G.mutual.p;
    int g = lanes_for(A.nnz, n);
    const unsigned grid = grid_for((int64_t)n * g, 256);
    dispatch_group(g, [&]<int W>() {
        k_strength<W><<<grid, 256, 0, s>>>(n, A.rp, A.ci, A.v, alpha, G.strong.p, cntS.p, cntT);
    });
    AIRG_LAUNCH_CHECK();
    exclusive_scan(cntS.p, G.srp.p, n, s, false);
    dispatch_group(g, [&]<int W>() {
        k_strength_mutual<W><<<grid, 256, 0, s>>>(n, A.rp, A.ci, G.strong.p, G.srp.p, G.sci.p, cntT, mutual);
    });
    AIRG_LAUNCH_CHECK();
    return G;
}

// ---------------------------------------------------------------- PMISR ---
__device__ inline uint32_t pmisr_hash_of(uint64_t seed, int32_t level, int64_t i) {
    return (uint32_t)(splitmix64(rng_counter(seed, 0, (uint32_t)level, (uint64_t)i)) >> 32);
}

// Batch segments: row i of segment p draws with p's seed at its index within
// the segment, exactly as in a setup of that segment alone.
__global__ void k_pmisr_hash_seg(int32_t n, const int32_t *__restrict__ off, int nseg,
                                 const uint64_t *__restrict__ seeds, int32_t level, uint32_t *__restrict__ h) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = seg_of(off, nseg, i);
    h[i] = pmisr_hash_of(seeds[p], level, i - off[p]);
}

void pmisr_hash_seg(int32_t n, const int32_t *off, int nseg, const uint64_t *seeds, int32_t level, uint32_t *h,
                    hipStream_t s) {
    if (n <= 0) return;
    k_pmisr_hash_seg<<<grid_for(n, 256), 256, 0, s>>>(n, off, nseg, seeds, level, h);
    AIRG_LAUNCH_CHECK();
}

// Measure order: (deg, h, index) lexicographic -- the integer form of
// w = deg + rand(0,1) with the index breaking exact ties.
__device__ inline bool key_less(int32_t dj, uint32_t hj, int32_t j, int32_t di, uint32_t hi, int32_t i) {
    if (dj != di) return dj < di;
    if (hj != hi) return hj < hi;
    return j < i;
}

// Per-node key for the rounds: (deg << 32) | h while unassigned, so that the
// unsigned order of keys is the (deg, h) order above, and kAssigned once the
// node has joined F or C -- a neighbour's state and measure are then one
// 8-byte load.  kAssigned exceeds every unassigned key (deg < 2^31).
constexpr uint64_t kAssigned = ~0ull;

// Keys from the degrees; the measures h come from memory, or with h null
// from the generator for (seed, level), as pmisr_hash_of draws them.
__global__ void k_pmisr_init(int32_t n, const int32_t *__restrict__ srp, const int32_t *__restrict__ cntT,
                             const int32_t *__restrict__ mutual, const uint32_t *__restrict__ h, uint64_t seed,
                             int32_t level, int8_t *__restrict__ cf, uint64_t *__restrict__ key,
                             uint8_t *__restrict__ beaten, uint8_t *__restrict__ markC) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t deg = strength_degree_of(srp, cntT, mutual, i);
    const bool isolated = deg == 0;
    const uint32_t hi = h ? h[i] : pmisr_hash_of(seed, level, i);
    cf[i] = isolated ? CF_F : CF_U;
    key[i] = isolated ? kAssigned : ((uint64_t)(uint32_t)deg << 32) | hi;
    beaten[i] = 0;
    markC[i] = 0;
}

// Neighbour j (key kj) beats node i (key ki, unassigned): j is unassigned
// and key_less(j, i).
__device__ inline bool beats(uint64_t kj, int32_t j, uint64_t ki, int32_t i) {
    return kj < ki || (kj == ki && j < i);
}

// Rounds in push/pull form over the rows of S only (S^T is never formed).
// A round's independent set D holds the unassigned nodes that no unassigned
// neighbour in S_i u S_i^T beats, taken from the state at the start of the
// round; then D joins F and the unassigned nodes with a neighbour in D join C.
// Neighbours j in S_i are read from row i (pull); a node j with i in S_j
// reaches i through its own row (push), by setting a flag that i consumes and
// clears:
//   beaten[i]: some unassigned j with i in S_j beats i (pushed before the round);
//   markC[x]:  some y in D has x in S_y (pushed by y during the round).
// Several pushers store the same 1, so the flags do not depend on the order.

// Pushes for the first round.
template <int G>
__global__ void __launch_bounds__(256) k_pmisr_push(int32_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const uint64_t *__restrict__ key, uint8_t *__restrict__ beaten) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    const uint64_t kj = key[row];
    if (kj == kAssigned) return;
    for (int32_t k = rp[row] + lane; k < rp[row + 1]; k += G) {
        const int32_t i = ci[k];
        if (beats(kj, row, key[i], i)) beaten[i] = 1;
    }
}

// Selection: inD[i] for every node; a node of D pushes markC along its row.
template <int G>
__global__ void __launch_bounds__(256) k_pmisr_select(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const uint64_t *__restrict__ key,
                                                      uint8_t *__restrict__ beaten, uint8_t *__restrict__ inD,
                                                      uint8_t *__restrict__ markC, int32_t *__restrict__ nu) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    const uint64_t ki = key[row];
    if (ki == kAssigned) {
        if (lane == 0) inD[row] = 0;
        return;
    }
    if (nu && lane == 0) atomicAdd(nu, 1);   // unassigned at the start of the round
    bool lost = beaten[row] != 0;
    const int32_t b = rp[row], e = rp[row + 1];
    for (int32_t base = b; base < e && !lost; base += G) {
        int32_t k = base + lane;
        bool lose = false;
        if (k < e) {
            int32_t j = ci[k];
            lose = beats(key[j], j, ki, row);
        }
        lost = group_any<G>(lose);
    }
    if (lane == 0) {
        beaten[row] = 0;
        inD[row] = !lost;
    }
    if (!lost)
        for (int32_t k = b + lane; k < e; k += G) markC[ci[k]] = 1;
}

// Update: D joins F; an unassigned node with a neighbour in D joins C; a node
// still unassigned pushes beaten along its row for the next round, or, after
// the last of a fixed number of rounds (LAST), joins C.
template <int G>
__global__ void __launch_bounds__(256) k_pmisr_update(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const uint8_t *__restrict__ inD, int8_t *__restrict__ cf,
                                                      uint64_t *__restrict__ key, uint8_t *__restrict__ markC,
                                                      uint8_t *__restrict__ beaten, int last) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    const uint64_t kx = key[row];
    if (kx == kAssigned) return;
    if (inD[row]) {
        if (lane == 0) {
            cf[row] = CF_F;
            key[row] = kAssigned;
        }
        return;
    }
    bool hit = markC[row] != 0;
    const int32_t b = rp[row], e = rp[row + 1];
    for (int32_t base = b; base < e && !hit; base += G) {
        int32_t k = base + lane;
        bool p = k < e && inD[ci[k]];
        hit = group_any<G>(p);
    }
    if (hit) {
        if (lane == 0) {
            markC[row] = 0;
            cf[row] = CF_C;
            key[row] = kAssigned;
        }
        return;
    }
    if (last) {
        if (lane == 0) {
            cf[row] = CF_C;
            key[row] = kAssigned;
        }
        return;
    }
    // a neighbour assigned in this same pass may be pushed to: its flag is
    // never read again
    for (int32_t k = b + lane; k < e; k += G) {
        const int32_t i = ci[k];
        if (beats(kx, row, key[i], i)) beaten[i] = 1;
    }
}

__global__ void k_pmisr_finish(int32_t n, int8_t *__restrict__ cf, int32_t *__restrict__ nu) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == CF_U) {
        if (nu) atomicAdd(nu, 1);
        else cf[i] = CF_C;
    }
}

// Until no node is unassigned (max_rounds <= 0), every round's selection pass
// also counts the unassigned nodes it starts from into nu[round]; the counts
// are read back every kPmisrCheck rounds.  A round that starts with none
// changes nothing, so the rounds run past the end are no-ops and the count
// of rounds is the first round that found none.
constexpr int kPmisrCheck = 2;
constexpr int kPmisrSlots = 4096;

int pmisr(const CsrView &A, const StrengthGraph &G, const uint32_t *h, int max_rounds, int8_t *cf, hipStream_t s,
          uint64_t seed, int32_t level) {
    int32_t n = A.nr;
    DBuf<uint8_t> inD((size_t)n, s);
    const bool until_done = max_rounds <= 0;
    DBuf<int32_t> nu(until_done ? (size_t)kPmisrSlots : 1, s);
    if (until_done) fill_zero(nu.p, (size_t)kPmisrSlots * 4, s);
    DBuf<uint64_t> key((size_t)n, s);
    DBuf<uint8_t> flags((size_t)2 * n, s);
    uint8_t *beaten = flags.p, *markC = flags.p + n;
    k_pmisr_init<<<grid_for(n, 256), 256, 0, s>>>(n, G.srp.p, G.cntT.p, G.mutual.p, h, seed, level, cf, key.p,
                                                  beaten, markC);
    AIRG_LAUNCH_CHECK();
    int g = lanes_for(A.nnz / 2, n);   // rows of S: about half of A's entries
    const unsigned grid = grid_for((int64_t)n * g, 256);
    dispatch_group(g, [&]<int W>() {
        k_pmisr_push<W><<<grid, 256, 0, s>>>(n, G.srp.p, G.sci.p, key.p, beaten);
    });
    AIRG_LAUNCH_CHECK();
    int rounds = 0;
    for (;;) {
        if (!until_done && rounds >= max_rounds) break;
        AIRG_REQUIRE(rounds < kPmisrSlots, ST_STALL, "PMISR did not finish");
        int32_t *cnt = until_done ? nu.p + rounds : nullptr;
        dispatch_group(g, [&]<int W>() {
            k_pmisr_select<W><<<grid, 256, 0, s>>>(n, G.srp.p, G.sci.p, key.p, beaten, inD.p, markC, cnt);
            k_pmisr_update<W><<<grid, 256, 0, s>>>(n, G.srp.p, G.sci.p, inD.p, cf, key.p, markC, beaten,
                                                   !until_done && rounds + 1 == max_rounds);
        });
        AIRG_LAUNCH_CHECK();
        ++rounds;
        if (until_done && rounds % kPmisrCheck == 0) {
            int32_t got[kPmisrCheck];
            d2h(got, nu.p + rounds - kPmisrCheck, kPmisrCheck, s);
            int first_zero = -1;
            for (int q = 0; q < kPmisrCheck && first_zero < 0; ++q)
                if (got[q] == 0) first_zero = rounds - kPmisrCheck + q;
            if (first_zero >= 0) {
                rounds = first_zero;
                break;
            }
        }
    }
    if (until_done) {   // a fixed number of rounds ended in its last update
        k_pmisr_finish<<<grid_for(n, 256), 256, 0, s>>>(n, cf, nullptr);
        AIRG_LAUNCH_CHECK();
    }
    return rounds;
}

// ------------------------------------------------------------------ DDC ---
// theta_i = (sum over F columns j != i of |a_ij|, in ascending column order
// from +0.0) / |a_ii|.  The group loads a chunk of the row coalesced and every
// lane folds the chunk in order from the broadcast terms, so the sum is the
// sequential one.
template <int G>
__device__ inline void ddc_row_theta(const int32_t *rp, const int32_t *ci, const double *v, const int8_t *cf,
                                     int32_t row, int lane, double *s_out, double *d_out) {
    double s = 0.0, d = 0.0;
    int32_t e = rp[row + 1];
    for (int32_t base = rp[row]; base < e; base += G) {
        int32_t k = base + lane;
        double term = 0.0, dd = 0.0;
        if (k < e) {
            int32_t j = ci[k];
            if (j == row) dd = v[k];
            else if (cf[j] == CF_F) term = fabs(v[k]);
        }
        int cnt = e - base < G ? e - base : G;
        for (int q = 0; q < cnt; ++q) {
            s += group_bcast<G>(term, q);
        }
        d += group_sum<G>(dd);   // exactly one lane holds the diagonal
    }
    *s_out = s;
    *d_out = d;
}

template <int G>
__global__ void __launch_bounds__(256) k_ddc(int32_t n, const int32_t *__restrict__ rp,
                                             const int32_t *__restrict__ ci, const double *__restrict__ v,
                                             double alpha_diag, const int8_t *__restrict__ cf_in,
                                             int8_t *__restrict__ cf_out, double *__restrict__ theta,
                                             int32_t *__restrict__ flags3) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    auto put = [&](int8_t c) {
        cf_out[row] = c;
        if (flags3) {
            flags3[row] = c == CF_F;
            flags3[(int64_t)n + row] = c == CF_C;
            flags3[2 * (int64_t)n + row] = c == CF_T;
        }
    };
    int8_t c = cf_in[row];
    if (c != CF_F) {
        if (lane == 0) {
            put(c);
            if (theta) theta[row] = -1.0;
        }
        return;
    }
    double sum, d;
    ddc_row_theta<G>(rp, ci, v, cf_in, row, lane, &sum, &d);
    double th = d == 0.0 ? INFINITY : sum / fabs(d);
    bool conv = d == 0.0 || isinf(th) || (th > alpha_diag && th != 0.0);
    if (lane == 0) {
        put(conv ? CF_C : CF_F);
        if (theta) theta[row] = th;
    }
}

void ddc(const CsrView &A, double alpha_diag, const int8_t *cf_in, int8_t *cf_out, double *theta, hipStream_t s,
         int32_t *flags3) {
    int g = lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int W>() {
        k_ddc<W><<<grid_for((int64_t)A.nr * W, 256), 256, 0, s>>>(A.nr, A.rp, A.ci, A.v, alpha_diag, cf_in, cf_out,
                                                                   theta, flags3);
    });
    AIRG_LAUNCH_CHECK();
}

// ---------------------------------------------------- DDC fraction mode ---
__global__ void k_theta_max(int32_t n, const double *__restrict__ theta, unsigned long long *__restrict__ mx,
                            int32_t *__restrict__ nF) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = theta[i];
    if (t >= 0.0) atomicAdd(nF, 1);
    if (t >= 0.0 && isfinite(t)) atomicMax(mx, (unsigned long long)__double_as_longlong(t));
}

// hist[q] counts F rows whose theta exceeds exactly the boundaries b_0..b_{q-1}
// (b_k = theta_max * k / 1000), so #{theta > b_k} = sum_{q > k} hist[q].
__global__ void k_theta_hist(int32_t n, const double *__restrict__ theta, double tmax,
                             int32_t *__restrict__ hist) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = theta[i];
    if (!(t >= 0.0)) return;
    int q;
    if (!isfinite(t)) {
        q = 1001;
    } else {
        int lo = 0, hi = 1001;   // first k with b_k >= t, in [0, 1001]
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            double bk = tmax * (double)mid / 1000.0;
            if (bk >= t) hi = mid;
            else lo = mid + 1;
        }
        q = lo;
    }
    atomicAdd(&hist[q], 1);
}

// The boundary b_k = tmax k / 1000 whose count #{theta > b_k} is closest to
// ceil(fraction #F), ties to the larger k.  hist has 1002 bins as written by
// k_theta_hist; walking k downwards accumulates the counts, and a strict
// comparison keeps the larger k on a tie.
static double fraction_boundary(const int32_t *hist, int32_t nf, double tmax, double fraction) {
    int64_t target = (int64_t)std::ceil(fraction * (double)nf);
    int64_t above = hist[1001];   // #{theta > b_1000}
    int64_t bestd = above > target ? above - target : target - above;
    int bestk = 1000;
    for (int k = 999; k >= 0; --k) {
        above += hist[k + 1];
        int64_t d = above > target ? above - target : target - above;
        if (d < bestd) {
            bestd = d;
            bestk = k;
        }
    }
    return tmax * (double)bestk / 1000.0;
}

double ddc_fraction_threshold(const CsrView &A, const int8_t *cf, double fraction, hipStream_t s) {
    int32_t n = A.nr;
    DBuf<int8_t> tmp((size_t)n, s);
    DBuf<double> theta((size_t)n, s);
    ddc(A, 0.0, cf, tmp.p, theta.p, s);
    DBuf<unsigned long long> mx(1, s);
    DBuf<int32_t> nF(1, s), hist(1002, s);
    fill_zero(mx.p, 8, s);
    fill_zero(nF.p, 4, s);
    fill_zero(hist.p, 1002 * 4, s);
    k_theta_max<<<grid_for(n, 256), 256, 0, s>>>(n, theta.p, mx.p, nF.p);
    AIRG_LAUNCH_CHECK();
    unsigned long long mbits = d2h_one(mx.p, s);
    double tmax;
    std::memcpy(&tmax, &mbits, 8);
    int32_t nf = d2h_one(nF.p, s);
    k_theta_hist<<<grid_for(n, 256), 256, 0, s>>>(n, theta.p, tmax, hist.p);
    AIRG_LAUNCH_CHECK();
    std::vector<int32_t> hh(1002);
    d2h(hh.data(), hist.p, 1002, s);
    return fraction_boundary(hh.data(), nf, tmax, fraction);
}

// ------------------------------------ fraction rule without allocation ---
// The same threshold for callers that cannot allocate device memory (code
// under graph capture, serving loops): theta and the counters live in a
// fixed device array of this file.  Layout: max bits (8 B) at 0, #F (4 B) at
// 8, the 1002 histogram bins at 16, theta (8 B per row) from kNaThetaOff.
// Every call on a device shares that device's copy and keeps the previous
// call's contents; calls that overlap on one device race.
constexpr size_t kNaThetaOff = 4096;
constexpr int64_t kNaMaxRows = (int64_t)1 << 21;
static __device__ __align__(256) unsigned char scratch[kNaThetaOff + (size_t)kNaMaxRows * 8];

constexpr int kNaMaxDevices = 64;
static std::mutex g_na_mu;
static unsigned char *g_na_ptr[kNaMaxDevices];

// Device address of this device's scratch, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
static unsigned char *noalloc_scratch() {
    int dev = -1;
    AIRG_HIP(hipGetDevice(&dev));
    AIRG_REQUIRE(dev >= 0 && dev < kNaMaxDevices, ST_LIMIT, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        AIRG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        AIRG_REQUIRE(p != nullptr, ST_HIP, "no device address for the scratch array");
        g_na_ptr[dev] = (unsigned char *)p;
    }
    return g_na_ptr[dev];
}

int64_t ddc_fraction_noalloc_max_rows() { return kNaMaxRows; }

// theta_i of every row (-1 off F), by the same row sum as k_ddc.
template <int G>
__global__ void __launch_bounds__(256) k_ddc_theta(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   const int8_t *__restrict__ cf, double *__restrict__ theta) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t row = (int32_t)(t / G);
    int lane = group_lane<G>();
    if (row >= n) return;
    if (cf[row] != CF_F) {
        if (lane == 0) theta[row] = -1.0;
        return;
    }
    double sum, d;
    ddc_row_theta<G>(rp, ci, v, cf, row, lane, &sum, &d);
    if (lane == 0) theta[row] = d == 0.0 ? INFINITY : sum / fabs(d);
}

double ddc_fraction_threshold_noalloc(const CsrView &A, const int8_t *cf, double fraction, hipStream_t s) {
    int32_t n = A.nr;
    AIRG_REQUIRE(n <= kNaMaxRows, ST_LIMIT,
                 "ddc_fraction_threshold_noalloc: " + std::to_string(n) + " rows exceed the scratch limit of " +
                     std::to_string(kNaMaxRows));
    unsigned char *base = noalloc_scratch();
    auto *mx = (unsigned long long *)base;
    auto *nF = (int32_t *)(base + 8);
    auto *hist = (int32_t *)(base + 16);
    auto *theta = (double *)(base + kNaThetaOff);
    fill_zero(base, 16 + 1002 * 4, s);
    int g = lanes_for(A.nnz, A.nr);
    dispatch_group(g, [&]<int W>() {
        k_ddc_theta<W><<<grid_for((int64_t)n * W, 256), 256, 0, s>>>(n, A.rp, A.ci, A.v, cf, theta);
    });
    AIRG_LAUNCH_CHECK();
    k_theta_max<<<grid_for(n, 256), 256, 0, s>>>(n, theta, mx, nF);
    AIRG_LAUNCH_CHECK();
    unsigned char head[16];
    AIRG_HIP(hipMemcpyAsync(head, base, 16, hipMemcpyDeviceToHost, s));
    AIRG_HIP(hipStreamSynchronize(s));
    double tmax;
    int32_t nf;
    std::memcpy(&tmax, head, 8);
    std::memcpy(&nf, head + 8, 4);
    k_theta_hist<<<grid_for(n, 256), 256, 0, s>>>(n, theta, tmax, hist);
    AIRG_LAUNCH_CHECK();
    int32_t hh[1002];
    AIRG_HIP(hipMemcpyAsync(hh, hist, sizeof hh, hipMemcpyDeviceToHost, s));
    AIRG_HIP(hipStreamSynchronize(s));
    return fraction_boundary(hh, nf, tmax, fraction);
}

// ---------------------------------------------------------- full split ---
std::pair<int32_t, int32_t> cf_split(const CsrView &A, const CfParams &p, int32_t level, int8_t *cf, hipStream_t s) {
    int32_t n = A.nr;
    StrengthGraph G = strength_graph(A, p.strong_threshold, s);
    DBuf<int8_t> cf0((size_t)n, s);
    pmisr(A, G, nullptr, p.max_rounds, cf0.p, s, p.seed, level);
    double ad = p.ddc_threshold;
    if (ad < 0.0) ad = ddc_fraction_threshold(A, cf0.p, p.ddc_fraction, s);
    ddc(A, ad, cf0.p, cf, nullptr, s);
    DBuf<int32_t> rank((size_t)n, s);
    return cf_ranks(cf, n, rank.p, s);
}

}  // namespace airg

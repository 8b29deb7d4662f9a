// Sub-wave group primitives: G consecutive lanes of a 64-lane wavefront
// cooperate on one row.  G is a power of two in [1, 64].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace airg {

template <int G>
__device__ inline int group_lane() {
    return (int)(threadIdx.x & (G - 1));
}

// Bits of a wave ballot that belong to the caller's group, shifted to bit 0.
template <int G>
__device__ inline uint64_t group_ballot(bool pred) {
    constexpr uint64_t kMask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull);
    uint64_t m = __ballot(pred);
    if (G == 64) return m;
    int base = (int)(threadIdx.x & 63) & ~(G - 1);
    return (m >> base) & kMask;
}

// Number of set predicates on lanes below this one in the group, and total.
template <int G>
__device__ inline int group_prefix(bool pred, int *total) {
    uint64_t gm = group_ballot<G>(pred);
    int lane = group_lane<G>();
    *total = __popcll(gm);
    return __popcll(gm & ((1ull << lane) - 1ull));
}

template <int G, class T>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Sum over a whole wavefront (all 64 lanes active) returned to every lane:
// a butterfly inside each row of 16 lanes on the DPP crossbar (lane swaps
// within quads, then the half-row and row mirrors), then the four row sums
// read out through scalar registers.  No LDS traffic, unlike the shuffle
// tree of group_sum.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, true);
}
__device__ inline double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

template <int G, class T>
__device__ inline T group_max(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, G);
        v = w > v ? w : v;
    }
    return v;
}

template <int G>
__device__ inline bool group_any(bool p) {
    return group_ballot<G>(p) != 0;
}

template <int G, class T>
__device__ inline T group_bcast(T v, int src) {
    return __shfl(v, src, G);
}

// Calls f.template operator()<G>() with G the runtime group width.
template <class F>
inline void dispatch_group(int g, F &&f) {
    switch (g) {
    case 1: f.template operator()<1>(); break;
    case 2: f.template operator()<2>(); break;
    case 4: f.template operator()<4>(); break;
    case 8: f.template operator()<8>(); break;
    case 16: f.template operator()<16>(); break;
    case 32: f.template operator()<32>(); break;
    default: f.template operator()<64>(); break;
    }
}

}  // namespace airg

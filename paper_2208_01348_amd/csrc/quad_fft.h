// Line transforms held in registers, one line per quad of adjacent lanes.
//
// A line of length L (L/4 of the form 2^a 3^b) belongs to four adjacent lanes:
// lane n2 holds the L/4 points x[4 n1 + n2] and takes their L/4-point DFT in
// registers (the compile-time Stockham stages of fft_core.h); after the
// twiddle W_L^{n2 k1} the four lanes finish with a radix-4 butterfly through
// quad DPP moves, lane n2 ending with X[k1 + (L/4) rev2(n2)] (rev2 swaps the
// two bits).  quad_fft_blk is the mirror image, from that blocked layout back
// to the decimated one.
//
// Two twiddle tables, both holding W_L^t = exp(-2 pi i t / L) for t < L:
// tw_reg is read at compile-time indices only (the in-register stages; a
// global table there gives scalar loads), tw_lane at the per-lane index
// n2 k1 (a table in LDS or in global memory).
#pragma once

#include "fft_core.h"

namespace dda {

// Quad lane exchange (every lane of a quad is active): bound_ctrl set and a
// zero old value let the compiler fold the move into the consuming add.
__device__ __forceinline__ float dpp_x1(float v) {  // value of lane ^ 1 (quad_perm 1,0,3,2)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_x2(float v) {  // value of lane ^ 2 (quad_perm 2,3,0,1)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ double dpp_x1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0xB1, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double dpp_x2(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x4E, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x4E, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Q-point DFT of v in registers (reg_dft of fft_core.h with the L-entry
// twiddle table, W_Q^t = tw[t L/Q]).
template <typename T, int L, int Q, int NS, bool INV>
__device__ __forceinline__ void reg_stages(cx<T> (&v)[Q], const cx<T>* __restrict__ tw) {
    reg_dft<T, Q, NS, INV, L / Q>(v, tw);
}

// DFT of one line of length L spread over a lane quad (see above).
template <typename T, int L, bool INV>
__device__ __forceinline__ void quad_fft(cx<T> (&v)[L / 4], int n2, const cx<T>* __restrict__ tw_reg,
                                         const cx<T>* __restrict__ tw_lane) {
    constexpr int Q = L / 4;
    reg_stages<T, L, Q, 1, INV>(v, tw_reg);
#pragma unroll
    for (int k1 = 1; k1 < Q; ++k1) {
        cx<T> t = tw_lane[n2 * k1];
        if (INV) t.y = -t.y;
        v[k1] = v[k1] * t;
    }
    // butterflies as partner + sign * own: the lower lane of a pair adds,
    // the upper one subtracts, with no select
    const bool hi = (n2 & 2) != 0, odd = (n2 & 1) != 0;
    const T s2 = hi ? T(-1) : T(1), s1 = odd ? T(-1) : T(1);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {  // pairs (n2, n2 ^ 2); W_4 on lane 3
        cx<T> r{dpp_x2(v[k1].x) + s2 * v[k1].x, dpp_x2(v[k1].y) + s2 * v[k1].y};
        if (hi && odd) r = mul_mi<INV>(r);
        v[k1] = r;
    }
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1)  // pairs (n2, n2 ^ 1)
        v[k1] = cx<T>{dpp_x1(v[k1].x) + s1 * v[k1].x, dpp_x1(v[k1].y) + s1 * v[k1].y};
}

// The mirror image of quad_fft: input in the layout quad_fft leaves (lane l
// holds X[k1 + (L/4) rev2(l)]), output decimated (lane n2 holds
// y[4 n1 + n2], n1 in natural order).  Radix-4 across the quad first (pairs
// l ^ 1, the factor W_4 on lane 3, pairs l ^ 2), then the twiddle
// W_L^{n2 k1} and the L/4-point DFT in registers.
template <typename T, int L, bool INV>
__device__ __forceinline__ void quad_fft_blk(cx<T> (&v)[L / 4], int n2,
                                             const cx<T>* __restrict__ tw_reg,
                                             const cx<T>* __restrict__ tw_lane) {
    constexpr int Q = L / 4;
    const bool hi = (n2 & 2) != 0, odd = (n2 & 1) != 0;
    const T s2 = hi ? T(-1) : T(1), s1 = odd ? T(-1) : T(1);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {
        cx<T> r{dpp_x1(v[k1].x) + s1 * v[k1].x, dpp_x1(v[k1].y) + s1 * v[k1].y};
        if (hi && odd) r = mul_mi<INV>(r);
        v[k1] = r;
    }
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1)
        v[k1] = cx<T>{dpp_x2(v[k1].x) + s2 * v[k1].x, dpp_x2(v[k1].y) + s2 * v[k1].y};
#pragma unroll
    for (int k1 = 1; k1 < Q; ++k1) {
        cx<T> t = tw_lane[n2 * k1];
        if (INV) t.y = -t.y;
        v[k1] = v[k1] * t;
    }
    reg_stages<T, L, Q, 1, INV>(v, tw_reg);
}

}  // namespace dda

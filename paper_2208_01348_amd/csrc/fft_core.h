// LDS-resident mixed-radix FFT of a tile of lines, with the whole plan fixed
// at compile time (line length L = 2^a 3^b, radices 8/4/2/3).
//
// Stockham autosort formulation (Govindaraju et al., SC'08): stage s with
// radix R and Ns = product of the earlier radices reads the R inputs
// x[j + m L/R], twiddles the m-th by exp(-+2 pi i m (j mod Ns)/(Ns R)), takes
// an R-point DFT and writes output m to (j div Ns) Ns R + (j mod Ns) + m Ns.
// Every stage reads all its inputs into registers, synchronises, then writes
// in place, so one LDS buffer suffices.  Output is in natural order.
//
// Element e of line l lives at lds[l*LS + e*ES].  When ES == 1 (rows), lanes
// walk along a line; otherwise (column tiles) consecutive lanes take
// consecutive lines so that LDS accesses stay contiguous.
#pragma once

#include "common.h"

namespace dda {

constexpr int pick_radix(int rem) {
    return rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 2 == 0 ? 2 : rem % 3 == 0 ? 3 : 1;
}

constexpr bool fft_size_ok(int L) {
    int r = L;
    while (r > 1) {
        int p = pick_radix(r);
        if (p == 1) return false;
        r /= p;
    }
    return L >= 1;
}

template <typename T>
struct Consts;
template <>
struct Consts<double> {
    static constexpr double rsqrt2 = 0.70710678118654752440;
    static constexpr double sqrt3_2 = 0.86602540378443864676;
};
template <>
struct Consts<float> {
    static constexpr float rsqrt2 = 0.70710678118654752440f;
    static constexpr float sqrt3_2 = 0.86602540378443864676f;
};

template <bool INV, typename T>
__device__ __forceinline__ void dft2(cx<T>* a) {
    cx<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi<INV>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft3(cx<T>* a) {
    const T h = Consts<T>::sqrt3_2;
    cx<T> t = a[1] + a[2];
    cx<T> m = a[0] - T(0.5) * t;
    cx<T> d = a[1] - a[2];
    // u = d * (-i h) forward, d * (+i h) inverse
    cx<T> u = INV ? cx<T>{-h * d.y, h * d.x} : cx<T>{h * d.y, -h * d.x};
    a[0] = a[0] + t;
    a[1] = m + u;
    a[2] = m - u;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
    const T s = Consts<T>::rsqrt2;
    cx<T> b0 = a[0] + a[4], b1 = a[1] + a[5], b2 = a[2] + a[6], b3 = a[3] + a[7];
    cx<T> c0 = a[0] - a[4], c1 = a[1] - a[5], c2 = a[2] - a[6], c3 = a[3] - a[7];
    // c_k *= w8^{-+k}
    if (INV) {
        c1 = cx<T>{s * (c1.x - c1.y), s * (c1.x + c1.y)};
        c2 = cx<T>{-c2.y, c2.x};
        c3 = cx<T>{-s * (c3.x + c3.y), s * (c3.x - c3.y)};
    } else {
        c1 = cx<T>{s * (c1.x + c1.y), s * (c1.y - c1.x)};
        c2 = cx<T>{c2.y, -c2.x};
        c3 = cx<T>{s * (c3.y - c3.x), -s * (c3.x + c3.y)};
    }
    dft4<INV>(b0, b1, b2, b3);
    dft4<INV>(c0, c1, c2, c3);
    a[0] = b0; a[2] = b1; a[4] = b2; a[6] = b3;
    a[1] = c0; a[3] = c1; a[5] = c2; a[7] = c3;
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T>* a) {
    if constexpr (R == 2) dft2<INV>(a);
    else if constexpr (R == 3) dft3<INV>(a);
    else if constexpr (R == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
    else if constexpr (R == 8) dft8<INV>(a);
}

// Position of element i of a line whose LDS layout has one spare slot after
// every 16 elements (PAD), or none.  A radix-R Stockham stage stores each
// lane's R outputs next to each other, so at one store the lanes of a wave are
// R elements apart; with 16-byte elements and R = 8 that puts 16 lanes on two
// groups of banks, and the spare slots spread them over all of them (the
// reads, at consecutive positions, stay conflict-free).
template <bool PAD>
__device__ __forceinline__ constexpr int line_pos(int i) { return PAD ? i + (i >> 4) : i; }
// Line pitch for the padded layout of a line of L elements.
template <int L>
constexpr int padded_len() { return L + (L + 15) / 16; }

template <typename T, int L, int R, int NS, bool INV, int NLINES, int LS, int ES, int NTHR,
          bool PAD = false>
__device__ __forceinline__ void fft_stage(cx<T>* lds, const cx<T>* __restrict__ tw, int tid,
                                          int nl) {
    constexpr int LR = L / R;
    constexpr int NB = NLINES * LR;
    constexpr int NQ = (NB + NTHR - 1) / NTHR;
    constexpr bool LINE_FAST = (ES != 1);
    const int nb = nl * LR;  // nl <= NLINES lines are live
    cx<T> v[NQ][R];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int b = tid + q * NTHR;
        if (b < nb) {
            const int line = LINE_FAST ? b % NLINES : b / LR;
            const int j = LINE_FAST ? b / NLINES : b % LR;
#pragma unroll
            for (int m = 0; m < R; ++m) v[q][m] = lds[line * LS + line_pos<PAD>((j + m * LR) * ES)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int b = tid + q * NTHR;
        if (b < nb) {
            const int line = LINE_FAST ? b % NLINES : b / LR;
            const int j = LINE_FAST ? b / NLINES : b % LR;
            const int k = j % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    cx<T> w = tw[m * k * (L / (NS * R))];
                    if (INV) w.y = -w.y;
                    v[q][m] = v[q][m] * w;
                }
            }
            dft<R, INV>(v[q]);
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) lds[line * LS + line_pos<PAD>((base + m * NS) * ES)] = v[q][m];
        }
    }
    __syncthreads();
}

template <typename T, int L, int NS, bool INV, int NLINES, int LS, int ES, int NTHR, bool PAD,
          bool R3F>
__device__ __forceinline__ void fft_stages(cx<T>* lds, const cx<T>* __restrict__ tw, int tid,
                                           int nl) {
    if constexpr (NS < L) {
        constexpr int R = (R3F && (L / NS) % 3 == 0) ? 3 : pick_radix(L / NS);
        static_assert(R > 1, "FFT length must be 2^a 3^b");
        fft_stage<T, L, R, NS, INV, NLINES, LS, ES, NTHR, PAD>(lds, tw, tid, nl);
        fft_stages<T, L, NS * R, INV, NLINES, LS, ES, NTHR, PAD, R3F>(lds, tw, tid, nl);
    }
}

// Q-point DFT of v held in registers, natural order in and out, by the same
// Stockham stages (radices from pick_radix) with every index known at compile
// time.  The twiddle W_Q^t is read as tw[t * TS] (tw holds W_{Q TS}^t).
template <typename T, int Q, int NS, bool INV, int TS>
__device__ __forceinline__ void reg_dft(cx<T> (&v)[Q], const cx<T>* __restrict__ tw) {
    if constexpr (NS < Q) {
        constexpr int R = pick_radix(Q / NS);
        static_assert(R > 1, "line length must be 2^a 3^b");
        constexpr int QR = Q / R;
        cx<T> w[Q];
#pragma unroll
        for (int j = 0; j < QR; ++j) {
            cx<T> a[R];
#pragma unroll
            for (int m = 0; m < R; ++m) a[m] = v[j + m * QR];
            const int k = j % NS;
            if (NS > 1 && k != 0) {
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    cx<T> t = tw[(m * k * (Q / (NS * R))) * TS];
                    if (INV) t.y = -t.y;
                    a[m] = a[m] * t;
                }
            }
            dft<R, INV>(a);
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) w[base + m * NS] = a[m];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = w[i];
        reg_dft<T, Q, NS * R, INV, TS>(v, tw);
    }
}

// Unnormalised DFT (forward: exp(-2 pi i jk/L); inverse: exp(+2 pi i jk/L))
// of NLINES lines held in LDS.  tw[t] = exp(-2 pi i t / L), t < L.
// Must be called by all NTHR threads of the block; ends with a barrier.  Only
// the first nl lines are transformed (nl <= NLINES; ES == 1 when nl < NLINES).
// PAD: lines in the padded layout of line_pos (ES == 1, LS >= padded_len<L>()).
// R3F: the radix-3 stage first (for L = 3 * 2^k: its stores are 3 elements
// apart, and the radix-8 stages after it store 3 and 24 elements apart instead
// of 1 and 8, which spreads the lanes of a row over more LDS banks).
template <typename T, int L, bool INV, int NLINES, int LS, int ES, int NTHR, bool PAD = false,
          bool R3F = false>
__device__ __forceinline__ void fft_tile(cx<T>* lds, const cx<T>* __restrict__ tw, int tid,
                                         int nl = NLINES) {
    static_assert(fft_size_ok(L), "FFT length must be 2^a 3^b");
    static_assert(!PAD || (ES == 1 && LS >= padded_len<L>()), "padded lines need ES == 1");
    fft_stages<T, L, 1, INV, NLINES, LS, ES, NTHR, PAD, R3F>(lds, tw, tid, nl);
}

}  // namespace dda

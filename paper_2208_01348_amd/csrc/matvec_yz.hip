// Three-pass FFT matvec for lattices whose padded yz plane fits in LDS.
//
// MI355X's 160 KB of LDS per CU holds a whole zero-padded yz plane of the
// three field components for cross-sections up to 48 x 48 cells in FP64 and
// 64 x 64 in FP32 (my = mz = L).  The y and z transforms, the 3x3 product
// with D and the inverse transforms then happen in one kernel per kx column,
// without the two 12N-sized intermediates that the five-pass chain streams
// through HBM:
//   X1 gather + x-FFT   : rows of one (component, z) plane, stored kx-major
//                         T[kx][c][z][y] (only y < ny, z < nz are non-zero)
//   YZ y-FFT, z-FFT, D u, z-iFFT, y-iFFT on the plane of one kx in LDS
//   X2 x-iFFT + pack    : back to the compact vector, x/alpha - (G x)
// HBM traffic per right-hand side: about 24N complex instead of 72N.
#include <algorithm>

#include "fft_core.h"
#include "kernels.h"
#include "quad_fft.h"

namespace dda {

namespace {

constexpr int NT = 512;    // x kernels (measured best of 192 ... 1024 on the nanorod lattice)
constexpr int NTYZ = 512;  // yz kernel, default threads per block (the autotuner
                           // may pick 256 or 1024 for L >= 24; the butterflies
                           // are the same whichever thread computes them)

// Position of y inside one line (c, z) of the T buffer.  When ny is a
// multiple of 8 every block of 8 is stored in the order (y mod 4, bit 2 of
// y): the pair y = 8j + n2, 8j + 4 + n2 that lane n2 of a quad holds in the
// decimated layout of the register line transforms is then contiguous, and
// a quad reads or writes 64 contiguous bytes (FP32).  Otherwise natural order.
__device__ __forceinline__ int tpos(int y, bool perm) {
    return perm ? (y & ~7) | ((y & 3) << 1) | ((y >> 2) & 1) : y;
}

// At most this many rows of one (component, z) plane per x-kernel block
// (about 37 KB of LDS); the rows of a plane are split evenly over
// ceil(ny / max) blocks.
template <typename T, int LX>
constexpr int xrows_max() {
    constexpr int r = (sizeof(T) == 4 ? 4608 : 2304) / LX;
    return r < 1 ? 1 : r > 64 ? 64 : r;
}

template <typename T, int L>
constexpr size_t yz_lds_bytes() { return size_t(L) * 3 * (L + 1) * 2 * sizeof(T); }

}  // namespace

bool yz_fused_ok(const Geo& g, int csize) {
    if (g.my != g.mz) return false;
    const size_t L = size_t(g.my);
    if (L > 64) return false;
    return L * 3 * (L + 1) * size_t(csize) <= size_t(120) << 10;
}

// (row groups per plane, rows per group) of the x kernels
template <typename T>
static void xsplit(const Geo& g, int& ng, int& nr) {
    int rmax = 0;
    switch (g.mx) {
#define DDA_CASE(N)                   \
    case N:                           \
        rmax = xrows_max<T, N>();     \
        break;
        DDA_CASE(1) DDA_CASE(2) DDA_CASE(3) DDA_CASE(4) DDA_CASE(6) DDA_CASE(8) DDA_CASE(12)
        DDA_CASE(16) DDA_CASE(24) DDA_CASE(32) DDA_CASE(48) DDA_CASE(64) DDA_CASE(96)
        DDA_CASE(128) DDA_CASE(192) DDA_CASE(256) DDA_CASE(384) DDA_CASE(512)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    ng = (g.ny + rmax - 1) / rmax;
    nr = (g.ny + ng - 1) / ng;
}

static int xgroups(const Geo& g, int csize) {
    int ng, nr;
    if (csize == int(sizeof(cx<float>))) xsplit<float>(g, ng, nr);
    else xsplit<double>(g, ng, nr);
    return ng;
}

int yz_pack_blocks_per_slot(const Geo& g, int csize) { return 3 * g.nz * xgroups(g, csize); }

// ------------------------------------------------------------------ X1 -----
// One block: rows y0 .. y0 + nrow - 1 of the (component c, z) plane.  The
// gather issues every index load of a thread before any data load, and every
// data load before the first use, so a block waits for memory twice rather
// than once per element.  Only x < HX = ceil(LX / 2) can be occupied
// (LX >= 2 nx - 1).
// FUSE: 0 plain gather; FUSE_COCG the COCG direction update p = r + beta p in
// place (fo: its folded finalizer); FUSE_BICG_S / FUSE_BICG_P the BiCGStab
// s = r - alpha v / p = r + beta (p - omega v) (bf), written in place of the
// input for an iterating slot.
template <typename T, int LX, int FUSE>
__global__ __launch_bounds__(NT) void k_xfft_t(cx<T>* __restrict__ xin,
                                               const int* __restrict__ map,
                                               cx<T>* __restrict__ Tb,
                                               const cx<T>* __restrict__ tw, Geo g,
                                               const int* __restrict__ act,
                                               const cx<T>* __restrict__ fuse_r, SlotFilter f,
                                               int ngroups, int nr, CocgFold fo, BicgFold bf) {
    constexpr bool FUSE_P = FUSE == FUSE_COCG;
    constexpr bool FUSE_S = FUSE == FUSE_BICG_S;
    constexpr bool FUSE_BP = FUSE == FUSE_BICG_P;
    constexpr int NR = xrows_max<T, LX>();
    constexpr int LP = LX + 1;  // padded LDS row: the transposed accesses hit spread banks
    constexpr int HX = (LX + 1) / 2;
    constexpr int NE = (NR * HX + NT - 1) / NT;
    __shared__ cx<T> lds[NR * LP];
    __shared__ cx<T> twl[LX];  // twiddles in LDS: the stage loads index them per lane
    const int tid = threadIdx.x;
    const int pos = blockIdx.y;
    const int64_t slot = act ? act[pos] : pos;
    const bool fold = FUSE_P && fo.nblk > 0;
    bool sact = false;  // FUSE_S, FUSE_BP: this slot iterates, so the block updates
    int status0 = SLOT_ACTIVE;
    if (fold || FUSE_S || FUSE_BP) {  // a folded step may change the status: one read per block
        __shared__ int st0;
        if (tid == 0) st0 = (FUSE_S || FUSE_BP ? bf.st : f.st)[slot].status;
        __syncthreads();
        status0 = st0;
        if (fold && status0 != SLOT_ACTIVE) return;
        sact = status0 == SLOT_ACTIVE;
    } else if (!slot_live(f, slot)) {
        return;
    }
    map += slot * g.map_stride;
    for (int t = tid; t < LX; t += NT) twl[t] = tw[t];
    const int grp = blockIdx.x % ngroups;
    const int cz = blockIdx.x / ngroups;
    const int c = cz / g.nz, z = cz - (cz / g.nz) * g.nz;
    const int y0 = grp * nr;
    const int nrow = min(nr, g.ny - y0);
    cx<T>* src = xin + (slot * 3 + c) * g.n_occ;
    const cx<T>* rsrc = FUSE ? fuse_r + (slot * 3 + c) * g.n_occ : nullptr;
    const cx<T>* vsrc = (FUSE_S || FUSE_BP)
                            ? static_cast<const cx<T>*>(bf.v) + (slot * 3 + c) * g.n_occ
                            : nullptr;
    // every index load, then every data load, is in flight before the first use
    int idx[NE];
    row_indices<NE, NT, HX>(map + (int64_t(z) * g.ny + y0) * g.nx, nrow, g.nx, tid, idx);
    // the direction update's scalars: the folded finalizer's row loads go
    // out while the index loads are in flight, ahead of the data loads
    cx<T> beta{T(0), T(0)};
    bool reset = false;
    if (FUSE_P) {
        if (fold) {
            z128 b;
            if (!cocg_fold<NT>(fo, int(slot), blockIdx.x == 0, b)) return;
            beta = cvt<T>(b);
        } else {
            beta = cvt<T>(f.st[slot].beta);
        }
        reset = f.st[slot].reset_p != 0;
    }
    cx<T> alpha{T(0), T(0)}, bt{T(0), T(0)}, om{T(0), T(0)};
    if constexpr (FUSE_S) {
        if (sact) {  // block-uniform
            z128 a;
            sact = bicg_sfold<NT>(bf, int(slot), blockIdx.x == 0, a);
            alpha = cvt<T>(a);
        }
    }
    if constexpr (FUSE_BP) {
        z128 b, o;
        sact = bicg_pfold<NT>(bf, int(slot), status0, blockIdx.x == 0, b, o);
        bt = cvt<T>(b);
        om = cvt<T>(o);
    }
    cx<T> v[NE], w[NE], u[FUSE_S || FUSE_BP ? NE : 1];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int i = max(idx[q], 0);
        if constexpr (FUSE_S) {
            if (sact) {
                w[q] = rsrc[i];
                u[q] = vsrc[i];
            } else {
                v[q] = src[i];
            }
        } else if constexpr (FUSE_BP) {
            v[q] = src[i];
            if (sact) {
                w[q] = rsrc[i];
                u[q] = vsrc[i];
            }
        } else {
            v[q] = src[i];
            if (FUSE_P) w[q] = rsrc[i];
        }
    }
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if constexpr (FUSE_S) {
            if (sact) {
                v[q] = bicg_s_of(w[q], alpha, u[q]);
                if (idx[q] >= 0) s2 += bicg_norm2(v[q]);
            }
        }
        if constexpr (FUSE_BP) {
            if (sact) v[q] = bicg_p_of(w[q], bt, v[q], om, u[q]);
        }
        if (idx[q] < 0) v[q] = cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + q * NT;
        const int r = e / HX, x = e - (e / HX) * HX;
        if (FUSE_P && idx[q] >= 0) {  // each occupied element is visited by exactly one thread
            v[q] = reset ? w[q] : w[q] + beta * v[q];
            src[idx[q]] = v[q];
        }
        if constexpr (FUSE_S || FUSE_BP) {
            if (sact && idx[q] >= 0) src[idx[q]] = v[q];
        }
        if (r < nrow) {
            lds[r * LP + x] = v[q];
            if (x + HX < LX) lds[r * LP + x + HX] = cx<T>{T(0), T(0)};
        }
    }
    if constexpr (FUSE_S) {
        if (sact) {  // ||s||^2 rows, one per block of the slot (block-uniform)
            double pr[1] = {s2};
            block_partial<1, NT, 6>(pr, bf.red, int(slot), blockIdx.x);
        }
    }
    __syncthreads();
    fft_tile<T, LX, false, NR, LP, 1, NT, false, true>(lds, twl, tid, nrow);
    const int64_t cplane = int64_t(3) * g.nz * g.ny;  // one kx column
    cx<T>* dst = Tb + int64_t(pos) * g.mx * cplane + (int64_t(c) * g.nz + z) * g.ny;
    const bool perm = (g.ny & 7) == 0;
    {
        // element e = (kx, r) with the compile-time row count NR (rows r >= nrow
        // idle): no run-time division; every LDS read before the first store
        constexpr int NS = (NR * LX + NT - 1) / NT;
        cx<T> t[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int e = tid + q * NT;
            const int kx = e / NR, r = e - (e / NR) * NR;
            t[q] = lds[min(r, nrow - 1) * LP + min(kx, LX - 1)];
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int e = tid + q * NT;
            const int kx = e / NR, r = e - (e / NR) * NR;
            if (kx < LX && r < nrow) dst[kx * cplane + tpos(y0 + r, perm)] = t[q];
        }
    }
}

// ------------------------------------------------------------------ X2 -----
template <typename T, int LX, int MODE>
__global__ __launch_bounds__(NT) void k_ixfft_t(const cx<T>* __restrict__ Tb,
                                                const cx<T>* __restrict__ xin,
                                                const cx<T>* __restrict__ ainv,
                                                cx<T>* __restrict__ yout,
                                                const int* __restrict__ map,
                                                const cx<T>* __restrict__ tw, Geo g,
                                                const int* __restrict__ act,
                                                const int* __restrict__ slot_sys, SlotFilter f,
                                                RedScratch red, int ngroups, int nr,
                                                const cx<T>* __restrict__ wv) {
    constexpr int NR = xrows_max<T, LX>();
    constexpr int LP = LX + 1;
    constexpr int HX = (LX + 1) / 2;
    constexpr int NL = (NR * LX + NT - 1) / NT;
    constexpr int NE = (NR * HX + NT - 1) / NT;
    __shared__ cx<T> lds[NR * LP];
    __shared__ cx<T> twl[LX];
    const int tid = threadIdx.x;
    const int pos = blockIdx.y;
    const int64_t slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    map += slot * g.map_stride;
    for (int t = tid; t < LX; t += NT) twl[t] = tw[t];
    const int64_t sys = slot_sys[slot];
    const int grp = blockIdx.x % ngroups;
    const int cz = blockIdx.x / ngroups;
    const int c = cz / g.nz, z = cz - (cz / g.nz) * g.nz;
    const int y0 = grp * nr;
    const int nrow = min(nr, g.ny - y0);
    const int64_t cplane = int64_t(3) * g.nz * g.ny;
    const cx<T>* src = Tb + int64_t(pos) * g.mx * cplane + (int64_t(c) * g.nz + z) * g.ny;
    const bool perm = (g.ny & 7) == 0;
    {
        // element e = (kx, r) with the compile-time row count NR (rows r >= nrow
        // idle), so no run-time division
        cx<T> t[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + q * NT;
            const int kx = e / NR, r = e - (e / NR) * NR;
            t[q] = src[min(kx, LX - 1) * cplane + tpos(y0 + min(r, nrow - 1), perm)];
        }
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + q * NT;
            const int kx = e / NR, r = e - (e / NR) * NR;
            if (kx < LX && r < nrow) lds[r * LP + kx] = t[q];
        }
    }
    __syncthreads();
    fft_tile<T, LX, true, NR, LP, 1, NT, false, true>(lds, twl, tid, nrow);
    const int64_t voff = (slot * 3 + c) * g.n_occ;
    int idx[NE];
    row_indices<NE, NT, HX>(map + (int64_t(z) * g.ny + y0) * g.nx, nrow, g.nx, tid, idx);
    cx<T> xv[NE], av[NE], wq[MODE == PACK_AX_DOTW ? NE : 1];
    if (MODE != PACK_GX) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int i = max(idx[q], 0);
            xv[q] = xin[voff + i];
            av[q] = ainv[sys * g.n_occ + i];
            if constexpr (MODE == PACK_AX_DOTW) wq[q] = wv[voff + i];
        }
    }
    double mu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if (idx[q] < 0) continue;
        const int e = tid + q * NT;
        const int r = e / HX, x = e - (e / HX) * HX;
        const cx<T> conv = lds[r * LP + x];
        if (MODE == PACK_GX) {
            yout[voff + idx[q]] = conv;
        } else {
            const cx<T> yi = xv[q] * av[q] - conv;
            yout[voff + idx[q]] = yi;
            if constexpr (MODE == PACK_AX_DOTW) pack_dots<T, MODE>(mu, xv[q], yi, wq[q]);
            else pack_dots<T, MODE>(mu, xv[q], yi, yi);
        }
    }
    // partial rows; the Krylov update kernels sum them
    pack_rows<MODE, NT>(mu, red, int(slot), blockIdx.x);
}

// ------------------------------------------------------------------ YZ -----
// One kx column of one right-hand side: the plane [z][component][y] lives in
// LDS (row stride L + 1).  D comes from its kx-slab layout
// [kx' <= mx/2][6][kz' <= L/2][ky' <= L/2]; one load serves the (up to) four
// frequencies (ky or L - ky) x (kz or L - kz) that share it, with the sign
// flips of the odd components.
template <typename T, int L, int NTY>
__global__ __launch_bounds__(NTY) void k_yzconv(cx<T>* __restrict__ Tb,
                                                 const cx<T>* const* __restrict__ Dptr,
                                                 const cx<T>* __restrict__ twy,
                                                 const cx<T>* __restrict__ twz, Geo g,
                                                 const int* __restrict__ act,
                                                 const int* __restrict__ slot_sys, SlotFilter f) {
    constexpr int SY = L + 1;
    constexpr int H = L / 2 + 1;  // z rows that can be non-zero (nz <= H)
    constexpr int ROW = 3 * SY;   // one z row: three components
    __shared__ cx<T> lds[L * ROW];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x;
    const int pos = blockIdx.y;
    const int slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int sys = slot_sys[slot];
    const int64_t cplane = int64_t(3) * g.nz * g.ny;
    cx<T>* col = Tb + (int64_t(pos) * g.mx + kx) * cplane;
    const bool perm = (g.ny & 7) == 0;
    for (int e = tid; e < L * ROW; e += NTY) {
        const int z = e / ROW, rem = e % ROW, c = rem / SY, y = rem % SY;
        lds[e] = (z < g.nz && y < g.ny) ? col[(int64_t(c) * g.nz + z) * g.ny + tpos(y, perm)]
                                        : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_tile<T, L, false, 3 * H, SY, 1, NTY>(lds, twy, tid);    // y: lines (z < H, c)
    fft_tile<T, L, false, 3 * SY, 1, ROW, NTY>(lds, twz, tid);  // z: lines (c, ky)
    const bool fx = kx > g.mx / 2;
    const int kxr = fx ? g.mx - kx : kx;
    const cx<T>* dslab = Dptr[sys] + int64_t(kxr) * 6 * H * H;
    for (int e = tid; e < H * H; e += NTY) {
        const int kzp = e / H, kyp = e % H;
        const cx<T>* dp = dslab + e;
        const cx<T> dxx = dp[0], dxy0 = dp[H * H], dxz0 = dp[2 * H * H];
        const cx<T> dyy = dp[3 * H * H], dyz0 = dp[4 * H * H], dzz = dp[5 * H * H];
        const int kz1 = (L - kzp) % L, ky1 = (L - kyp) % L;
        const int nzs = (kz1 != kzp) ? 2 : 1, nys = (ky1 != kyp) ? 2 : 1;
        for (int zi = 0; zi < nzs; ++zi) {
            const bool fz = zi != 0;
            const int kz = fz ? kz1 : kzp;
            for (int yi = 0; yi < nys; ++yi) {
                const bool fy = yi != 0;
                const int ky = fy ? ky1 : kyp;
                const cx<T> dxy = (fx != fy) ? -dxy0 : dxy0;
                const cx<T> dxz = (fx != fz) ? -dxz0 : dxz0;
                const cx<T> dyz = (fy != fz) ? -dyz0 : dyz0;
                cx<T>* u = lds + kz * ROW + ky;
                const cx<T> ux = u[0], uy = u[SY], uz = u[2 * SY];
                u[0] = dxx * ux + dxy * uy + dxz * uz;
                u[SY] = dxy * ux + dyy * uy + dyz * uz;
                u[2 * SY] = dxz * ux + dyz * uy + dzz * uz;
            }
        }
    }
    __syncthreads();
    fft_tile<T, L, true, 3 * SY, 1, ROW, NTY>(lds, twz, tid);
    fft_tile<T, L, true, 3 * H, SY, 1, NTY>(lds, twy, tid);
    for (int e = tid; e < 3 * g.nz * g.ny; e += NTY) {
        const int y = e % g.ny, cz = e / g.ny, z = cz % g.nz, c = cz / g.nz;
        col[int64_t(cz) * g.ny + tpos(y, perm)] = lds[z * ROW + c * SY + y];
    }
}

// ------------------------------------------------------ YZ (registers) -----
// The same column pass for L = 16 ... 64 (L divisible by 8) with the line
// transforms held in registers.  A line of length L belongs to a quad of
// adjacent lanes: lane n2 holds the L/4 points x[4 n1 + n2] and takes their
// L/4-point DFT in registers (compile-time Stockham stages); after the twiddle
// W_L^{n2 k1} the four lanes finish with a radix-4 butterfly through quad DPP
// moves, lane n2 ending with X[k1 + (L/4) rev2(n2)] (rev2 swaps the two bits).
// LDS only carries the transposes between the y and z passes: the plane as
// rows [c][ky] of length L + 1, over z.
//   phase 1: y-FFT of the lines (c, z < nz), loaded straight from HBM (the
//            zero padding y >= ny is never read), stored to LDS by ky;
//   phase 2: one quad per (c, ky): z-FFT back into its row; then D u over
//            all (ky, kz) by every thread; then one quad per (c, ky) again for
//            the z-iFFT (quad_fft_blk), keeping z < nz;
//   phase 3: y-iFFT of the lines (c, z < nz), y < ny stored straight to HBM.
template <int L>
constexpr bool yzr_ok() { return L % 8 == 0 && L >= 16 && L <= 64; }
template <int L>
constexpr int yzr_threads() { return (12 * L + 63) / 64 * 64; }  // a quad per (c, ky)

// Two adjacent complex values of a T line (16-byte aligned for FP32 when the
// line is permuted: ny is then a multiple of 8).
__device__ __forceinline__ void load_pair(const cx<float>* p, cx<float>& a, cx<float>& b) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    a = cx<float>{t.x, t.y};
    b = cx<float>{t.z, t.w};
}
__device__ __forceinline__ void load_pair(const cx<double>* p, cx<double>& a, cx<double>& b) {
    a = p[0];
    b = p[1];
}
__device__ __forceinline__ void store_pair(cx<float>* p, cx<float> a, cx<float> b) {
    *reinterpret_cast<float4*>(p) = float4{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ void store_pair(cx<double>* p, cx<double> a, cx<double> b) {
    p[0] = a;
    p[1] = b;
}

template <typename T, int L>
__global__ __launch_bounds__(yzr_threads<L>()) void k_yzconv_r(
    cx<T>* __restrict__ Tb, const cx<T>* const* __restrict__ Dptr, const cx<T>* __restrict__ twy,
    const cx<T>* __restrict__ twz, Geo g, const int* __restrict__ act,
    const int* __restrict__ slot_sys, SlotFilter f) {
    constexpr int Q = L / 4;
    constexpr int ZS = L + 1;      // LDS row stride over z / kz
    constexpr int HD = L / 2 + 1;  // D slab corner
    constexpr int NTR = yzr_threads<L>();
    __shared__ cx<T> lds[3 * L * ZS];
    const int tid = threadIdx.x;
    const int grp = tid >> 2, n2 = tid & 3;
    const int rb = ((n2 & 1) << 1) | (n2 >> 1);  // rev2(n2)
    const int kx = blockIdx.x;
    const int pos = blockIdx.y;
    const int slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int sys = slot_sys[slot];
    const int nz = g.nz, ny = g.ny;
    cx<T>* col = Tb + (int64_t(pos) * g.mx + kx) * (int64_t(3) * nz * ny);
    const cx<T> zero{T(0), T(0)};

    // phase 1: y-FFT of the lines (c, z)
    const bool perm = (ny & 7) == 0;
    for (int line = grp; line < 3 * nz; line += NTR / 4) {
        const int c = line / nz, z = line - (line / nz) * nz;
        const cx<T>* src = col + int64_t(line) * ny;
        cx<T> v[Q];
#pragma unroll
        for (int n1 = 0; n1 < Q; ++n1) v[n1] = zero;
        // raised wave priority while the loads go out: they start ahead of the
        // arithmetic of the other block on the CU (1.5 % on the nanorod lattice)
        __builtin_amdgcn_s_setprio(2);
        if (perm) {  // whole blocks of 8: lane n2 reads its pair at 8j + 2 n2
#pragma unroll
            for (int j = 0; 2 * j + 1 < Q / 2 + 1; ++j) {
                if (8 * j + 8 <= ny) load_pair(src + 8 * j + 2 * n2, v[2 * j], v[2 * j + 1]);
            }
        } else {
#pragma unroll
            for (int n1 = 0; n1 < Q / 2; ++n1) {
                const int y = 4 * n1 + n2;
                if (y < ny) v[n1] = src[y];
            }
        }
        __builtin_amdgcn_s_setprio(0);
        quad_fft<T, L, false>(v, n2, twy, twy);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) lds[(c * L + k1 + Q * rb) * ZS + z] = v[k1];
    }
    __syncthreads();

    // D slab of this kx (phase 2b).  The slab holds the corner ky', kz' <= L/2,
    // and one entry serves the frequencies (ky' or L - ky') x (kz' or L - kz')
    // through the parity of each component.  Interior entries
    // (0 < ky', kz' < L/2) give one work item of four frequencies for six
    // loads; consecutive lanes take consecutive ky', the fastest slab index
    // (coalesced).  The 4L - 4 frequencies on the lines ky or kz in {0, L/2}
    // are one item each.
    constexpr int HI = L / 2 - 1;
    constexpr int NI = HI * HI;
    constexpr int NEG = 4 * L - 4;
    constexpr int NII = (NI + NTR - 1) / NTR;
    constexpr int NIE = (NEG + NTR - 1) / NTR;
    constexpr int H2 = HD * HD;
    const bool fx = kx > g.mx / 2;
    const int kxr = fx ? g.mx - kx : kx;
    const cx<T>* __restrict__ dslab = Dptr[sys] + int64_t(kxr) * 6 * H2;
    const T sx = fx ? T(-1) : T(1);
    // edge frequency p: kz = 0 and kz = L/2 (all ky), then ky = 0 and
    // ky = L/2 (kz off those two)
    auto edge = [](int p, int& ky, int& kz) {
        if (p < 2 * L) {
            kz = p < L ? 0 : L / 2;
            ky = p < L ? p : p - L;
        } else {
            const int q = p - 2 * L;
            ky = q < L - 2 ? 0 : L / 2;
            kz = 1 + (q < L - 2 ? q : q - (L - 2));
            if (kz >= L / 2) ++kz;
        }
    };
    cx<T> di[NII][6], de[NIE][6];

    // phase 2a: z-FFT of the rows (c, ky), spectrum back into the row
    if (grp < 3 * L) {
        cx<T>* row = lds + grp * ZS;
        cx<T> u[Q];
#pragma unroll
        for (int n1 = 0; n1 < Q; ++n1) {
            const int z = 4 * n1 + n2;
            u[n1] = (n1 < Q / 2 && z < nz) ? row[z] : zero;
        }
        quad_fft<T, L, false>(u, n2, twz, twz);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) row[k1 + Q * rb] = u[k1];
    }
    // All D loads of a thread go out here, after its row is stored (the line
    // registers are free again) and before the barrier, so their latency
    // overlaps the wait for the other waves' z-FFTs.  Issued before the z-FFT
    // instead they would stay live through it and take the kernel past the
    // registers of five waves per SIMD.
    {
        __builtin_amdgcn_s_setprio(2);  // as for the loads of phase 1
#pragma unroll
        for (int it = 0; it < NII; ++it) {
            const int t = min(tid + it * NTR, NI - 1);
            const int kzp = 1 + t / HI, kyp = 1 + (t - (t / HI) * HI);
#pragma unroll
            for (int q = 0; q < 6; ++q) di[it][q] = gload(dslab + kzp * HD + kyp + q * H2);
        }
        const int wbase = tid & ~63;  // waves past the last edge item skip its loads
#pragma unroll
        for (int it = 0; it < NIE; ++it) {
            if (wbase + it * NTR < NEG) {
                int ky, kz;
                edge(min(tid + it * NTR, NEG - 1), ky, kz);
                const int o = (kz > L / 2 ? L - kz : kz) * HD + (ky > L / 2 ? L - ky : ky);
#pragma unroll
                for (int q = 0; q < 6; ++q) de[it][q] = gload(dslab + o + q * H2);
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    // phase 2b: D u at every (ky, kz), from the slab entries loaded above (a
    // wave that skipped the edge loads has no lane with p < NEG).  LDS rows at
    // an odd stride keep accesses in distinct banks.
    {
#pragma unroll
        for (int it = 0; it < NII; ++it) {
            const int t = tid + it * NTR;
            if (t < NI) {
                const int kzp = 1 + t / HI, kyp = 1 + (t - (t / HI) * HI);
                const cx<T>* d = di[it];
                const cx<T> dxy = sx * d[1], dxz = sx * d[2];  // parities at ky', kz'
                dmul3<T, L * ZS>(lds + kyp * ZS + kzp, d[0], dxy, dxz, d[3], d[4], d[5]);
                dmul3<T, L * ZS>(lds + (L - kyp) * ZS + kzp, d[0], -dxy, dxz, d[3], -d[4],
                                 d[5]);
                dmul3<T, L * ZS>(lds + kyp * ZS + (L - kzp), d[0], dxy, -dxz, d[3], -d[4],
                                 d[5]);
                dmul3<T, L * ZS>(lds + (L - kyp) * ZS + (L - kzp), d[0], -dxy, -dxz, d[3],
                                 d[4], d[5]);
            }
        }
#pragma unroll
        for (int it = 0; it < NIE; ++it) {
            const int p = tid + it * NTR;
            if (p < NEG) {
                int ky, kz;
                edge(p, ky, kz);
                const bool fy = ky > L / 2, fz = kz > L / 2;
                const cx<T>* d = de[it];
                const cx<T> dxy = (fx != fy) ? -d[1] : d[1];
                const cx<T> dxz = (fx != fz) ? -d[2] : d[2];
                const cx<T> dyz = (fy != fz) ? -d[4] : d[4];
                dmul3<T, L * ZS>(lds + ky * ZS + kz, d[0], dxy, dxz, d[3], dyz, d[5]);
            }
        }
    }
    __syncthreads();
    // phase 2c: z-iFFT of the rows (c, ky), keeping z < nz
    if (grp < 3 * L) {
        cx<T>* row = lds + grp * ZS;
        cx<T> u[Q];
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) u[k1] = row[k1 + Q * rb];
        quad_fft_blk<T, L, true>(u, n2, twz, twz);
        // z = 4 n1 + n2 < L/2: the row's slots z >= nz are never read again,
        // so every one is written (no branch per store)
#pragma unroll
        for (int n1 = 0; n1 < Q / 2; ++n1) row[4 * n1 + n2] = u[n1];
    }
    __syncthreads();

    // phase 3: y-iFFT of the lines (c, z) from the blocked spectrum (lane n2
    // reads ky = k1 + (L/4) rev2(n2)), output decimated (lane n2 holds
    // y = 4 n1 + n2); y < ny back to HBM, in pairs when the line is permuted
    for (int line = grp; line < 3 * nz; line += NTR / 4) {
        const int c = line / nz, z = line - (line / nz) * nz;
        cx<T> v[Q];
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) v[k1] = lds[(c * L + k1 + Q * rb) * ZS + z];
        quad_fft_blk<T, L, true>(v, n2, twy, twy);
        cx<T>* dst = col + int64_t(line) * ny;
        if (perm) {
#pragma unroll
            for (int j = 0; 2 * j + 1 < Q / 2 + 1; ++j) {
                if (8 * j + 8 <= ny) store_pair(dst + 8 * j + 2 * n2, v[2 * j], v[2 * j + 1]);
            }
        } else {
#pragma unroll
            for (int n1 = 0; n1 < Q / 2; ++n1) {
                const int y = 4 * n1 + n2;
                if (y < ny) dst[y] = v[n1];
            }
        }
    }
}

// ------------------------------------------------------------ launchers ----
#define DDA_FOR_EACH_LX(X) \
    X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#define DDA_FOR_EACH_LYZ(X) X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64)

template <typename T>
void launch_xfft_t(cx<T>* xin, const int* map, cx<T>* Tb, const cx<T>* tw_x, const Geo& g,
                   const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f,
                   hipStream_t s, CocgFold fo, BicgFold bf) {
    if (n_act == 0) return;
    if (2 * g.nx - 1 > g.mx) throw Error(-1, "x grid shorter than 2 nx - 1");
    int ng, nr;
    xsplit<T>(g, ng, nr);
    dim3 grid(3 * g.nz * ng, n_act);
    switch (g.mx) {
#define DDA_CASE(N)                                                                         \
    case N:                                                                                 \
        if (fuse_r)                                                                         \
            if (bf.kind == BICG_FOLD_S)                                                     \
                k_xfft_t<T, N, FUSE_BICG_S><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act,  \
                                                                fuse_r, f, ng, nr,           \
                                                                CocgFold{}, bf);             \
            else if (bf.kind == BICG_FOLD_P)                                                \
                k_xfft_t<T, N, FUSE_BICG_P><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act,  \
                                                                fuse_r, f, ng, nr,           \
                                                                CocgFold{}, bf);             \
            else                                                                            \
                k_xfft_t<T, N, FUSE_COCG><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act,    \
                                                              fuse_r, f, ng, nr, fo,         \
                                                              BicgFold{});                   \
        else                                                                                \
            k_xfft_t<T, N, 0><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act, nullptr, f, ng, \
                                                  nr, CocgFold{}, BicgFold{});              \
        break;
        DDA_FOR_EACH_LX(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    DDA_LAUNCH_CHECK();
}

template <typename T>
void launch_ixfft_t(const cx<T>* Tb, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                    const int* map, const cx<T>* tw_x, const Geo& g, const int* act,
                    const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                    hipStream_t s, const cx<T>* wv) {
    if (n_act == 0) return;
    if (2 * g.nx - 1 > g.mx) throw Error(-1, "x grid shorter than 2 nx - 1");
    if (mode == PACK_AX_DOTW && !wv) throw Error(-1, "PACK_AX_DOTW needs the vector w");
    int ng, nr;
    xsplit<T>(g, ng, nr);
    if (pack_fused(mode) && 3 * g.nz * ng > red.max_blocks)
        throw Error(-3, "reduction scratch too small for the fused pack kernel");
    dim3 grid(3 * g.nz * ng, n_act);
    switch (g.mx) {
#define DDA_IXT(N, M)                                                                        \
    k_ixfft_t<T, N, M><<<grid, NT, 0, s>>>(Tb, xin, ainv, yout, map, tw_x, g, act, slot_sys, f, \
                                           red, ng, nr, wv)
#define DDA_CASE(N)                                                                          \
    case N:                                                                                  \
        switch (mode) {                                                                      \
            case PACK_GX: DDA_IXT(N, PACK_GX); break;                                        \
            case PACK_AX: DDA_IXT(N, PACK_AX); break;                                        \
            case PACK_AX_COCG: DDA_IXT(N, PACK_AX_COCG); break;                              \
            case PACK_AX_DOTW: DDA_IXT(N, PACK_AX_DOTW); break;                              \
            case PACK_AX_TS: DDA_IXT(N, PACK_AX_TS); break;                                  \
            default: throw Error(-1, "unknown pack mode");                                   \
        }                                                                                    \
        break;
        DDA_FOR_EACH_LX(DDA_CASE)
#undef DDA_CASE
#undef DDA_IXT
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    DDA_LAUNCH_CHECK();
}

template <typename T>
void launch_yzconv(cx<T>* Tb, const cx<T>* const* Dptr, const cx<T>* tw_y, const cx<T>* tw_z,
                   const Geo& g, const int* act, const int* slot_sys, int n_act, SlotFilter f,
                   int nthreads, hipStream_t s) {
    if (n_act == 0) return;
    if (!yz_fused_ok(g, int(sizeof(cx<T>)))) throw Error(-1, "yz plane does not fit in LDS");
    dim3 grid(g.mx, n_act);
    switch (g.my) {
#define DDA_CASE(N)                                                                          \
    case N:                                                                                  \
        if constexpr (yzr_ok<N>() && yz_lds_bytes<T, N>() <= (size_t(120) << 10)) {        \
            (void)nthreads;                                                                  \
            k_yzconv_r<T, N><<<grid, yzr_threads<N>(), 0, s>>>(Tb, Dptr, tw_y, tw_z, g, act, \
                                                               slot_sys, f);                 \
        } else if constexpr (yz_lds_bytes<T, N>() <= (size_t(120) << 10)) {                  \
            k_yzconv<T, N, NTYZ><<<grid, NTYZ, 0, s>>>(Tb, Dptr, tw_y, tw_z, g, act,         \
                                                       slot_sys, f);                         \
        } else {                                                                             \
            throw Error(-1, "yz plane does not fit in LDS");                                 \
        }                                                                                    \
        break;
        DDA_FOR_EACH_LYZ(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "yz plane does not fit in LDS");
    }
    DDA_LAUNCH_CHECK();
}

// D (full grid, FP64) -> kx-slab layout [kx' <= mx/2][6][kz' <= L/2][ky' <= L/2]
template <typename T>
__global__ __launch_bounds__(256) void k_extract_yz(const z128* __restrict__ full,
                                                    cx<T>* __restrict__ out, Geo g) {
    const int hx = g.mx / 2 + 1, H = g.my / 2 + 1;
    const int64_t total = int64_t(hx) * 6 * H * H;
    for (int64_t t = blockIdx.x * int64_t(256) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * 256) {
        int64_t r = t;
        const int ky = int(r % H); r /= H;
        const int kz = int(r % H); r /= H;
        const int q = int(r % 6);
        const int kx = int(r / 6);
        out[t] = cvt<T>(full[((int64_t(q) * g.mz + kz) * g.my + ky) * g.mx + kx]);
    }
}

int64_t dyz_elems(const Geo& g) {
    return int64_t(g.mx / 2 + 1) * 6 * (g.my / 2 + 1) * (g.my / 2 + 1);
}

template <typename T>
void launch_extract_yz(const z128* full, cx<T>* out, const Geo& g, hipStream_t s) {
    const int64_t n = dyz_elems(g);
    const unsigned b = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
    k_extract_yz<T><<<b, 256, 0, s>>>(full, out, g);
    DDA_LAUNCH_CHECK();
}

template void launch_xfft_t<double>(z128*, const int*, z128*, const z128*, const Geo&, const int*,
                                    int, const z128*, SlotFilter, hipStream_t, CocgFold,
                                    BicgFold);
template void launch_xfft_t<float>(z64*, const int*, z64*, const z64*, const Geo&, const int*, int,
                                   const z64*, SlotFilter, hipStream_t, CocgFold, BicgFold);
template void launch_ixfft_t<double>(const z128*, const z128*, const z128*, z128*, const int*,
                                     const z128*, const Geo&, const int*, const int*, int, int,
                                     SlotFilter, RedScratch, hipStream_t, const z128*);
template void launch_ixfft_t<float>(const z64*, const z64*, const z64*, z64*, const int*,
                                    const z64*, const Geo&, const int*, const int*, int, int,
                                    SlotFilter, RedScratch, hipStream_t, const z64*);
template void launch_yzconv<double>(z128*, const z128* const*, const z128*, const z128*,
                                    const Geo&, const int*, const int*, int, SlotFilter, int,
                                    hipStream_t);
template void launch_yzconv<float>(z64*, const z64* const*, const z64*, const z64*, const Geo&,
                                   const int*, const int*, int, SlotFilter, int, hipStream_t);

std::vector<int> yz_thread_candidates(int L) {
    (void)L;  // the register kernel has one shape per L: nothing to tune
    return {};
}
template void launch_extract_yz<double>(const z128*, z128*, const Geo&, hipStream_t);
template void launch_extract_yz<float>(const z128*, z64*, const Geo&, hipStream_t);

}  // namespace dda

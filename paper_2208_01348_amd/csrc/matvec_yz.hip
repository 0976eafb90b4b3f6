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

namespace dda {

namespace {

constexpr int NT = 256;    // x kernels
constexpr int NTYZ = 512;  // yz kernel, default threads per block (the autotuner
                           // may pick 256 or 1024 for L >= 24; the butterflies
                           // are the same whichever thread computes them)

// rows of one (component, z) plane per x-kernel block
template <int LX>
constexpr int xrows() { return LX >= 1024 ? 2 : 2048 / LX; }

template <typename T, int L>
constexpr size_t yz_lds_bytes() { return size_t(L) * 3 * (L + 1) * 2 * sizeof(T); }

}  // namespace

bool yz_fused_ok(const Geo& g, int csize) {
    if (g.my != g.mz) return false;
    const size_t L = size_t(g.my);
    if (L > 64) return false;
    return L * 3 * (L + 1) * size_t(csize) <= size_t(120) << 10;
}

static int xgroups(const Geo& g) {
    int nr = 0;
    switch (g.mx) {
#define DDA_CASE(N) \
    case N:         \
        nr = xrows<N>(); \
        break;
        DDA_CASE(1) DDA_CASE(2) DDA_CASE(3) DDA_CASE(4) DDA_CASE(6) DDA_CASE(8) DDA_CASE(12)
        DDA_CASE(16) DDA_CASE(24) DDA_CASE(32) DDA_CASE(48) DDA_CASE(64) DDA_CASE(96)
        DDA_CASE(128) DDA_CASE(192) DDA_CASE(256) DDA_CASE(384) DDA_CASE(512)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    return (g.ny + nr - 1) / nr;
}

int yz_pack_blocks_per_slot(const Geo& g) { return 3 * g.nz * xgroups(g); }

// ------------------------------------------------------------------ X1 -----
template <typename T, int LX, bool FUSE_P>
__global__ __launch_bounds__(NT) void k_xfft_t(cx<T>* __restrict__ xin,
                                               const int* __restrict__ map,
                                               cx<T>* __restrict__ Tb,
                                               const cx<T>* __restrict__ tw, Geo g,
                                               const int* __restrict__ act,
                                               const cx<T>* __restrict__ fuse_r, SlotFilter f,
                                               int ngroups) {
    constexpr int NR = xrows<LX>();
    constexpr int LP = LX + 1;  // padded LDS row: the transposed read below hits spread banks
    __shared__ cx<T> lds[NR * LP];
    const int tid = threadIdx.x;
    const int pos = blockIdx.y;
    const int64_t slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int grp = blockIdx.x % ngroups;
    const int cz = blockIdx.x / ngroups;
    const int c = cz / g.nz, z = cz - (cz / g.nz) * g.nz;
    const int y0 = grp * NR;
    cx<T>* src = xin + (slot * 3 + c) * g.n_occ;
    const cx<T>* rsrc = FUSE_P ? fuse_r + (slot * 3 + c) * g.n_occ : nullptr;
    cx<T> beta{T(0), T(0)};
    bool reset = false;
    if (FUSE_P) {
        beta = cvt<T>(f.st[slot].beta);
        reset = f.st[slot].reset_p != 0;
    }
    for (int e = tid; e < NR * LX; e += NT) {
        const int r = e / LX, x = e % LX;
        const int y = y0 + r;
        cx<T> v{T(0), T(0)};
        if (y < g.ny && x < g.nx) {
            const int idx = map[(int64_t(z) * g.ny + y) * g.nx + x];
            if (idx >= 0) {
                v = src[idx];
                if (FUSE_P) {  // each occupied element is visited by exactly one thread
                    v = reset ? rsrc[idx] : rsrc[idx] + beta * v;
                    src[idx] = v;
                }
            }
        }
        lds[r * LP + x] = v;
    }
    __syncthreads();
    fft_tile<T, LX, false, NR, LP, 1, NT>(lds, tw, tid);
    const int64_t cplane = int64_t(3) * g.nz * g.ny;  // one kx column
    cx<T>* dst = Tb + int64_t(pos) * g.mx * cplane + (int64_t(c) * g.nz + z) * g.ny;
    for (int e = tid; e < NR * LX; e += NT) {
        const int kx = e / NR, r = e % NR;
        const int y = y0 + r;
        if (y < g.ny) dst[kx * cplane + y] = lds[r * LP + kx];
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
                                                RedScratch red, int ngroups) {
    constexpr int NR = xrows<LX>();
    constexpr int LP = LX + 1;
    __shared__ cx<T> lds[NR * LP];
    const int tid = threadIdx.x;
    const int pos = blockIdx.y;
    const int64_t slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int64_t sys = slot_sys[slot];
    const int grp = blockIdx.x % ngroups;
    const int cz = blockIdx.x / ngroups;
    const int c = cz / g.nz, z = cz - (cz / g.nz) * g.nz;
    const int y0 = grp * NR;
    const int64_t cplane = int64_t(3) * g.nz * g.ny;
    const cx<T>* src = Tb + int64_t(pos) * g.mx * cplane + (int64_t(c) * g.nz + z) * g.ny;
    for (int e = tid; e < NR * LX; e += NT) {
        const int kx = e / NR, r = e % NR;
        const int y = y0 + r;
        lds[r * LP + kx] = (y < g.ny) ? src[kx * cplane + y] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_tile<T, LX, true, NR, LP, 1, NT>(lds, tw, tid);
    const int64_t voff = (slot * 3 + c) * g.n_occ;
    double mu[2] = {0.0, 0.0};
    for (int e = tid; e < NR * LX; e += NT) {
        const int r = e / LX, x = e % LX;
        const int y = y0 + r;
        if (y < g.ny && x < g.nx) {
            const int idx = map[(int64_t(z) * g.ny + y) * g.nx + x];
            if (idx >= 0) {
                const cx<T> conv = lds[r * LP + x];
                if (MODE == PACK_GX) {
                    yout[voff + idx] = conv;
                } else {
                    const cx<T> xi = xin[voff + idx];
                    const cx<T> yi = xi * ainv[sys * g.n_occ + idx] - conv;
                    yout[voff + idx] = yi;
                    if (MODE == PACK_AX_COCG) {  // bilinear x^T y
                        mu[0] += double(xi.x) * yi.x - double(xi.y) * yi.y;
                        mu[1] += double(xi.x) * yi.y + double(xi.y) * yi.x;
                    }
                }
            }
        }
    }
    if constexpr (MODE == PACK_AX_COCG)  // partial rows; alpha is finalized by the caller
        block_partial<2, NT>(mu, red, int(slot), blockIdx.x);
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
    for (int e = tid; e < L * ROW; e += NTY) {
        const int z = e / ROW, rem = e % ROW, c = rem / SY, y = rem % SY;
        lds[e] = (z < g.nz && y < g.ny) ? col[(int64_t(c) * g.nz + z) * g.ny + y]
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
        col[e] = lds[z * ROW + c * SY + y];
    }
}

// ------------------------------------------------------------ launchers ----
#define DDA_FOR_EACH_LX(X) \
    X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#define DDA_FOR_EACH_LYZ(X) X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64)

template <typename T>
void launch_xfft_t(cx<T>* xin, const int* map, cx<T>* Tb, const cx<T>* tw_x, const Geo& g,
                   const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f,
                   hipStream_t s) {
    if (n_act == 0) return;
    const int ng = xgroups(g);
    dim3 grid(3 * g.nz * ng, n_act);
    switch (g.mx) {
#define DDA_CASE(N)                                                                         \
    case N:                                                                                 \
        if (fuse_r)                                                                         \
            k_xfft_t<T, N, true><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act, fuse_r, f,  \
                                                     ng);                                   \
        else                                                                                \
            k_xfft_t<T, N, false><<<grid, NT, 0, s>>>(xin, map, Tb, tw_x, g, act, nullptr,   \
                                                      f, ng);                               \
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
                    hipStream_t s) {
    if (n_act == 0) return;
    const int ng = xgroups(g);
    if (mode == PACK_AX_COCG && 3 * g.nz * ng > red.max_blocks)
        throw Error(-3, "reduction scratch too small for the fused pack kernel");
    dim3 grid(3 * g.nz * ng, n_act);
    switch (g.mx) {
#define DDA_CASE(N)                                                                          \
    case N:                                                                                  \
        if (mode == PACK_GX)                                                                 \
            k_ixfft_t<T, N, PACK_GX><<<grid, NT, 0, s>>>(Tb, xin, ainv, yout, map, tw_x, g,   \
                                                         act, slot_sys, f, red, ng);            \
        else if (mode == PACK_AX)                                                            \
            k_ixfft_t<T, N, PACK_AX><<<grid, NT, 0, s>>>(Tb, xin, ainv, yout, map, tw_x, g,   \
                                                         act, slot_sys, f, red, ng);            \
        else                                                                                 \
            k_ixfft_t<T, N, PACK_AX_COCG><<<grid, NT, 0, s>>>(Tb, xin, ainv, yout, map, tw_x, \
                                                              g, act, slot_sys, f, red, ng);    \
        break;
        DDA_FOR_EACH_LX(DDA_CASE)
#undef DDA_CASE
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
        if constexpr (yz_lds_bytes<T, N>() <= (size_t(120) << 10)) {                         \
            if constexpr (N >= 24) {                                                         \
                if (nthreads == 256) {                                                       \
                    k_yzconv<T, N, 256><<<grid, 256, 0, s>>>(Tb, Dptr, tw_y, tw_z, g, act,   \
                                                             slot_sys, f);                   \
                    break;                                                                   \
                }                                                                            \
                if (nthreads == 1024) {                                                      \
                    k_yzconv<T, N, 1024><<<grid, 1024, 0, s>>>(Tb, Dptr, tw_y, tw_z, g, act, \
                                                               slot_sys, f);                 \
                    break;                                                                   \
                }                                                                            \
            }                                                                                \
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
                                    int, const z128*, SlotFilter, hipStream_t);
template void launch_xfft_t<float>(z64*, const int*, z64*, const z64*, const Geo&, const int*, int,
                                   const z64*, SlotFilter, hipStream_t);
template void launch_ixfft_t<double>(const z128*, const z128*, const z128*, z128*, const int*,
                                     const z128*, const Geo&, const int*, const int*, int, int,
                                     SlotFilter, RedScratch, hipStream_t);
template void launch_ixfft_t<float>(const z64*, const z64*, const z64*, z64*, const int*,
                                    const z64*, const Geo&, const int*, const int*, int, int,
                                    SlotFilter, RedScratch, hipStream_t);
template void launch_yzconv<double>(z128*, const z128* const*, const z128*, const z128*,
                                    const Geo&, const int*, const int*, int, SlotFilter, int,
                                    hipStream_t);
template void launch_yzconv<float>(z64*, const z64* const*, const z64*, const z64*, const Geo&,
                                   const int*, const int*, int, SlotFilter, int, hipStream_t);

std::vector<int> yz_thread_candidates(int L) {
    if (L >= 24) return {256, 512, 1024};
    return {NTYZ};
}
template void launch_extract_yz<double>(const z128*, z128*, const Geo&, hipStream_t);
template void launch_extract_yz<float>(const z128*, z64*, const Geo&, hipStream_t);

}  // namespace dda

// Three-kernel FFT matvec for lattices whose zero-padded xy plane of one field
// component fits in LDS (FP32, mx = my = 96 or 128).
//
// The five-pass chain streams two intermediates through HBM between its x and
// y passes: the x-transformed rows (6N complex per right-hand side on a cube)
// are written by the x pass and read back by the y pass, and the same on the
// way back.  Here one block takes a whole (component, z) plane in LDS: it
// gathers the rows y < ny, takes the x-FFT of every row and then the y-FFT of
// every column, each line held in registers by a lane quad (quad_fft.h), and
// stores the spectrum rows straight into the grid buffer the z pass reads.
// The inverse kernel mirrors it and ends with the pack of the five-pass
// chain.  HBM traffic per right-hand side: 48N complex instead of
// 72N (the z pass, 24N, is unchanged).
//   XY  gather (+ the folded Krylov update) + x-FFT + y-FFT -> G[c][z][ky][kx]
//   Z   k_zconv2 (z-FFT, D u, z-iFFT), as in the five-pass chain
//   IXY y-iFFT + x-iFFT + pack (x/alpha - (G x), the fused partial rows)
// The transforms are the same unnormalised DFTs as in the five-pass chain;
// only their factorisation differs, so results agree to rounding.
#include <algorithm>

#include "fft_core.h"
#include "kernels.h"
#include "quad_fft.h"

namespace dda {

namespace {

// The plane in LDS: rows y < ny of stride L + 4 complex elements.  A row
// holds either the values x < L/2 at position x, or the x spectrum with kx at
// position kx + kx / (L/4) (one spare slot per quarter of the row).  With a
// stride of 4 mod 16, the 16 lanes of each quarter-wave touch 16 distinct
// 8-byte bank pairs in every access pattern of the kernels: 4 columns x 4
// rows 4 n1 + n2 (column transforms), and 4 rows x 4 lanes of a row quad
// (x = 4 n1 + n2, or kx = k1 + (L/4) rev2(n2)).
template <int L>
constexpr int xy_stride() { return L + 4; }
template <int L>
__device__ __forceinline__ int xy_kpos(int kx) { return kx + kx / (L / 4); }
// Waves per SIMD to fit: two blocks of 4 L threads per CU, which the LDS
// plane allows (at most 128 VGPRs for L = 128).
constexpr int kXyWavesPerEu = 4;

}  // namespace

bool xy_fused_ok(const Geo& g, int csize) {
    if (csize != int(sizeof(z64)) || yz_fused_ok(g, csize)) return false;
    if (g.mx != g.my || (g.mx != 96 && g.mx != 128)) return false;
    return 2 * g.nx <= g.mx && 2 * g.ny <= g.my;
}

int xy_pack_blocks_per_slot(const Geo& g) { return 3 * g.nz; }

// Gather of the plane's rows y < ny (x < nx; the columns x >= L/2 are the
// zero padding, never stored), with the Krylov update of the mode FUSE done
// in place as in k_unpack_xfft (the COCG direction update, with or without
// the folded end of the previous iteration, or the BiCGStab s or p update);
// then the x-FFT of each row by a lane quad (lane n2 holds x = 4 n1 + n2 and
// ends with kx = k1 + (L/4) rev2(n2)), written back into the row, and the
// y-FFT of the L columns, one quad per column, stored straight to the grid
// buffer.  The blocks of a slot are its 3 nz planes (z fastest): the rows a
// folded s update writes are xy_pack_blocks_per_slot of them.
template <typename T, int L, int FUSE>
__global__ __launch_bounds__(4 * L, kXyWavesPerEu) void k_xyfft(cx<T>* __restrict__ xin,
                                                               const int* __restrict__ map,
                                                               cx<T>* __restrict__ G,
                                                               const cx<T>* __restrict__ tw, Geo g,
                                                               const int* __restrict__ act,
                                                               const cx<T>* __restrict__ fuse_r,
                                                               SlotFilter f, CocgFold fo,
                                                               BicgFold bf) {
    constexpr int NTB = 4 * L;
    constexpr int S = xy_stride<L>();
    constexpr int HL = L / 2;
    constexpr int Q = L / 4;
    constexpr bool FUSE_P = FUSE == FUSE_COCG;
    constexpr bool FUSE_S = FUSE == FUSE_BICG_S;
    constexpr bool FUSE_BP = FUSE == FUSE_BICG_P;
    __shared__ cx<T> lds[HL * S];
    __shared__ cx<T> twl[L];
    const int tid = threadIdx.x;
    const int z = blockIdx.x, c = blockIdx.y, pos = blockIdx.z;
    const int64_t slot = act ? act[pos] : pos;
    const bool lead = z == 0 && c == 0;
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
    for (int t = tid; t < L; t += NTB) twl[t] = tw[t];
    const int ny = g.ny;
    cx<T>* src = xin + (slot * 3 + c) * g.n_occ;
    const cx<T>* rsrc = FUSE ? fuse_r + (slot * 3 + c) * g.n_occ : nullptr;
    const cx<T>* vsrc = (FUSE_S || FUSE_BP)
                            ? static_cast<const cx<T>*>(bf.v) + (slot * 3 + c) * g.n_occ
                            : nullptr;
    // element e of the plane: row y = e / HL, column x = e % HL; every index
    // load, then every data load, is issued before the first use
    constexpr int NE = (HL * HL + NTB - 1) / NTB;
    const cx<T> zero{T(0), T(0)};
    int idx[NE];
    row_indices<NE, NTB, HL>(map + int64_t(z) * ny * g.nx, ny, g.nx, tid, idx);
    // the update's scalars: the folded row sums go out while the index loads
    // are in flight, ahead of the data loads
    cx<T> beta{T(0), T(0)};
    bool reset = false;
    if (FUSE_P) {
        if (fold) {
            z128 b;
            if (!cocg_fold<NTB>(fo, int(slot), lead, b)) return;
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
            sact = bicg_sfold<NTB>(bf, int(slot), lead, a);
            alpha = cvt<T>(a);
        }
    }
    if constexpr (FUSE_BP) {
        z128 b, o;
        sact = bicg_pfold<NTB>(bf, int(slot), status0, lead, b, o);
        bt = cvt<T>(b);
        om = cvt<T>(o);
    }
    cx<T> v[NE], w[FUSE ? NE : 1], u[FUSE_S || FUSE_BP ? NE : 1];
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
            if constexpr (FUSE_P) w[q] = rsrc[i];
        }
    }
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + q * NTB;
        const int y = e / HL, x = e - (e / HL) * HL;
        const bool occ = idx[q] >= 0;
        cx<T> vq;
        if constexpr (FUSE_S) {
            if (sact) {
                vq = bicg_s_of(w[q], alpha, u[q]);
                if (occ) s2 += bicg_norm2(vq);
            } else {
                vq = v[q];
            }
        } else if constexpr (FUSE_BP) {
            vq = v[q];
            if (sact) {
                const cx<T> upd = bicg_p_of(w[q], bt, vq, om, u[q]);
                vq.x = upd.x;  // component-wise, as in k_unpack_xfft
                vq.y = upd.y;
            }
        } else {
            vq = v[q];
        }
        if constexpr (FUSE_P) {
            const cx<T> upd = w[q] + beta * vq;
            vq.x = reset ? w[q].x : upd.x;
            vq.y = reset ? w[q].y : upd.y;
        }
        vq.x = occ ? vq.x : T(0);
        vq.y = occ ? vq.y : T(0);
        // each occupied element: exactly one thread
        if ((FUSE_P || ((FUSE_S || FUSE_BP) && sact)) && occ) src[idx[q]] = vq;
        if (y < ny) lds[y * S + x] = vq;
    }
    if constexpr (FUSE_S) {
        if (sact) {  // ||s||^2 rows, one per block of the slot (block-uniform)
            double pr[1] = {s2};
            block_partial<1, NTB, 6>(pr, bf.red, int(slot), blockIdx.x + gridDim.x * c);
        }
    }
    __syncthreads();
    const int grp = tid >> 2, n2 = tid & 3;
    const int rb = ((n2 & 1) << 1) | (n2 >> 1);  // rev2(n2)
    cx<T> a[Q];
    if (grp < ny) {  // x-FFT of row y = grp, in place (one wave holds the whole quad)
        cx<T>* row = lds + grp * S;
#pragma unroll
        for (int n1 = 0; n1 < Q; ++n1) a[n1] = n1 < Q / 2 ? row[4 * n1 + n2] : zero;
        quad_fft<T, L, false>(a, n2, tw, twl);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) row[xy_kpos<L>(k1 + Q * rb)] = a[k1];
    }
    __syncthreads();
    // y-FFT of column kx = grp: rows y >= ny are the zero padding (never written)
    const int kx = grp;
#pragma unroll
    for (int n1 = 0; n1 < Q; ++n1) {
        const int y = 4 * n1 + n2;
        a[n1] = zero;
        if (n1 < Q / 2) {
            const cx<T> t = lds[y * S + xy_kpos<L>(kx)];
            a[n1].x = y < ny ? t.x : T(0);
            a[n1].y = y < ny ? t.y : T(0);
        }
    }
    quad_fft<T, L, false>(a, n2, tw, twl);
    cx<T>* dst = G + ((int64_t(pos) * 3 + c) * g.nz + z) * int64_t(L) * L + kx;
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) dst[int64_t(k1 + Q * rb) * L] = a[k1];
}

// y-iFFT of every column (one quad per column, from the blocked spectrum the
// z pass leaves in place) keeping y < ny, x-iFFT of those rows by a quad per
// row keeping x < L/2, then the pack of k_ixfft_pack for the plane's rows.
template <typename T, int L, int MODE>
__global__ __launch_bounds__(4 * L, kXyWavesPerEu) void k_ixyfft_pack(const cx<T>* __restrict__ G,
                                                       const cx<T>* __restrict__ xin,
                                                       const cx<T>* __restrict__ ainv,
                                                       cx<T>* __restrict__ yout,
                                                       const int* __restrict__ map,
                                                       const cx<T>* __restrict__ tw, Geo g,
                                                       const int* __restrict__ act,
                                                       const int* __restrict__ slot_sys,
                                                       SlotFilter f, RedScratch red,
                                                       const cx<T>* __restrict__ wv) {
    constexpr int NTB = 4 * L;
    constexpr int S = xy_stride<L>();
    constexpr int HL = L / 2;
    constexpr int Q = L / 4;
    __shared__ cx<T> lds[HL * S];
    __shared__ cx<T> twl[L];
    const int tid = threadIdx.x;
    const int z = blockIdx.x, c = blockIdx.y, pos = blockIdx.z;
    const int64_t slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    map += slot * g.map_stride;
    const int nx = g.nx, ny = g.ny;
    const int kx = tid >> 2, n2 = tid & 3;
    const int rb = ((n2 & 1) << 1) | (n2 >> 1);
    const cx<T>* src = G + ((int64_t(pos) * 3 + c) * g.nz + z) * int64_t(L) * L + kx;
    cx<T> a[Q];
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) a[k1] = src[int64_t(k1 + Q * rb) * L];
    for (int t = tid; t < L; t += NTB) twl[t] = tw[t];
    __syncthreads();
    quad_fft_blk<T, L, true>(a, n2, tw, twl);
    // every row y < L/2 is stored (rows y >= ny are never read): a test per
    // store would put each output's last butterfly in a branch of its own,
    // and the values held across those branches spill
#pragma unroll
    for (int n1 = 0; n1 < Q / 2; ++n1) lds[(4 * n1 + n2) * S + xy_kpos<L>(kx)] = a[n1];
    __syncthreads();
    if (kx < ny) {  // x-iFFT of row y = kx (the quad index), in place
        cx<T>* row = lds + kx * S;
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) a[k1] = row[xy_kpos<L>(k1 + Q * rb)];
        quad_fft_blk<T, L, true>(a, n2, tw, twl);
#pragma unroll
        for (int n1 = 0; n1 < Q / 2; ++n1) row[4 * n1 + n2] = a[n1];
    }
    __syncthreads();
    const int64_t sys = slot_sys[slot];
    const int64_t voff = (slot * 3 + c) * g.n_occ;
    constexpr int NE = (HL * HL + NTB - 1) / NTB;
    int idx[NE];
    row_indices<NE, NTB, HL>(map + int64_t(z) * ny * nx, ny, nx, tid, idx);
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
        const int e = tid + q * NTB;
        const int y = e / HL, x = e - (e / HL) * HL;
        const cx<T> conv = lds[y * S + x];
        if (MODE == PACK_GX) {
            yout[voff + idx[q]] = conv;
        } else {
            const cx<T> yi = xv[q] * av[q] - conv;
            yout[voff + idx[q]] = yi;
            if constexpr (MODE == PACK_AX_DOTW) pack_dots<T, MODE>(mu, xv[q], yi, wq[q]);
            else pack_dots<T, MODE>(mu, xv[q], yi, yi);
        }
    }
    pack_rows<MODE, NTB>(mu, red, int(slot), blockIdx.y * gridDim.x + blockIdx.x);
}

#define DDA_FOR_EACH_LXY(X) X(96) X(128)

template <typename T>
void launch_xyfft(cx<T>* xin, const int* map, cx<T>* G, const cx<T>* tw, const Geo& g,
                  const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f, hipStream_t s,
                  CocgFold fo, BicgFold bf) {
    if (n_act == 0) return;
    if constexpr (sizeof(T) != sizeof(float)) {
        throw Error(-1, "the fused xy chain is FP32 only");
    } else {
        if (!xy_fused_ok(g, int(sizeof(cx<T>)))) throw Error(-1, "xy plane does not fit in LDS");
        const dim3 grid(unsigned(g.nz), 3, unsigned(n_act));
        switch (g.mx) {
#define DDA_XY(N, M, FO, BF, R)                                                               \
    k_xyfft<T, N, M><<<grid, 4 * N, 0, s>>>(xin, map, G, tw, g, act, R, f, FO, BF)
#define DDA_CASE(N)                                                                           \
    case N:                                                                                   \
        if (fuse_r && bf.kind == BICG_FOLD_S) DDA_XY(N, FUSE_BICG_S, CocgFold{}, bf, fuse_r);   \
        else if (fuse_r && bf.kind == BICG_FOLD_P) DDA_XY(N, FUSE_BICG_P, CocgFold{}, bf, fuse_r); \
        else if (fuse_r) DDA_XY(N, FUSE_COCG, fo, BicgFold{}, fuse_r);                        \
        else DDA_XY(N, FUSE_NONE, CocgFold{}, BicgFold{}, nullptr);                           \
        break;
            DDA_FOR_EACH_LXY(DDA_CASE)
#undef DDA_CASE
#undef DDA_XY
            default:
                throw Error(-1, "unsupported xy plane length");
        }
        DDA_LAUNCH_CHECK();
    }
}

template <typename T>
void launch_ixyfft_pack(const cx<T>* G, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                        const int* map, const cx<T>* tw, const Geo& g, const int* act,
                        const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                        hipStream_t s, const cx<T>* wv) {
    if (n_act == 0) return;
    if constexpr (sizeof(T) != sizeof(float)) {
        throw Error(-1, "the fused xy chain is FP32 only");
    } else {
        if (!xy_fused_ok(g, int(sizeof(cx<T>)))) throw Error(-1, "xy plane does not fit in LDS");
        if (pack_fused(mode) && xy_pack_blocks_per_slot(g) > red.max_blocks)
            throw Error(-3, "reduction scratch too small for the fused pack kernel");
        if (mode == PACK_AX_DOTW && !wv) throw Error(-1, "PACK_AX_DOTW needs the vector w");
        const dim3 grid(unsigned(g.nz), 3, unsigned(n_act));
        switch (g.mx) {
#define DDA_IXP(N, M)                                                                      \
    k_ixyfft_pack<T, N, M><<<grid, 4 * N, 0, s>>>(G, xin, ainv, yout, map, tw, g, act,       \
                                                  slot_sys, f, red, wv)
#define DDA_CASE(N)                                                                        \
    case N:                                                                                \
        switch (mode) {                                                                    \
            case PACK_GX: DDA_IXP(N, PACK_GX); break;                                      \
            case PACK_AX: DDA_IXP(N, PACK_AX); break;                                      \
            case PACK_AX_COCG: DDA_IXP(N, PACK_AX_COCG); break;                            \
            case PACK_AX_DOTW: DDA_IXP(N, PACK_AX_DOTW); break;                            \
            case PACK_AX_TS: DDA_IXP(N, PACK_AX_TS); break;                                \
            default: throw Error(-1, "unknown pack mode");                                 \
        }                                                                                  \
        break;
            DDA_FOR_EACH_LXY(DDA_CASE)
#undef DDA_CASE
#undef DDA_IXP
            default:
                throw Error(-1, "unsupported xy plane length");
        }
        DDA_LAUNCH_CHECK();
    }
}

template void launch_xyfft<double>(z128*, const int*, z128*, const z128*, const Geo&, const int*,
                                   int, const z128*, SlotFilter, hipStream_t, CocgFold, BicgFold);
template void launch_xyfft<float>(z64*, const int*, z64*, const z64*, const Geo&, const int*, int,
                                  const z64*, SlotFilter, hipStream_t, CocgFold, BicgFold);
template void launch_ixyfft_pack<double>(const z128*, const z128*, const z128*, z128*,
                                         const int*, const z128*, const Geo&, const int*,
                                         const int*, int, int, SlotFilter, RedScratch,
                                         hipStream_t, const z128*);
template void launch_ixyfft_pack<float>(const z64*, const z64*, const z64*, z64*, const int*,
                                        const z64*, const Geo&, const int*, const int*, int, int,
                                        SlotFilter, RedScratch, hipStream_t, const z64*);

}  // namespace dda

// FFT matvec chain of the DDA operator on gfx950, and the interaction
// spectrum D it multiplies by.
//
// The DDA operator (A x)_i = x_i/alpha_i - sum_{j != i} G(r_i - r_j) x_j has a
// block-Toeplitz interaction part on the cubic lattice.  Embedding it in a
// circulant of size mx x my x mz (each >= 2n - 1) turns it into a 3D cyclic
// convolution: zero-pad x, forward FFT, multiply by the 3x3 symmetric
// spectrum D at every frequency, inverse FFT, keep the lattice part.
//
// The 3D transforms are done axis by axis so that every pass streams HBM
// once, and each pass skips what the zero padding makes trivial:
//   K1 unpack + x-FFT : rows (z<nz, y<ny) gathered from the compact vector
//   K2 y-FFT          : columns of the nz planes, ny non-zero inputs
//   K3 z-conv         : z-FFT of nz inputs, D multiply, z-iFFT keeping nz
//   K4 y-iFFT         : keep ny outputs
//   K5 x-iFFT + pack  : keep nx outputs, scatter to occupied cells, add x/alpha
// Lines are staged in LDS in tiles whose global rows are contiguous
// (coalesced), and transformed there by the compile-time planned Stockham
// kernels of fft_core.h.
#include <algorithm>
#include <cmath>

#include "fft_core.h"
#include "kernels.h"

namespace dda {

constexpr int NTHR = 256;

constexpr int pow2floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}
constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// rows per block for row kernels: about 2048 elements per block in FP32 and
// 1024 in FP64 (16 KB of LDS either way, so more blocks are resident to hide
// the gather and store latencies of the FP64 x kernels)
constexpr int row_elems(int csize) { return csize == 16 ? 1024 : 2048; }
template <typename T, int L>
constexpr int rows_nl() {
    constexpr int R = row_elems(int(sizeof(cx<T>)));
    return L >= R ? 1 : R / L;
}
// columns per block for strided-axis kernels (default; the autotuner may
// pick another width for L >= kTuneMinL)
template <typename T, int L>
constexpr int mid_tx() { return clampi(pow2floor(2048 / L), 1, sizeof(T) == 8 ? 16 : 32); }
// columns per z-conv block: two mirror sets x 3 components x TX lines of
// length L (default: within 32 KB of LDS)
template <typename T, int L>
constexpr int zconv_tx() {
    return clampi(pow2floor(32768 / (6 * L * int(2 * sizeof(T)))), 1, sizeof(T) == 8 ? 4 : 8);
}
// Tile widths the autotuner may choose (at most 64 KB of LDS per block).
// The width only changes how many lines share a block; every line's
// arithmetic is the same, so all widths give identical results.
constexpr int kTuneMinL = 24;
template <typename T, int L, int TX>
constexpr bool mid_fits() { return size_t(L) * TX * 2 * sizeof(T) <= (size_t(64) << 10); }
template <typename T, int L, int TX>
constexpr bool zconv_fits() { return size_t(6) * L * TX * 2 * sizeof(T) <= (size_t(64) << 10); }

#define DDA_FOR_EACH_L(X) \
    X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

bool fft_length_supported(int L) {
    switch (L) {
#define DDA_CASE(N) case N:
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        return true;
        default:
            return false;
    }
}

// ---------------------------------------------------------------- K1 ------
// FUSE: as k_xfft_t (plain gather, the COCG direction update, or the
// BiCGStab s or p update).
template <typename T, int L, int FUSE>
__global__ __launch_bounds__(NTHR) void k_unpack_xfft(cx<T>* __restrict__ xin,
                                                      const int* __restrict__ map,
                                                      cx<T>* __restrict__ G,
                                                      const cx<T>* __restrict__ tw, Geo g,
                                                      const int* __restrict__ act,
                                                      const cx<T>* __restrict__ fuse_r,
                                                      SlotFilter f, CocgFold fo, BicgFold bf) {
    constexpr bool FUSE_P = FUSE == FUSE_COCG;
    constexpr bool FUSE_S = FUSE == FUSE_BICG_S;
    constexpr bool FUSE_BP = FUSE == FUSE_BICG_P;
    constexpr int NL = rows_nl<T, L>();
    constexpr int RP = padded_len<L>();  // row pitch (one spare slot per 16 elements)
    __shared__ cx<T> lds[NL * RP];
    __shared__ cx<T> twl[L];
    const int tid = threadIdx.x;
    const int c = blockIdx.y;
    const int pos = blockIdx.z;
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
    for (int t = tid; t < L; t += NTHR) twl[t] = tw[t];
    const int nrows = g.nz * g.ny;
    const int row0 = blockIdx.x * NL;
    cx<T>* src = xin + (slot * 3 + c) * g.n_occ;
    const cx<T>* rsrc = FUSE ? fuse_r + (slot * 3 + c) * g.n_occ : nullptr;
    const cx<T>* vsrc = (FUSE_S || FUSE_BP)
                            ? static_cast<const cx<T>*>(bf.v) + (slot * 3 + c) * g.n_occ
                            : nullptr;
    // only x < (L+1)/2 can be occupied; every index load, then every data
    // load, is issued before the first use (clamped addresses, masked after)
    constexpr int HX = (L + 1) / 2;
    constexpr int NE = (NL * HX + NTHR - 1) / NTHR;
    const cx<T> zero{T(0), T(0)};
    int idx[NE];
    row_indices<NE, NTHR, HX>(map + int64_t(row0) * g.nx, min(NL, nrows - row0), g.nx, tid, idx);
    // the direction update's scalars: the folded finalizer's row loads go
    // out while the index loads are in flight, ahead of the data loads
    cx<T> beta{T(0), T(0)};
    bool reset = false;
    if (FUSE_P) {
        if (fold) {
            z128 b;
            if (!cocg_fold<NTHR>(fo, int(slot), blockIdx.x == 0 && c == 0, b)) return;
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
            sact = bicg_sfold<NTHR>(bf, int(slot), blockIdx.x == 0 && c == 0, a);
            alpha = cvt<T>(a);
        }
    }
    if constexpr (FUSE_BP) {
        z128 b, o;
        sact = bicg_pfold<NTHR>(bf, int(slot), status0, blockIdx.x == 0 && c == 0, b, o);
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
        const int e = tid + q * NTHR;
        const int rr = e / HX, x = e - (e / HX) * HX;
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
                vq.x = upd.x;  // component-wise: a select of the whole FP64 pair goes
                vq.y = upd.y;  // through scratch
            }
        } else {
            vq = v[q];
        }
        if constexpr (FUSE_P) {
            const cx<T> upd = w[q] + beta * vq;
            vq.x = reset ? w[q].x : upd.x;  // component selects: a select of the
            vq.y = reset ? w[q].y : upd.y;  // whole FP64 pair goes through scratch
        }
        vq.x = occ ? vq.x : T(0);
        vq.y = occ ? vq.y : T(0);
        // each occupied element: exactly one thread
        if ((FUSE_P || ((FUSE_S || FUSE_BP) && sact)) && occ) src[idx[q]] = vq;
        // (no test where the elements cover the rows exactly: the compiler does
        // not prove rr < NL from the block size, and the branch it made held back
        // that element's index and data loads until the others had returned)
        if (NE * NTHR <= NL * HX || rr < NL) {
            lds[rr * RP + line_pos<true>(x)] = vq;
            if (x + HX < L) lds[rr * RP + line_pos<true>(x + HX)] = zero;
        }
    }
    if constexpr (FUSE_S) {
        if (sact) {  // ||s||^2 rows, one per block of the slot (block-uniform)
            double pr[1] = {s2};
            block_partial<1, NTHR, 6>(pr, bf.red, int(slot), blockIdx.x + gridDim.x * c);
        }
    }
    __syncthreads();
    fft_tile<T, L, false, NL, RP, 1, NTHR, true>(lds, twl, tid);
    cx<T>* dst = G + (int64_t(pos) * 3 + c) * g.nz * g.my * int64_t(g.mx);
    if constexpr (sizeof(T) == 4) {
        // FP32: every LDS read before the first store (32.8 against 34.6 us on
        // 64^3); in FP64 the held values cost more than they gain
        constexpr int NST = (NL * L + NTHR - 1) / NTHR;
        cx<T> t[NST];
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            const int e = min(tid + q * NTHR, NL * L - 1);
            t[q] = lds[(e / L) * RP + line_pos<true>(e % L)];
        }
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            const int e = tid + q * NTHR;
            const int rr = e / L, x = e % L;
            const int row = row0 + rr;
            if (e < NL * L && row < nrows) {
                const int z = row / g.ny, y = row - z * g.ny;
                dst[(int64_t(z) * g.my + y) * g.mx + x] = t[q];
            }
        }
    } else {
        for (int e = tid; e < NL * L; e += NTHR) {
            const int rr = e / L, x = e % L;
            const int row = row0 + rr;
            if (row < nrows) {
                const int z = row / g.ny, y = row - z * g.ny;
                dst[(int64_t(z) * g.my + y) * g.mx + x] = lds[rr * RP + line_pos<true>(x)];
            }
        }
    }
}

// ------------------------------------------------------------ K2 / K4 -----
// FFT along the middle axis of data[outer][L][inner]: the first n_in rows are
// read (the rest are zero), the first n_out rows are written.
template <typename T, int L, bool INV, int TX>
__global__ __launch_bounds__(NTHR) void k_fft_mid(cx<T>* __restrict__ data,
                                                  const cx<T>* __restrict__ tw, int64_t inner,
                                                  int n_in, int n_out, int64_t outer_stride,
                                                  int64_t tiles_per_outer) {
    __shared__ cx<T> lds[L * TX];
    __shared__ cx<T> twl[L];  // twiddles in LDS (51 against 55 us, FP32 y pass on 64^3)
    const int tid = threadIdx.x;
    for (int t = tid; t < L; t += NTHR) twl[t] = tw[t];
    const int64_t o = blockIdx.x / tiles_per_outer;
    const int64_t col0 = (blockIdx.x - o * tiles_per_outer) * TX;
    cx<T>* base = data + o * outer_stride + col0;
    {
        constexpr int NLD = (L * TX + NTHR - 1) / NTHR;
        cx<T> t[NLD];
#pragma unroll
        for (int q = 0; q < NLD; ++q) {  // every load issued before the first store
            const int e = tid + q * NTHR;
            const int row = e / TX, col = e % TX;
            t[q] = cx<T>{T(0), T(0)};
            if (row < n_in && col0 + col < inner) t[q] = base[int64_t(row) * inner + col];
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * NTHR;
            if (e < L * TX) lds[e] = t[q];
        }
    }
    __syncthreads();
    fft_tile<T, L, INV, TX, 1, TX, NTHR>(lds, twl, tid);
    for (int e = tid; e < n_out * TX; e += NTHR) {
        const int row = e / TX, col = e % TX;
        if (col0 + col < inner) base[int64_t(row) * inner + col] = lds[e];
    }
}

// ---------------------------------------------------------------- K3 ------
// (column tile, ky, slot) of a z-conv block.  A tile's rows are TX columns
// wide, so the tiles that share a 128-byte line would otherwise go to
// different XCDs (blocks are handed to the eight XCDs in turn) and each XCD
// would fetch the line from memory for itself.  Within every run of 8 G block
// ids (G tiles per line), the G blocks that one XCD receives one after the
// other take the G tiles of one line.  The ids past the last whole run keep
// the plain order.  On the 64^3 lattice (FP32, 8 right-hand sides, TX = 4)
// this cut the kernel's fetched bytes 2.5-fold and its time from 272 to 222 us.
// The launcher keeps the grid below 2^31 blocks, so the block id is done in
// 32-bit arithmetic (64-bit divisions of it cost some 500 scalar
// instructions per wave).
template <typename T, int TX>
__device__ __forceinline__ void zconv_block_map(int& tile, int& ky0, int& pos) {
    constexpr unsigned G = (128 / int(TX * sizeof(cx<T>))) > 1 ? 128 / int(TX * sizeof(cx<T>)) : 1;
    const unsigned nxt = gridDim.x, nky = gridDim.y;
    const unsigned per_slot = nxt * nky;
    unsigned id = blockIdx.x + nxt * (blockIdx.y + nky * blockIdx.z);
    constexpr unsigned run = 8 * G;
    if (nxt % G == 0 && id < (per_slot * gridDim.z / run) * run) {
        const unsigned q = id / run, r = id - q * run;
        id = q * run + (r & 7) * G + (r >> 3);
    }
    pos = int(id / per_slot);
    const unsigned rem = id - unsigned(pos) * per_slot;
    ky0 = int(rem / nxt);
    tile = int(rem - unsigned(ky0) * nxt);
}
// Per (kx tile, ky pair, slot): z-FFT of the three components (nz non-zero
// inputs), w = D u with D the symmetric 3x3 spectrum, z-iFFT, keep nz rows.
// A block takes the pencils of ky and of its mirror my - ky, and every D
// value it loads from the stored corner serves the four frequencies
// (+-kx fixed by the column, ky or my - ky, kz or mz - kz) that share it,
// with the sign flips of the odd components: four times fewer D loads.
template <typename T, int L, int TX>
__global__ __launch_bounds__(NTHR) void k_zconv(cx<T>* __restrict__ G,
                                                const cx<T>* const* __restrict__ Dptr,
                                                const cx<T>* __restrict__ tw, Geo g,
                                                const int* __restrict__ act,
                                                const int* __restrict__ slot_sys, SlotFilter f) {
    constexpr int W = 6 * TX;  // lines per tile: (mirror set, component, column)
    __shared__ cx<T> lds[L * W];
    // FP32: twiddles in LDS, which the FFT stages index per lane (190 against
    // 217 us on the 64^3 lattice); FP64 measured slower with them (534 against 524)
    constexpr bool TWL = sizeof(T) == 4;
    __shared__ cx<T> twl[TWL ? L : 1];
    const int tid = threadIdx.x;
    int tile, ky0, pos;
    zconv_block_map<T, TX>(tile, ky0, pos);
    const int col0 = tile * TX;
    const int ky1 = (g.my - ky0) % g.my;        // its mirror; 0 <= ky0 <= my/2
    const bool pair = ky1 != ky0;
    const int slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int sys = slot_sys[slot];
    const int64_t plane = int64_t(g.my) * g.mx;
    cx<T>* gb = G + int64_t(pos) * 3 * g.nz * plane + col0;
    cx<T>* gset[2] = {gb + int64_t(ky0) * g.mx, gb + int64_t(ky1) * g.mx};
    // each thread keeps one line (set, component, column) and walks z: the
    // index arithmetic is done once, and consecutive threads still read
    // consecutive columns
    static_assert(W <= NTHR, "a block must cover every line");
    constexpr int ZT = NTHR / W;  // threads per line
    const int lrem = tid % W, z0 = tid / W;
    const int lset = lrem / (3 * TX), lc = (lrem / TX) % 3, lcol = lrem % TX;
    const bool lok = tid < ZT * W && col0 + lcol < g.mx && (lset == 0 || pair);
    if (TWL)
        for (int t = tid; t < L; t += NTHR) twl[t] = tw[t];
    const cx<T>* twp = TWL ? twl : tw;
    if (tid < ZT * W) {
        // the z < nz <= (L+1)/2 loads of the line are all issued first (clamped
        // addresses), then stored; the rest of the line is zero
        constexpr int NZ = ((L + 1) / 2 + ZT - 1) / ZT;
        const cx<T>* src = gset[lset] + int64_t(lc) * g.nz * plane + min(lcol, g.mx - 1 - col0);
        cx<T> tv[NZ];
#pragma unroll
        for (int k = 0; k < NZ; ++k) tv[k] = src[int64_t(min(z0 + k * ZT, g.nz - 1)) * plane];
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            const int z = z0 + k * ZT;
            if (z < L) lds[z * W + lrem] = (lok && z < g.nz) ? tv[k] : cx<T>{T(0), T(0)};
        }
        for (int z = z0 + NZ * ZT; z < L; z += ZT) lds[z * W + lrem] = cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_tile<T, L, false, W, 1, W, NTHR>(lds, twp, tid);
    // D from its stored corner [0, M/2]^3: index M - k reads k, odd
    // components flip sign (xy: x and y, xz: x and z, yz: y and z)
    const int mxh = g.mx / 2 + 1, myh = g.my / 2 + 1, mzh = g.mz / 2 + 1;
    const int64_t dcomp = int64_t(mzh) * myh * mxh;
    const cx<T>* dbase = Dptr[sys] + int64_t(ky0) * mxh;
    for (int e = tid; e < mzh * TX; e += NTHR) {
        const int kzp = e / TX, col = e % TX;
        const int kx = col0 + col;
        if (kx >= g.mx) continue;
        const bool fx = kx > g.mx / 2;
        const int kxr = fx ? g.mx - kx : kx;
        const cx<T>* dp = dbase + int64_t(kzp) * myh * mxh + kxr;
        const cx<T> dxx = dp[0], dxy0 = dp[dcomp], dxz0 = dp[2 * dcomp];
        const cx<T> dyy = dp[3 * dcomp], dyz0 = dp[4 * dcomp], dzz = dp[5 * dcomp];
        const int kz1 = (g.mz - kzp) % g.mz;
        const int nz_ = (kz1 != kzp) ? 2 : 1;
        const int nset = pair ? 2 : 1;
        for (int zi = 0; zi < nz_; ++zi) {
            const int kz = zi ? kz1 : kzp;
            const bool fz = zi != 0;
            for (int set = 0; set < nset; ++set) {
                const bool fy = set != 0;
                const cx<T> dxy = (fx != fy) ? -dxy0 : dxy0;
                const cx<T> dxz = (fx != fz) ? -dxz0 : dxz0;
                const cx<T> dyz = (fy != fz) ? -dyz0 : dyz0;
                cx<T>* u = lds + kz * W + set * 3 * TX + col;
                const cx<T> ux = u[0], uy = u[TX], uz = u[2 * TX];
                u[0] = dxx * ux + dxy * uy + dxz * uz;
                u[TX] = dxy * ux + dyy * uy + dyz * uz;
                u[2 * TX] = dxz * ux + dyz * uy + dzz * uz;
            }
        }
    }
    __syncthreads();
    fft_tile<T, L, true, W, 1, W, NTHR>(lds, twp, tid);
    if (lok) {
        cx<T>* dst = gset[lset] + int64_t(lc) * g.nz * plane + lcol;
        if constexpr (sizeof(T) == 4) {
            // FP32: the line's LDS reads before its stores (182 against 191 us on
            // 64^3); FP64 measured slower with it (569 against 457)
            constexpr int NZ = ((L + 1) / 2 + ZT - 1) / ZT;  // z < nz <= (L+1)/2
            cx<T> tv[NZ];
#pragma unroll
            for (int k = 0; k < NZ; ++k) tv[k] = lds[min(z0 + k * ZT, L - 1) * W + lrem];
#pragma unroll
            for (int k = 0; k < NZ; ++k) {
                const int z = z0 + k * ZT;
                if (z < g.nz) dst[int64_t(z) * plane] = tv[k];
            }
        } else {
            for (int z = z0; z < g.nz; z += ZT) dst[int64_t(z) * plane] = lds[z * W + lrem];
        }
    }
}

// ------------------------------------------------------- K3 (two-stage) ----
// The same column pass with each z transform done as two register stages,
// L = R1 * R2 (Stockham: first R1-point DFTs of the inputs z = j + m R2, then
// after the twiddle W_L^{m j} R2-point DFTs that read and write the same
// indices j + m R1).  The first stage reads its inputs straight from global
// memory (only z < nz <= L/2, so half its inputs are the known zero padding)
// and the last inverse stage writes z < nz straight back; LDS carries one
// transpose per direction and the D product (the spectrum of the block's
// lines as [kz][line]), with five barriers per block.  Lines are
// (mirror set, component, column), consecutive lanes taking consecutive
// columns, so every global access is a run of TX columns.
template <int L>
constexpr int zc2_r1() {
    return L == 48 ? 8 : L == 64 ? 8 : L == 96 ? 16 : L == 128 ? 16 : L == 192 ? 16
         : L == 256 ? 16 : 0;
}
template <int L>
constexpr bool zc2_ok() { return zc2_r1<L>() > 0; }
template <typename T, int L, int TX>
constexpr size_t zc2_lds_bytes() { return size_t(L) * (6 * TX) * sizeof(cx<T>) + L * sizeof(cx<T>); }

template <typename T, int L, int TX, int NT, int R1>
__global__ __launch_bounds__(NT) void k_zconv2(cx<T>* __restrict__ G,
                                               const cx<T>* const* __restrict__ Dptr,
                                               const cx<T>* __restrict__ tw, Geo g,
                                               const int* __restrict__ act,
                                               const int* __restrict__ slot_sys, SlotFilter f) {
    constexpr int R2 = L / R1;
    constexpr int W = 6 * TX;  // lines: (mirror set, component, column)
    static_assert(R1 % 2 == 0, "the first radix must be even");
    __shared__ cx<T> lds[L * W];
    __shared__ cx<T> twl[L];
    const int tid = threadIdx.x;
    int tile, ky0, pos;
    zconv_block_map<T, TX>(tile, ky0, pos);
    const int col0 = tile * TX;
    const int ky1 = (g.my - ky0) % g.my;
    const bool pair = ky1 != ky0;
    const int slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    const int sys = slot_sys[slot];
    for (int t = tid; t < L; t += NT) twl[t] = tw[t];
    const int64_t plane = int64_t(g.my) * g.mx;
    cx<T>* gb = G + int64_t(pos) * 3 * g.nz * plane + col0;
    const int nz = g.nz;
    const cx<T> zero{T(0), T(0)};
    auto line_ptr = [&](int line, bool& ok) {
        const int lset = line / (3 * TX), lc = (line / TX) % 3, lcol = line % TX;
        ok = col0 + lcol < g.mx && (lset == 0 || pair);
        return gb + int64_t(lset ? ky1 : ky0) * g.mx + int64_t(lc) * nz * plane +
               min(lcol, g.mx - 1 - col0);
    };
    // forward stage 1: R1-point DFTs of x[j + m R2] (m < R1/2 can be non-zero)
    constexpr int NB1 = W * R2;
    for (int b = tid; b < NB1; b += NT) {
        const int line = b % W, j = b / W;
        bool ok;
        const cx<T>* src = line_ptr(line, ok);
        cx<T> a[R1];
#pragma unroll
        for (int m = 0; m < R1 / 2; ++m) {
            const int z = j + m * R2;
            a[m] = gload(src + int64_t(min(z, nz - 1)) * plane);
        }
#pragma unroll
        for (int m = 0; m < R1 / 2; ++m) {
            const int z = j + m * R2;
            if (!ok || z >= nz) a[m] = zero;
        }
#pragma unroll
        for (int m = R1 / 2; m < R1; ++m) a[m] = zero;
        reg_dft<T, R1, 1, false, L / R1>(a, tw);
#pragma unroll
        for (int m = 0; m < R1; ++m) lds[(j * R1 + m) * W + line] = a[m];
    }
    __syncthreads();
    // forward stage 2: twiddle W_L^{m j}, R2-point DFTs in place (each thread
    // reads and writes only the indices j + m R1 of its line)
    constexpr int NB2 = W * R1;
    for (int b = tid; b < NB2; b += NT) {
        const int line = b % W, j = b / W;
        cx<T> a[R2];
#pragma unroll
        for (int m = 0; m < R2; ++m) a[m] = lds[(j + m * R1) * W + line];
#pragma unroll
        for (int m = 1; m < R2; ++m) a[m] = a[m] * twl[m * j];
        reg_dft<T, R2, 1, false, L / R2>(a, twl);
#pragma unroll
        for (int m = 0; m < R2; ++m) lds[(j + m * R1) * W + line] = a[m];
    }
    // D from its stored corner [0, M/2]^3 (index M - k reads k; the odd
    // components flip sign), one load for the four frequencies
    // (ky0 or ky1) x (kz' or L - kz') of a column.  With sx the x parity,
    // the xy entry flips with the y mirror, xz with the z mirror and yz with
    // either; the four products are written out so that the signs fold into
    // the multiply-adds.  A thread's D loads go out before the barrier (its
    // stage-2 registers are free by then), so their latency overlaps the
    // wait for the other waves.
    {
        constexpr int MZH = L / 2 + 1;
        constexpr int ND = (MZH * TX + NT - 1) / NT;
        const int mxh = g.mx / 2 + 1, myh = g.my / 2 + 1;
        const int dplane = myh * mxh;  // a corner component holds < 2^31 entries
        const int dcomp = MZH * dplane;
        const cx<T>* dbase = Dptr[sys] + ky0 * mxh;
        const int wbase = tid & ~63;
        cx<T> dv[ND][6];
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            if (wbase + q * NT < MZH * TX) {  // wave-uniform
                const int e = min(tid + q * NT, MZH * TX - 1);
                const int kzp = e / TX, col = e - (e / TX) * TX;
                const int kx = min(col0 + col, g.mx - 1);
                const cx<T>* dp = dbase + kzp * dplane + (kx > g.mx / 2 ? g.mx - kx : kx);
#pragma unroll
                for (int c = 0; c < 6; ++c) dv[q][c] = gload(dp + c * dcomp);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            const int e = tid + q * NT;
            if (e >= MZH * TX) continue;
            const int kzp = e / TX, col = e - (e / TX) * TX;
            const int kx = col0 + col;
            if (kx >= g.mx) continue;
            const bool fx = kx > g.mx / 2;
            const cx<T> dxx = dv[q][0], dxy = dv[q][1], dxz = dv[q][2];
            const cx<T> dyy = dv[q][3], dyz = dv[q][4], dzz = dv[q][5];
            const T sx = fx ? T(-1) : T(1);
            const cx<T> axy = sx * dxy, axz = sx * dxz;
            cx<T>* u = lds + kzp * W + col;  // kz', set 0 (ky0)
            dmul3<T, TX>(u, dxx, axy, axz, dyy, dyz, dzz);
            if (pair) dmul3<T, TX>(u + 3 * TX, dxx, -axy, axz, dyy, -dyz, dzz);
            if (kzp != 0 && kzp != L / 2) {  // the mirror L - kz'
                cx<T>* v = lds + (L - kzp) * W + col;
                dmul3<T, TX>(v, dxx, axy, -axz, dyy, -dyz, dzz);
                if (pair) dmul3<T, TX>(v + 3 * TX, dxx, -axy, -axz, dyy, dyz, dzz);
            }
        }
    }
    __syncthreads();
    // inverse stage 1: R1-point DFTs of X[j + m R2] -> [j R1 + m]; every read
    // of the block before any write
    constexpr int NQ1 = (NB1 + NT - 1) / NT;
    {
        cx<T> a[NQ1][R1];
#pragma unroll
        for (int q = 0; q < NQ1; ++q) {
            const int b = tid + q * NT;
            if (b < NB1) {
                const int line = b % W, j = b / W;
#pragma unroll
                for (int m = 0; m < R1; ++m) a[q][m] = lds[(j + m * R2) * W + line];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ1; ++q) {
            const int b = tid + q * NT;
            if (b < NB1) {
                const int line = b % W, j = b / W;
                reg_dft<T, R1, 1, true, L / R1>(a[q], twl);
#pragma unroll
                for (int m = 0; m < R1; ++m) lds[(j * R1 + m) * W + line] = a[q][m];
            }
        }
    }
    __syncthreads();
    // inverse stage 2: twiddle, R2-point DFTs; z = j + m R1 < nz back to memory
    for (int b = tid; b < NB2; b += NT) {
        const int line = b % W, j = b / W;
        bool ok;
        cx<T>* dst = const_cast<cx<T>*>(line_ptr(line, ok));
        cx<T> a[R2];
#pragma unroll
        for (int m = 0; m < R2; ++m) a[m] = lds[(j + m * R1) * W + line];
#pragma unroll
        for (int m = 1; m < R2; ++m) {
            cx<T> t = twl[m * j];
            t.y = -t.y;
            a[m] = a[m] * t;
        }
        reg_dft<T, R2, 1, true, L / R2>(a, twl);
        if (ok) {
#pragma unroll
            for (int m = 0; m < R2; ++m) {
                const int z = j + m * R1;
                if ((2 * m < R2 || (R2 & 1)) && z < nz) dst[int64_t(z) * plane] = a[m];
            }
        }
    }
}

// ---------------------------------------------------------------- K5 ------
template <typename T, int L, int MODE>
__global__ __launch_bounds__(NTHR) void k_ixfft_pack(const cx<T>* __restrict__ G,
                                                     const cx<T>* __restrict__ xin,
                                                     const cx<T>* __restrict__ ainv,
                                                     cx<T>* __restrict__ yout,
                                                     const int* __restrict__ map,
                                                     const cx<T>* __restrict__ tw, Geo g,
                                                     const int* __restrict__ act,
                                                     const int* __restrict__ slot_sys,
                                                     SlotFilter f, RedScratch red,
                                                     const cx<T>* __restrict__ wv) {
    constexpr int NL = rows_nl<T, L>();
    constexpr int RP = padded_len<L>();  // row pitch (one spare slot per 16 elements)
    __shared__ cx<T> lds[NL * RP];
    __shared__ cx<T> twl[L];
    const int tid = threadIdx.x;
    const int c = blockIdx.y;
    const int pos = blockIdx.z;
    const int64_t slot = act ? act[pos] : pos;
    if (!slot_live(f, slot)) return;
    map += slot * g.map_stride;
    for (int t = tid; t < L; t += NTHR) twl[t] = tw[t];
    const int64_t sys = slot_sys[slot];
    const int nrows = g.nz * g.ny;
    const int row0 = blockIdx.x * NL;
    const cx<T>* gsrc = G + (int64_t(pos) * 3 + c) * g.nz * g.my * int64_t(g.mx);
    // the index loads go out with the grid loads and return during the x-iFFT
    // (the vector loads that depend on them wait until after it: issued here
    // they would hold registers through it)
    const int64_t voff = (slot * 3 + c) * g.n_occ;
    constexpr int HX = (L + 1) / 2;  // x < (L+1)/2 holds every occupied cell
    constexpr int NE = (NL * HX + NTHR - 1) / NTHR;
    int idx[NE];
    row_indices<NE, NTHR, HX>(map + int64_t(row0) * g.nx, min(NL, nrows - row0), g.nx, tid, idx);
    cx<T> xv[NE], av[NE], wq[MODE == PACK_AX_DOTW ? NE : 1];
    {
        constexpr int NLD = (NL * L + NTHR - 1) / NTHR;
        cx<T> t[NLD];
#pragma unroll
        for (int q = 0; q < NLD; ++q) {  // all loads first (clamped rows)
            const int e = tid + q * NTHR;
            const int row = min(row0 + min(e / L, NL - 1), nrows - 1);
            const int z = row / g.ny, y = row - z * g.ny;
            t[q] = gsrc[(int64_t(z) * g.my + y) * g.mx + (e % L)];
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * NTHR;
            if (e < NL * L)
                lds[(e / L) * RP + line_pos<true>(e % L)] =
                    (row0 + e / L < nrows) ? t[q] : cx<T>{T(0), T(0)};
        }
    }
    __syncthreads();
    fft_tile<T, L, true, NL, RP, 1, NTHR, true>(lds, twl, tid);
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
        const int e = tid + q * NTHR;
        const int rr = e / HX, x = e - (e / HX) * HX;
        const cx<T> conv = lds[rr * RP + line_pos<true>(x)];
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
    pack_rows<MODE, NTHR>(mu, red, int(slot), blockIdx.y * gridDim.x + blockIdx.x);
}

// ------------------------------------------------------------ launchers ---
static inline unsigned nblk(int64_t n, int64_t per) { return unsigned((n + per - 1) / per); }

int xfft_blocks_per_slot(const Geo& g, int csize) {
    if (yz_fused_ok(g, csize)) return yz_pack_blocks_per_slot(g, csize);  // same grid as k_xfft_t
    return pack_blocks_per_slot(g, csize);  // k_unpack_xfft has the grid of k_ixfft_pack
}

int pack_blocks_per_slot(const Geo& g, int csize) {
    const int64_t nrows = int64_t(g.nz) * g.ny;
    const int r = row_elems(csize);
    const int nl = g.mx >= r ? 1 : r / g.mx;  // rows_nl<T, mx>()
    return int(3 * ((nrows + nl - 1) / nl));
}

template <typename T>
void launch_unpack_xfft(cx<T>* xin, const int* map, cx<T>* G, const cx<T>* tw_x, const Geo& g,
                        const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f,
                        hipStream_t s, CocgFold fo, BicgFold bf) {
    if (n_act == 0) return;
    const int64_t nrows = int64_t(g.nz) * g.ny;
    switch (g.mx) {
#define DDA_CASE(N)                                                                    \
    case N: {                                                                          \
        dim3 grid(nblk(nrows, rows_nl<T, N>()), 3, n_act);                             \
        if (fuse_r && bf.kind == BICG_FOLD_S)                                          \
            k_unpack_xfft<T, N, FUSE_BICG_S><<<grid, NTHR, 0, s>>>(                    \
                xin, map, G, tw_x, g, act, fuse_r, f, CocgFold{}, bf);                 \
        else if (fuse_r && bf.kind == BICG_FOLD_P)                                     \
            k_unpack_xfft<T, N, FUSE_BICG_P><<<grid, NTHR, 0, s>>>(                    \
                xin, map, G, tw_x, g, act, fuse_r, f, CocgFold{}, bf);                 \
        else if (fuse_r)                                                               \
            k_unpack_xfft<T, N, FUSE_COCG><<<grid, NTHR, 0, s>>>(                      \
                xin, map, G, tw_x, g, act, fuse_r, f, fo, BicgFold{});                 \
        else                                                                           \
            k_unpack_xfft<T, N, FUSE_NONE><<<grid, NTHR, 0, s>>>(                      \
                xin, map, G, tw_x, g, act, nullptr, f, CocgFold{}, BicgFold{});        \
        break;                                                                         \
    }
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    DDA_LAUNCH_CHECK();
}

template <typename T, int L, bool INV, int TX>
void run_fft_mid(cx<T>* data, const cx<T>* tw, int64_t n_outer, int64_t inner, int n_in, int n_out,
                 int64_t outer_stride, hipStream_t s) {
    const int64_t tiles = (inner + TX - 1) / TX;
    k_fft_mid<T, L, INV, TX><<<unsigned(tiles * n_outer), NTHR, 0, s>>>(data, tw, inner, n_in,
                                                                       n_out, outer_stride, tiles);
}

template <typename T, int L, bool INV>
void fft_mid_tx(int tx, cx<T>* data, const cx<T>* tw, int64_t n_outer, int64_t inner, int n_in,
                int n_out, int64_t outer_stride, hipStream_t s) {
    if constexpr (L >= kTuneMinL) {
#define DDA_TX(W)                                                                          \
    if constexpr (mid_fits<T, L, W>())                                                     \
        if (tx == W)                                                                       \
            return run_fft_mid<T, L, INV, W>(data, tw, n_outer, inner, n_in, n_out,        \
                                             outer_stride, s);
        DDA_TX(4) DDA_TX(8) DDA_TX(16) DDA_TX(32)
#undef DDA_TX
    }
    run_fft_mid<T, L, INV, mid_tx<T, L>()>(data, tw, n_outer, inner, n_in, n_out, outer_stride, s);
}

template <typename T>
void launch_fft_mid(cx<T>* data, const cx<T>* tw, int L, bool inverse, int64_t n_outer,
                    int64_t inner, int n_in, int n_out, int64_t outer_stride, int tx,
                    hipStream_t s) {
    switch (L) {
#define DDA_CASE(N)                                                                        \
    case N:                                                                                \
        if (inverse)                                                                       \
            fft_mid_tx<T, N, true>(tx, data, tw, n_outer, inner, n_in, n_out, outer_stride, s); \
        else                                                                               \
            fft_mid_tx<T, N, false>(tx, data, tw, n_outer, inner, n_in, n_out, outer_stride, s); \
        break;
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length");
    }
    DDA_LAUNCH_CHECK();
}

template <typename T, int L, int TX>
void run_zconv(cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
               const int* act, const int* slot_sys, int n_act, SlotFilter f, hipStream_t s) {
    dim3 grid(nblk(g.mx, TX), g.my / 2 + 1, n_act);
    if (int64_t(grid.x) * grid.y * grid.z >= (int64_t(1) << 31))
        throw Error(-1, "z pass: grid of 2^31 blocks or more");
    k_zconv<T, L, TX><<<grid, NTHR, 0, s>>>(G, Dptr, tw_z, g, act, slot_sys, f);
}

// Tile codes of the two-stage z pass: TX columns per block and NT threads,
// code = TX | (NT / 64) << 6.  Candidates keep the block's LDS within 100 KB;
// 512 threads only where every thread has a second-stage butterfly.  All codes
// of one radix plan give the same result bit for bit (they only regroup lines);
// the two plans of a length round differently.
// The radix plan is a tuning dimension too: ALT takes R1 = 8 (R2 = L/8 in the
// second stage) where the default first radix is 16 and L/8 <= 24; code bit 12.
constexpr int zc2_code(int tx, int nt, int alt = 0) { return tx | ((nt / 64) << 6) | (alt << 12); }
template <int L, int ALT>
constexpr int zc2_r1_of() { return ALT ? 8 : zc2_r1<L>(); }
template <typename T, int L, int TX, int NT, int ALT = 0>
constexpr bool zc2_fits() {
    return zc2_ok<L>() && zc2_lds_bytes<T, L, TX>() <= (size_t(100) << 10) &&
           (NT <= 256 || 6 * TX * zc2_r1_of<L, ALT>() >= NT) &&
           (!ALT || (zc2_r1<L>() == 16 && L / 8 <= 24));
}
template <typename T, int L>
constexpr int zc2_default() {
    return sizeof(T) == 4 ? (zc2_fits<T, L, 8, 256>() ? zc2_code(8, 256) : zc2_code(4, 256))
                          : (zc2_fits<T, L, 4, 256>() ? zc2_code(4, 256) : zc2_code(2, 256));
}
#define DDA_ZC2_TILES(X)                                                                   \
    X(4, 256, 0) X(4, 512, 0) X(8, 256, 0) X(8, 512, 0) X(16, 256, 0) X(16, 512, 0)       \
    X(2, 256, 0) X(4, 256, 1) X(8, 256, 1) X(8, 512, 1)

template <typename T, int L, int TX, int NT, int ALT>
void run_zconv2(cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
                const int* act, const int* slot_sys, int n_act, SlotFilter f, hipStream_t s) {
    dim3 grid(nblk(g.mx, TX), g.my / 2 + 1, n_act);
    if (int64_t(grid.x) * grid.y * grid.z >= (int64_t(1) << 31))
        throw Error(-1, "z pass: grid of 2^31 blocks or more");
    k_zconv2<T, L, TX, NT, zc2_r1_of<L, ALT>()><<<grid, NT, 0, s>>>(G, Dptr, tw_z, g, act,
                                                                    slot_sys, f);
}

template <typename T, int L>
void zconv_tx_run(int tx, cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
                  const int* act, const int* slot_sys, int n_act, SlotFilter f, hipStream_t s) {
    if constexpr (zc2_ok<L>()) {
        const int code = tx ? tx : zc2_default<T, L>();
#define DDA_TX(W, N, A)                                                                   \
    if constexpr (zc2_fits<T, L, W, N, A>())                                              \
        if (code == zc2_code(W, N, A))                                                    \
            return run_zconv2<T, L, W, N, A>(G, Dptr, tw_z, g, act, slot_sys, n_act, f, s);
        DDA_ZC2_TILES(DDA_TX)
#undef DDA_TX
        throw Error(-1, "z pass: not a tile of this length");
    } else {
        if constexpr (L >= kTuneMinL) {
#define DDA_TX(W)                                                                        \
    if constexpr (zconv_fits<T, L, W>())                                                 \
        if (tx == W) return run_zconv<T, L, W>(G, Dptr, tw_z, g, act, slot_sys, n_act, f, s);
            DDA_TX(1) DDA_TX(2) DDA_TX(4) DDA_TX(8)
#undef DDA_TX
        }
        run_zconv<T, L, zconv_tx<T, L>()>(G, Dptr, tw_z, g, act, slot_sys, n_act, f, s);
    }
}

template <typename T>
void launch_zconv(cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
                  const int* act, const int* slot_sys, int n_act, SlotFilter f, int tx,
                  hipStream_t s) {
    if (n_act == 0) return;
    switch (g.mz) {
#define DDA_CASE(N)                                                                    \
    case N:                                                                            \
        zconv_tx_run<T, N>(tx, G, Dptr, tw_z, g, act, slot_sys, n_act, f, s);           \
        break;
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along z");
    }
    DDA_LAUNCH_CHECK();
}

template <typename T>
std::vector<int> mid_tx_candidates(int L) {
    std::vector<int> v;
    switch (L) {
#define DDA_CASE(N)                                                                    \
    case N:                                                                            \
        if (N >= kTuneMinL) {                                                          \
            if (mid_fits<T, N, 4>()) v.push_back(4);                                   \
            if (mid_fits<T, N, 8>()) v.push_back(8);                                   \
            if (mid_fits<T, N, 16>()) v.push_back(16);                                 \
            if (mid_fits<T, N, 32>()) v.push_back(32);                                 \
        }                                                                              \
        if (v.empty()) v.push_back(mid_tx<T, N>());                                    \
        break;
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        default:
            break;
    }
    return v;
}

template <typename T>
std::vector<int> zconv_tx_candidates(int L) {
    std::vector<int> v;
    switch (L) {
#define DDA_ZC2C(W, N, A) \
    if constexpr (zc2_fits<T, LL, W, N, A>()) v.push_back(zc2_code(W, N, A));
#define DDA_CASE(N)                                                                    \
    case N: {                                                                          \
        constexpr int LL = N;                                                          \
        if constexpr (zc2_ok<LL>()) {                                                  \
            DDA_ZC2_TILES(DDA_ZC2C)                                                    \
        } else if (N >= kTuneMinL) {                                                   \
            if (zconv_fits<T, N, 1>()) v.push_back(1);                                 \
            if (zconv_fits<T, N, 2>()) v.push_back(2);                                 \
            if (zconv_fits<T, N, 4>()) v.push_back(4);                                 \
            if (zconv_fits<T, N, 8>()) v.push_back(8);                                 \
        }                                                                              \
        if (v.empty()) v.push_back(zconv_tx<T, N>());                                  \
        break;                                                                         \
    }
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
#undef DDA_ZC2C
        default:
            break;
    }
    return v;
}

template <typename T>
void launch_ixfft_pack(const cx<T>* G, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                       const int* map, const cx<T>* tw_x, const Geo& g, const int* act,
                       const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                       hipStream_t s, const cx<T>* wv) {
    if (n_act == 0) return;
    if (pack_fused(mode) && pack_blocks_per_slot(g, int(sizeof(cx<T>))) > red.max_blocks)
        throw Error(-3, "reduction scratch too small for the fused pack kernel");
    if (mode == PACK_AX_DOTW && !wv) throw Error(-1, "PACK_AX_DOTW needs the vector w");
    const int64_t nrows = int64_t(g.nz) * g.ny;
    switch (g.mx) {
#define DDA_IXP(N, M)                                                                      \
    k_ixfft_pack<T, N, M><<<grid, NTHR, 0, s>>>(G, xin, ainv, yout, map, tw_x, g, act,        \
                                                slot_sys, f, red, wv)
#define DDA_CASE(N)                                                                        \
    case N: {                                                                              \
        dim3 grid(nblk(nrows, rows_nl<T, N>()), 3, n_act);                                 \
        switch (mode) {                                                                    \
            case PACK_GX: DDA_IXP(N, PACK_GX); break;                                      \
            case PACK_AX: DDA_IXP(N, PACK_AX); break;                                      \
            case PACK_AX_COCG: DDA_IXP(N, PACK_AX_COCG); break;                            \
            case PACK_AX_DOTW: DDA_IXP(N, PACK_AX_DOTW); break;                            \
            case PACK_AX_TS: DDA_IXP(N, PACK_AX_TS); break;                                \
            default: throw Error(-1, "unknown pack mode");                                 \
        }                                                                                  \
        break;                                                                             \
    }
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
#undef DDA_IXP
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    DDA_LAUNCH_CHECK();
}

template void launch_unpack_xfft<double>(z128*, const int*, z128*, const z128*, const Geo&,
                                         const int*, int, const z128*, SlotFilter, hipStream_t,
                                         CocgFold, BicgFold);
template void launch_unpack_xfft<float>(z64*, const int*, z64*, const z64*, const Geo&, const int*,
                                        int, const z64*, SlotFilter, hipStream_t, CocgFold,
                                        BicgFold);
template void launch_fft_mid<double>(z128*, const z128*, int, bool, int64_t, int64_t, int, int,
                                     int64_t, int, hipStream_t);
template void launch_fft_mid<float>(z64*, const z64*, int, bool, int64_t, int64_t, int, int,
                                    int64_t, int, hipStream_t);
template void launch_zconv<double>(z128*, const z128* const*, const z128*, const Geo&, const int*,
                                   const int*, int, SlotFilter, int, hipStream_t);
template void launch_zconv<float>(z64*, const z64* const*, const z64*, const Geo&, const int*,
                                  const int*, int, SlotFilter, int, hipStream_t);
template std::vector<int> mid_tx_candidates<double>(int);
template std::vector<int> mid_tx_candidates<float>(int);
template std::vector<int> zconv_tx_candidates<double>(int);
template std::vector<int> zconv_tx_candidates<float>(int);
template void launch_ixfft_pack<double>(const z128*, const z128*, const z128*, z128*,
                                        const int*, const z128*, const Geo&, const int*,
                                        const int*, int, int, SlotFilter, RedScratch, hipStream_t,
                                        const z128*);
template void launch_ixfft_pack<float>(const z64*, const z64*, const z64*, z64*, const int*,
                                       const z64*, const Geo&, const int*, const int*, int, int,
                                       SlotFilter, RedScratch, hipStream_t, const z64*);

// ------------------------------------------------------------ D build -----
// G_tilde(R) = exp(ikR)/R^3 [(k^2R^2 + ikR - 1) I + (3 - 3ikR - k^2R^2) Rh Rh]
// at every point of the embedding grid: grid index m along an axis of n cells
// and size M stands for the offset m (m <= n-1) or m - M (m >= M - n + 1);
// the remaining indices, and the zero offset, hold 0.  Pre-scaled by
// 1/(mx my mz) so that the inverse FFTs of the matvec need no scaling.
__device__ __forceinline__ bool embed_offset(int m, int n, int M, int& off) {
    if (m <= n - 1) { off = m; return true; }
    if (m >= M - (n - 1)) { off = m - M; return true; }
    return false;
}

// The six components xx, xy, xz, yy, yz, zz of G_tilde(R), R != 0.
__device__ __forceinline__ void gtilde6(double rx, double ry, double rz, double k_re,
                                        double k_im, z128 (&v)[6]) {
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double r = sqrt(r2);
    const double hx = rx / r, hy = ry / r, hz = rz / r;
    // kr = k r (complex), e = exp(i k r) / r^3
    const z128 kr{k_re * r, k_im * r};
    double sn, cs;
    sincos(kr.x, &sn, &cs);
    const double mag = exp(-kr.y) / (r2 * r);
    const z128 e{mag * cs, mag * sn};
    const z128 kr2 = kr * kr;
    const z128 a = e * z128{kr2.x - 1.0 - kr.y, kr2.y + kr.x};          // k2r2 + ikr - 1
    const z128 b = e * z128{3.0 - kr2.x + 3.0 * kr.y, -3.0 * kr.x - kr2.y};  // 3 - 3ikr - k2r2
    const double h[3] = {hx, hy, hz};
    int q = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            z128 val = (h[i] * h[j]) * b;
            if (i == j) val = val + a;
            v[q++] = val;
        }
}

__global__ __launch_bounds__(NTHR) void k_gtens(z128* __restrict__ D, Geo g, double d,
                                                double k_re, double k_im, double scale) {
    const int64_t plane = int64_t(g.my) * g.mx;
    const int64_t total = plane * g.mz;
    for (int64_t t = blockIdx.x * int64_t(NTHR) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * NTHR) {
        const int mz = int(t / plane);
        const int64_t rem = t - mz * plane;
        const int my = int(rem / g.mx), mx = int(rem - int64_t(my) * g.mx);
        int ox, oy, oz;
        z128 v[6];
        for (int q = 0; q < 6; ++q) v[q] = z128{0.0, 0.0};
        if (embed_offset(mx, g.nx, g.mx, ox) && embed_offset(my, g.ny, g.my, oy) &&
            embed_offset(mz, g.nz, g.mz, oz) && (ox | oy | oz) != 0) {
            gtilde6(d * ox, d * oy, d * oz, k_re, k_im, v);
            for (int q = 0; q < 6; ++q) v[q] = scale * v[q];
        }
        for (int q = 0; q < 6; ++q) D[q * total + t] = v[q];
    }
}

// Near offsets of the integrated interaction: one block per offset averages
// G_tilde over the source cell with the tensor Gauss-Legendre rule (FP64,
// each thread a fixed share of the nodes, the block's sums added in a fixed
// order) and overwrites the point value at that offset.
__global__ __launch_bounds__(NTHR) void k_gtens_igt(z128* __restrict__ D, Geo g, double d,
                                                    double k_re, double k_im, double scale,
                                                    const int* __restrict__ off,
                                                    const double* __restrict__ rule) {
    constexpr int NG = kIgtNodes, NN = NG * NG * NG;
    __shared__ double sm[NTHR / 64][12];
    __shared__ double ru[2 * NG];
    const int tid = threadIdx.x;
    if (tid < 2 * NG) ru[tid] = rule[tid];
    __syncthreads();
    const int* o = off + 4 * blockIdx.x;
    const double rx = d * o[0], ry = d * o[1], rz = d * o[2];
    double acc[12];
    for (int q = 0; q < 12; ++q) acc[q] = 0.0;
    for (int p = tid; p < NN; p += NTHR) {
        const int a = p / (NG * NG), b = (p / NG) % NG, c = p % NG;
        const double w = 0.125 * ru[NG + a] * ru[NG + b] * ru[NG + c];
        z128 v[6];
        gtilde6(rx + 0.5 * d * ru[a], ry + 0.5 * d * ru[b], rz + 0.5 * d * ru[c], k_re, k_im, v);
        for (int q = 0; q < 6; ++q) {
            acc[2 * q] += w * v[q].x;
            acc[2 * q + 1] += w * v[q].y;
        }
    }
    for (int q = 0; q < 12; ++q) {
        double x = acc[q];
        for (int s = 32; s > 0; s >>= 1) x += __shfl_down(x, s, 64);
        acc[q] = x;
    }
    if ((tid & 63) == 0)
        for (int q = 0; q < 12; ++q) sm[tid >> 6][q] = acc[q];
    __syncthreads();
    if (tid < 6) {
        double re = 0.0, im = 0.0;
        for (int w = 0; w < NTHR / 64; ++w) {
            re += sm[w][2 * tid];
            im += sm[w][2 * tid + 1];
        }
        const int64_t total = int64_t(g.mx) * g.my * g.mz;
        D[tid * total + o[3]] = z128{scale * re, scale * im};
    }
}

void igt_host_tables(const Geo& g, std::vector<int>& off, std::vector<double>& rule) {
    constexpr int NG = kIgtNodes;
    rule.assign(2 * NG, 0.0);
    for (int i = 0; i < NG; ++i) {
        // Newton's method on P_NG from the Chebyshev-like first guess
        double x = std::cos(3.14159265358979323846 * (i + 0.75) / (NG + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= NG; ++n) {
                const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = NG * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        rule[i] = x;
        rule[NG + i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    off.clear();
    const int r = int(kIgtRadius);
    for (int oz = -r; oz <= r; ++oz)
        for (int oy = -r; oy <= r; ++oy)
            for (int ox = -r; ox <= r; ++ox) {
                const int q = ox * ox + oy * oy + oz * oz;
                if (q == 0 || q > int(kIgtRadius * kIgtRadius + 1e-9)) continue;
                if (std::abs(ox) > g.nx - 1 || std::abs(oy) > g.ny - 1 || std::abs(oz) > g.nz - 1)
                    continue;
                const int64_t ix = ox >= 0 ? ox : g.mx + ox, iy = oy >= 0 ? oy : g.my + oy;
                const int64_t iz = oz >= 0 ? oz : g.mz + oz;
                off.insert(off.end(), {ox, oy, oz, int((iz * g.my + iy) * g.mx + ix)});
            }
}

template <int L>
__global__ __launch_bounds__(NTHR) void k_fft_rows(z128* __restrict__ data,
                                                   const z128* __restrict__ tw, int64_t nrows) {
    constexpr int NL = rows_nl<double, L>();
    __shared__ z128 lds[NL * L];
    const int tid = threadIdx.x;
    const int64_t row0 = int64_t(blockIdx.x) * NL;
    for (int e = tid; e < NL * L; e += NTHR) {
        const int rr = e / L;
        lds[e] = (row0 + rr < nrows) ? data[row0 * L + e] : z128{0.0, 0.0};
    }
    __syncthreads();
    fft_tile<double, L, false, NL, L, 1, NTHR>(lds, tw, tid);
    for (int e = tid; e < NL * L; e += NTHR) {
        const int rr = e / L;
        if (row0 + rr < nrows) data[row0 * L + e] = lds[e];
    }
}

template <typename T>
__global__ __launch_bounds__(NTHR) void k_extract_corner(const z128* __restrict__ full,
                                                         cx<T>* __restrict__ red, Geo g) {
    const int mxh = g.mx / 2 + 1, myh = g.my / 2 + 1, mzh = g.mz / 2 + 1;
    const int64_t total = int64_t(6) * mzh * myh * mxh;
    for (int64_t t = blockIdx.x * int64_t(NTHR) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * NTHR) {
        int64_t r = t;
        const int kx = int(r % mxh); r /= mxh;
        const int ky = int(r % myh); r /= myh;
        const int kz = int(r % mzh);
        const int q = int(r / mzh);
        red[t] = cvt<T>(full[((int64_t(q) * g.mz + kz) * g.my + ky) * g.mx + kx]);
    }
}

template <typename T>
void launch_extract_corner(const z128* full, cx<T>* out, const Geo& g, hipStream_t s) {
    const int64_t nred = dred_elems(g);
    k_extract_corner<T><<<unsigned(std::min<int64_t>(nblk(nred, NTHR), 65536)), NTHR, 0, s>>>(
        full, out, g);
    DDA_LAUNCH_CHECK();
}
template void launch_extract_corner<double>(const z128*, z128*, const Geo&, hipStream_t);
template void launch_extract_corner<float>(const z128*, z64*, const Geo&, hipStream_t);

void launch_build_D(z128* D, const Geo& g, double d, double k_re, double k_im,
                    const z128* tw_x, const z128* tw_y, const z128* tw_z, hipStream_t s,
                    const IgtTable* igt) {
    const int64_t plane = int64_t(g.my) * g.mx;
    const int64_t total = plane * g.mz;
    const double scale = 1.0 / double(total);
    k_gtens<<<nblk(total, NTHR), NTHR, 0, s>>>(D, g, d, k_re, k_im, scale);
    DDA_LAUNCH_CHECK();
    if (igt && igt->n > 0) {
        k_gtens_igt<<<igt->n, NTHR, 0, s>>>(D, g, d, k_re, k_im, scale, igt->off, igt->rule);
        DDA_LAUNCH_CHECK();
    }
    const int64_t nrows = 6 * int64_t(g.mz) * g.my;
    switch (g.mx) {
#define DDA_CASE(N)                                                                \
    case N:                                                                        \
        k_fft_rows<N><<<nblk(nrows, rows_nl<double, N>()), NTHR, 0, s>>>(D, tw_x, nrows); \
        break;
        DDA_FOR_EACH_L(DDA_CASE)
#undef DDA_CASE
        default:
            throw Error(-1, "unsupported FFT length along x");
    }
    DDA_LAUNCH_CHECK();
    launch_fft_mid<double>(D, tw_y, g.my, false, 6 * int64_t(g.mz), g.mx, g.my, g.my, plane, 0, s);
    launch_fft_mid<double>(D, tw_z, g.mz, false, 6, plane, g.mz, g.mz, total, 0, s);
}

__global__ void k_z128_to_z64(const z128* __restrict__ in, z64* __restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = cvt<float>(in[i]);
}
__global__ void k_z64_to_z128(const z64* __restrict__ in, z128* __restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = cvt<double>(in[i]);
}

void launch_convert_z128_to_z64(const z128* in, z64* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const unsigned b = unsigned(std::min<int64_t>(nblk(n, NTHR), 65536));
    k_z128_to_z64<<<b, NTHR, 0, s>>>(in, out, n);
    DDA_LAUNCH_CHECK();
}
void launch_convert_z64_to_z128(const z64* in, z128* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const unsigned b = unsigned(std::min<int64_t>(nblk(n, NTHR), 65536));
    k_z64_to_z128<<<b, NTHR, 0, s>>>(in, out, n);
    DDA_LAUNCH_CHECK();
}

}  // namespace dda

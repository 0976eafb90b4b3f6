// Host-side launchers of the gfx950 kernels (implemented in the .hip files).
#pragma once

#include <vector>

#include "common.h"
#include "slots.h"

namespace dda {

// Lattice and FFT-grid geometry shared by the matvec kernels.
struct Geo {
    int nx, ny, nz;   // lattice cells per axis
    int mx, my, mz;   // FFT grid of the block-Toeplitz embedding (>= 2n - 1)
    int64_t n_occ;    // occupied cells (the per-slot vector length)
    // 0: one index map for every slot.  Otherwise slot s reads its own map at
    // map + s * map_stride (lattices of one box sharing an engine; a slot's
    // dipoles are a prefix of its n_occ entries, the rest stay zero).
    int64_t map_stride;
};

// Grid buffer per slot: [3][nz][my][mx] complex, rows y >= ny unused before the
// y-pass.
inline int64_t grid_elems(const Geo& g) { return int64_t(3) * g.nz * g.my * g.mx; }
// D per system, components xx xy xz yy yz zz.  Every component of the
// interaction is even or odd along each axis (xy odd in x and y, xz in x and
// z, yz in y and z, the diagonal ones even), and so is its transform over the
// circulant embedding: D(M - k) = +-D(k) per axis.  Only the corner
// k in [0, M/2] per axis is stored: [6][mz/2+1][my/2+1][mx/2+1].
inline int64_t dgrid_elems(const Geo& g) { return int64_t(6) * g.mz * g.my * g.mx; }
inline int64_t dred_elems(const Geo& g) {
    return int64_t(6) * (g.mz / 2 + 1) * (g.my / 2 + 1) * (g.mx / 2 + 1);
}

bool fft_length_supported(int L);

// Per-matvec kernel chain.  Input/output vectors are slot-indexed
// [slot][3][n_occ]; the grid buffer G is indexed by position in the active
// list: act[pos] = slot (act == NULL: pos = slot).  slot_sys[slot] is the
// system (energy) of a slot; D and 1/alpha are per system: Dptr[sys] points to
// [6][mz][my][mx], ainv + sys * n_occ to the dipoles' 1/alpha.
// With fuse_r != NULL the kernel first updates the input in place,
// x <- fuse_r + beta x with beta = f.st[slot].beta (the COCG direction update;
// x <- fuse_r when the slot's reset_p is set), and transforms the updated
// vector; with fo.nblk > 0 it first ends the previous COCG iteration itself
// (CocgFold: beta and the slot's status from that iteration's rows).  Every
// kernel of the chain skips the slots the filter rejects.
// With bf.kind set (BiCGStab) the kernel instead forms, for an iterating slot,
// s = fuse_r - alpha bf.v or p = fuse_r + beta (x - omega bf.v), writes it in
// place of x and transforms it (BicgFold).
enum FuseMode { FUSE_NONE = 0, FUSE_COCG = 1, FUSE_BICG_S = 2, FUSE_BICG_P = 3 };
template <typename T>
void launch_unpack_xfft(cx<T>* xin, const int* map, cx<T>* G, const cx<T>* tw_x, const Geo& g,
                        const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f,
                        hipStream_t s, CocgFold fo = CocgFold{}, BicgFold bf = BicgFold{});
// tx: columns per block (0: the default width; see mid_tx_candidates).
template <typename T>
void launch_fft_mid(cx<T>* data, const cx<T>* tw, int L, bool inverse, int64_t n_outer,
                    int64_t inner, int n_in, int n_out, int64_t outer_stride, int tx,
                    hipStream_t s);
// tx: columns per block (0: the default width; see zconv_tx_candidates).
template <typename T>
void launch_zconv(cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
                  const int* act, const int* slot_sys, int n_act, SlotFilter f, int tx,
                  hipStream_t s);
// Tile widths the autotuner may try for a transform length L; all of them
// give bit-identical results.
template <typename T>
std::vector<int> mid_tx_candidates(int L);
template <typename T>
std::vector<int> zconv_tx_candidates(int L);
// mode PACK_AX: y = x/alpha - G_off x; PACK_GX: y = G_off x; PACK_AX_COCG:
// y = A x and, fused, the partial rows of mu = x^T y per slot in `red`
// (pack_blocks_per_slot rows, which must not exceed max_blocks); the caller
// then runs cocg_update_xr, which reads them.  PACK_AX_DOTW: y = A x and the
// rows of <w, y> = sum conj(w) y at offset 0 (w given per slot like x);
// PACK_AX_TS: y = A x and the rows of <y, x> and ||y||^2 at offset 3 (the
// BiCGStab products <rhat, v> and <t, s>, ||t||^2).
enum PackMode { PACK_AX = 0, PACK_GX = 1, PACK_AX_COCG = 2, PACK_AX_DOTW = 3, PACK_AX_TS = 4 };
inline bool pack_fused(int mode) { return mode >= PACK_AX_COCG; }

// Compact-vector index of each element e = tid + q NTH (q < NE) of a block's
// rows: row r = e / HX, column x = e % HX, rows nx apart from mrow; -1 for
// r >= nrow, x >= nx or an empty cell.  Every load is issued before the first
// is used: the addresses are clamped into the rows, and the mask is applied
// afterwards in a loop of its own without a short-circuit test (next to the
// load, `a && b ? m : -1` let the compiler move each load into a branch that
// waited for it).
template <int NE, int NTH, int HX>
__device__ __forceinline__ void row_indices(const int* __restrict__ mrow, int nrow, int nx,
                                            int tid, int (&idx)[NE]) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + q * NTH;
        const int r = e / HX, x = e - (e / HX) * HX;
        idx[q] = mrow[min(r, nrow - 1) * nx + min(x, nx - 1)];
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + q * NTH;
        const int r = e / HX, x = e - (e / HX) * HX;
        idx[q] = ((r < nrow) & (x < nx)) ? idx[q] : -1;
    }
}

// a u + b v + c w of complex values as one chain of a product and five
// multiply-adds per part (the signs of negated operands fold into them).
template <typename T>
__device__ __forceinline__ cx<T> cdot3(cx<T> a, cx<T> u, cx<T> b, cx<T> v, cx<T> c, cx<T> w) {
    T re = a.x * u.x, im = a.x * u.y;
    re = fma(-a.y, u.y, re);
    im = fma(a.y, u.x, im);
    re = fma(b.x, v.x, re);
    im = fma(b.x, v.y, im);
    re = fma(-b.y, v.y, re);
    im = fma(b.y, v.x, im);
    re = fma(c.x, w.x, re);
    im = fma(c.x, w.y, im);
    re = fma(-c.y, w.y, re);
    im = fma(c.y, w.x, im);
    return cx<T>{re, im};
}
// u <- D u for the three components of one frequency (component stride CS)
// with the symmetric tensor D = [xx xy xz; xy yy yz; xz yz zz].
template <typename T, int CS>
__device__ __forceinline__ void dmul3(cx<T>* u, cx<T> dxx, cx<T> dxy, cx<T> dxz, cx<T> dyy,
                                      cx<T> dyz, cx<T> dzz) {
    const cx<T> ux = u[0], uy = u[CS], uz = u[2 * CS];
    u[0] = cdot3(dxx, ux, dxy, uy, dxz, uz);
    u[CS] = cdot3(dxy, ux, dyy, uy, dyz, uz);
    u[2 * CS] = cdot3(dxz, ux, dyz, uy, dzz, uz);
}

// Per-element products of the fused pack modes (x the input, y = A x, w the
// extra vector), accumulated in FP64.
template <typename T, int MODE>
__device__ __forceinline__ void pack_dots(double (&mu)[3], cx<T> x, cx<T> y, cx<T> w) {
    if constexpr (MODE == PACK_AX_COCG) {  // bilinear x^T y
        if constexpr (sizeof(T) == 8) {
            // the contraction written out, so that it does not depend on how
            // the compiler orders the expression in each kernel
            mu[0] += fma(x.x, y.x, -(x.y * y.y));
            mu[1] += fma(x.x, y.y, x.y * y.x);
        } else {
            mu[0] += double(x.x) * y.x - double(x.y) * y.y;
            mu[1] += double(x.x) * y.y + double(x.y) * y.x;
        }
    } else if constexpr (MODE == PACK_AX_DOTW) {  // conj(w) y
        const double wx = w.x, wy = w.y, yx = y.x, yy = y.y;
        mu[0] += wx * yx + wy * yy;
        mu[1] += wx * yy - wy * yx;
    } else if constexpr (MODE == PACK_AX_TS) {  // conj(y) x and |y|^2
        const double xx = x.x, xy = x.y, yx = y.x, yy = y.y;
        mu[0] += yx * xx + yy * xy;
        mu[1] += yx * xy - yy * xx;
        mu[2] += yx * yx + yy * yy;
    }
}
// Stores a pack block's partial row of the fused mode (every thread calls it).
template <int MODE, int NT>
__device__ __forceinline__ void pack_rows(double (&mu)[3], RedScratch red, int slot, int blk) {
    if constexpr (MODE == PACK_AX_COCG || MODE == PACK_AX_DOTW) {
        double m2[2] = {mu[0], mu[1]};
        block_partial<2, NT, 0>(m2, red, slot, blk);
    } else if constexpr (MODE == PACK_AX_TS) {
        block_partial<3, NT, 3>(mu, red, slot, blk);
    }
}
int pack_blocks_per_slot(const Geo& g, int csize);
template <typename T>
void launch_ixfft_pack(const cx<T>* G, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                       const int* map, const cx<T>* tw_x, const Geo& g, const int* act,
                       const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                       hipStream_t s, const cx<T>* wv = nullptr);

// Interaction spectrum: D = FFT3(G_tilde on the embedding grid) / (mx my mz),
// FP64 over the full grid (dgrid_elems), for one host wavenumber k.  The
// matvec reads one of two stored layouts, extracted from it:
//   corner [6][mz/2+1][my/2+1][mx/2+1]           (five-pass chain, dred_elems)
//   kx slabs [mx/2+1][6][L/2+1][L/2+1], L = my = mz (three-pass chain, dyz_elems)
// Integrated interaction (DDA_INT_IGT): near offsets o (|o| <= kIgtRadius,
// o != 0, inside the embedding) take the average of G_tilde over the source
// cell, d^-3 int_cube G_tilde(R + s) d^3 s, by a kIgtNodes-point
// Gauss-Legendre rule per axis; every other offset keeps the point value.
constexpr int kIgtNodes = 24;
constexpr double kIgtRadius = 3.0;
struct IgtTable {
    int n = 0;                     // near offsets
    const int* off = nullptr;      // device [n][4]: ox, oy, oz, linear index in the grid
    const double* rule = nullptr;  // device [2][kIgtNodes]: nodes on [-1, 1], weights
};
// Host tables for IgtTable: offsets [n][4] and the rule [2][kIgtNodes]
// (Legendre nodes by Newton's method on the three-term recurrence).
void igt_host_tables(const Geo& g, std::vector<int>& off, std::vector<double>& rule);
void launch_build_D(z128* full, const Geo& g, double d, double k_re, double k_im,
                    const z128* tw_x, const z128* tw_y, const z128* tw_z, hipStream_t s,
                    const IgtTable* igt = nullptr);
template <typename T>
void launch_extract_corner(const z128* full, cx<T>* out, const Geo& g, hipStream_t s);
template <typename T>
void launch_extract_yz(const z128* full, cx<T>* out, const Geo& g, hipStream_t s);
// Far-field amplitudes (farfield.hip).  p [e][t][3][n_occ], coord packed
// ix | iy << 10 | iz << 20 per dipole, dirs [n_dir][3], kd [e] = k d;
// amp [e][t][n_dir][3].  Then dP/dOmega [rhs][n_dir] = scale[rhs] |(I - nn) A|^2
// and pcl[rhs] = sum_q w_q dP/dOmega (either output may be NULL).
size_t ff_lds_bytes(int nx, int ny, int nz);
void launch_ff_amp(const z128* p, const int* coord, int64_t n_occ, int nx, int ny, int nz,
                   const double* dirs, int n_dir, const double* kd, int n_energy, int n_traj,
                   z128* amp, hipStream_t s);
void launch_ff_power(const z128* amp, const double* dirs, const double* w, int n_dir,
                     const double* scale, int64_t nrhs, double* dp, double* pcl, hipStream_t s);

int64_t dyz_elems(const Geo& g);

// Three-pass chain (matvec_yz.hip), used when the padded yz plane of the three
// components fits in LDS (my == mz, see yz_fused_ok).  The work buffer holds
// T[pos][kx][3][nz][ny] (at most grid_elems).
bool yz_fused_ok(const Geo& g, int csize);
// partial reduction rows per slot of the fused pack kernel (csize: 8 or 16)
int yz_pack_blocks_per_slot(const Geo& g, int csize);
template <typename T>
void launch_xfft_t(cx<T>* xin, const int* map, cx<T>* Tb, const cx<T>* tw_x, const Geo& g,
                   const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f, hipStream_t s,
                   CocgFold fo = CocgFold{}, BicgFold bf = BicgFold{});
// blocks per slot of the x kernel of the three-pass or the five-pass chain
// (the rows a folded s update writes; the fused xy chain has
// xy_pack_blocks_per_slot)
int xfft_blocks_per_slot(const Geo& g, int csize);
// nthreads: threads per block (0: the default; see yz_thread_candidates)
template <typename T>
void launch_yzconv(cx<T>* Tb, const cx<T>* const* Dptr, const cx<T>* tw_y, const cx<T>* tw_z,
                   const Geo& g, const int* act, const int* slot_sys, int n_act, SlotFilter f,
                   int nthreads, hipStream_t s);
std::vector<int> yz_thread_candidates(int L);
template <typename T>
void launch_ixfft_t(const cx<T>* Tb, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                    const int* map, const cx<T>* tw_x, const Geo& g, const int* act,
                    const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                    hipStream_t s, const cx<T>* wv = nullptr);
// Three-kernel chain (matvec_xy.hip) for the other lattices whose zero-padded
// xy plane of one component fits in LDS (FP32, mx == my in {96, 128}): the
// x and y passes of the five-pass chain fused on either side of its z pass.
// The work buffer holds G[pos][3][nz][my][mx] as in the five-pass chain;
// launch_xyfft takes the fused Krylov updates of launch_unpack_xfft.
bool xy_fused_ok(const Geo& g, int csize);
// blocks per slot of both kernels (one per (component, z) plane): the partial
// rows of the fused pack modes and of a folded s update
int xy_pack_blocks_per_slot(const Geo& g);
template <typename T>
void launch_xyfft(cx<T>* xin, const int* map, cx<T>* G, const cx<T>* tw, const Geo& g,
                  const int* act, int n_act, const cx<T>* fuse_r, SlotFilter f, hipStream_t s,
                  CocgFold fo = CocgFold{}, BicgFold bf = BicgFold{});
template <typename T>
void launch_ixyfft_pack(const cx<T>* G, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                        const int* map, const cx<T>* tw, const Geo& g, const int* act,
                        const int* slot_sys, int n_act, int mode, SlotFilter f, RedScratch red,
                        hipStream_t s, const cx<T>* wv = nullptr);
void launch_convert_z128_to_z64(const z128* in, z64* out, int64_t n, hipStream_t s);
void launch_convert_z64_to_z128(const z64* in, z128* out, int64_t n, hipStream_t s);

// Electron field (eq. 25), FP64.
struct EincSys {   // per energy
    double k0;            // omega/c, 1/nm
    double kt_re, kt_im;  // k_t = omega / (gamma_h v)
    double ig_re, ig_im;  // -i / gamma_h
};
void launch_einc(z128* einc, const int* occ_lin, const Geo& g, double d, double beta,
                 const EincSys* sys /*device [n_energy]*/, const double* r0 /*device [n_traj][3]*/,
                 int n_energy, int n_traj, hipStream_t s);

// Device staging of one electron-field call: the energies [n_energy] and the
// trajectory points [n_traj][3] as copied from the host, and the per-energy
// constants that launch_einc_prep derives from the energies.  The layout
// holds up to `cap_e` energies; every array starts on a 256-byte boundary.
struct EincStage {
    double* energy;
    EincSys* sys;
    double* r0;
};
constexpr size_t einc_round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t einc_stage_bytes(size_t cap_e, size_t n_traj) {
    return einc_round256(cap_e * sizeof(double)) + einc_round256(cap_e * sizeof(EincSys)) +
           n_traj * 3 * sizeof(double);
}
inline EincStage einc_stage_layout(void* base, size_t cap_e) {
    char* b = static_cast<char*>(base);
    const size_t o1 = einc_round256(cap_e * sizeof(double));
    const size_t o2 = o1 + einc_round256(cap_e * sizeof(EincSys));
    return EincStage{reinterpret_cast<double*>(b), reinterpret_cast<EincSys*>(b + o1),
                     reinterpret_cast<double*>(b + o2)};
}
// sys[e] = {k0, k0 * inv_bg, ig} with k0 = energy[e] / hbar_c, for e < n
// (inv_bg = 1/(beta gamma_h), ig = -i/gamma_h, both per call).
void launch_einc_prep(const double* energy, EincSys* sys, int n, double hbar_c, z128 inv_bg,
                      z128 ig, hipStream_t s);

// The library's own staging area for callers that cannot allocate: a
// file-scope device array of einc_stage_bytes(kEincNoallocMaxEnergies,
// kEincNoallocMaxTraj) bytes (288 KiB) on every GPU the library runs on.
constexpr int kEincNoallocMaxEnergies = 4096;
constexpr int kEincNoallocMaxTraj = 4096;
// Looks up the array's address on the current device (once per device;
// thread-safe).  Throws dda::Error when the runtime cannot resolve it.
void einc_scratch_init();
// The address found for `device` by einc_scratch_init, or nullptr.
void* einc_scratch(int device);

// Material terms (material.hip), FP64: for system s < ns and dipole i < n,
// from eps[s][i] (absolute permittivity), the host index sys[s].mh and the
// host wavenumber sys[s].k,
// 1/alpha into ainv128[o][i] (and rounded into ainv64) and the absorption
// weight into w[o][i], with o = out_row[s] (o = s when out_row is NULL); any
// output may be NULL.  err[s] becomes non-zero for a non-finite permittivity
// (1) or a zero or infinite polarizability (2); the caller clears err[0..ns).
struct MatSys {
    double k_re, k_im;    // m_h omega / c
    double mh_re, mh_im;  // host index (Im m_h == 0: radiative-reaction form of w)
};
struct MatParams {
    int kind;  // 0 LDR, 1 CM, 2 RR
    double d;
};
void launch_material(const z128* eps, const MatSys* sys, int64_t n, int ns, MatParams mp,
                     const int* out_row, z128* ainv128, z64* ainv64, double* w, int* err,
                     hipStream_t s);

// Debug/test helper: K0, K1 at n complex points (device arrays).
void launch_besselk01(const z128* z, z128* k0, z128* k1, int64_t n, hipStream_t s);

}  // namespace dda

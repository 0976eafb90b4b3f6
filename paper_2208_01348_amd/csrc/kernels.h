// Host-side launchers of the gfx950 kernels (implemented in the .hip files).
#pragma once

#include "common.h"

namespace dda {

// Lattice and FFT-grid geometry shared by the matvec kernels.
struct Geo {
    int nx, ny, nz;   // lattice cells per axis
    int mx, my, mz;   // FFT grid of the block-Toeplitz embedding (>= 2n - 1)
    int64_t n_occ;    // occupied cells
};

// Grid buffer per slot: [3][nz][my][mx] complex, rows y >= ny unused before the
// y-pass.  D per system: [6][mz][my][mx] complex, components xx xy xz yy yz zz.
inline int64_t grid_elems(const Geo& g) { return int64_t(3) * g.nz * g.my * g.mx; }
inline int64_t dgrid_elems(const Geo& g) { return int64_t(6) * g.mz * g.my * g.mx; }

bool fft_length_supported(int L);

// Per-matvec kernel chain.  Input/output vectors are slot-indexed
// [slot][3][n_occ]; the grid buffer G is indexed by position in the active
// list: act[pos] = slot (act == NULL: pos = slot).  slot_sys[slot] is the
// system (energy) of a slot; D and 1/alpha are per system: Dptr[sys] points to
// [6][mz][my][mx], ainv + sys * n_occ to the dipoles' 1/alpha.
template <typename T>
void launch_unpack_xfft(const cx<T>* xin, const int* map, cx<T>* G, const cx<T>* tw_x,
                        const Geo& g, const int* act, int n_act, hipStream_t s);
template <typename T>
void launch_fft_mid(cx<T>* data, const cx<T>* tw, int L, bool inverse, int64_t n_outer,
                    int64_t inner, int n_in, int n_out, int64_t outer_stride, hipStream_t s);
template <typename T>
void launch_zconv(cx<T>* G, const cx<T>* const* Dptr, const cx<T>* tw_z, const Geo& g,
                  const int* act, const int* slot_sys, int n_act, hipStream_t s);
template <typename T>
void launch_ixfft_pack(const cx<T>* G, const cx<T>* xin, const cx<T>* ainv, cx<T>* yout,
                       const int* map, const cx<T>* tw_x, const Geo& g, const int* act,
                       const int* slot_sys, int n_act, bool interaction_only, hipStream_t s);

// Interaction spectrum: D = FFT3(G_tilde on the embedding grid) / (mx my mz),
// FP64, for one host wavenumber k.
void launch_build_D(z128* D, const Geo& g, double d, double k_re, double k_im,
                    const z128* tw_x, const z128* tw_y, const z128* tw_z, hipStream_t s);
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

// Debug/test helper: K0, K1 at n complex points (device arrays).
void launch_besselk01(const z128* z, z128* k0, z128* k1, int64_t n, hipStream_t s);

}  // namespace dda

// Far-field amplitudes of the dipoles and CL resolved over directions, FP64.
//
// For a non-absorbing host (k = m_h k0 real) the field radiated by the
// dipoles in direction n is proportional to (I - n n) A(n) with
//     A(n) = sum_j p_j exp(-i k n . r_j),
// and since Im G(R) = (k^3 / 4 pi) * integral over the sphere of (I - n n)
// e^{i k n . R}, the quadratic form of P_CL (eq. 42) is the angular integral
// of (k^3 / 4 pi) |(I - n n) A(n)|^2: the CL signal per unit solid angle.
//
// For one energy the amplitudes of all trajectories are one complex product
// (directions x dipoles) . (dipoles x 3 n_traj), done here on the FP64
// matrix cores (v_mfma_f64_16x16x4f64).  The phase factor of a (direction,
// dipole) pair is the product of three one-dimensional factors along the
// lattice axes, tabulated in LDS per block and energy, so a phase costs two
// complex products instead of a sincos.
#include <algorithm>

#include "kernels.h"

namespace dda {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int FF_DIRS = 16;             // MFMA rows: directions per block
constexpr int FF_TILES = 4;             // MFMA column tiles of 16 per block
constexpr int FF_COLS = 16 * FF_TILES;  // columns (trajectory, component) per block
constexpr int FF_WAVES = 4;             // the dipole sum is split over the waves
constexpr int FF_NT = 64 * FF_WAVES;

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// grid: x = tiles of 16 directions, y = tiles of 64 columns of one energy,
// z = energy.  Columns of energy e are c = 3 t + component for trajectory t;
// p is [e][t][3][n_occ]; amp is [e][t][n_dir][3].  Dynamic LDS: the
// per-axis phase tables of the block's directions (then reused for the
// partial sums of the waves).
__global__ __launch_bounds__(FF_NT) void k_ff_amp(const z128* __restrict__ p,
                                                 const int* __restrict__ coord, int64_t n_occ,
                                                 int nx, int ny, int nz,
                                                 const double* __restrict__ dirs, int n_dir,
                                                 const double* __restrict__ kd, int ncols,
                                                 z128* __restrict__ amp) {
    extern __shared__ z128 ffs[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int dir0 = blockIdx.x * FF_DIRS;
    const int col0 = blockIdx.y * FF_COLS;
    const int e = blockIdx.z;
    const int S = nx + ny + nz;
    const double kde = kd[e];
    // phase tables: row q holds exp(-i k d n_a (i_a - (n_a - 1)/2)) along x, y, z
    for (int t = tid; t < FF_DIRS * S; t += FF_NT) {
        const int q = t / S, a = t - (t / S) * S;
        const int dq = min(dir0 + q, n_dir - 1);
        double nc, u;
        if (a < nx) {
            nc = dirs[3 * dq];
            u = a - 0.5 * (nx - 1);
        } else if (a < nx + ny) {
            nc = dirs[3 * dq + 1];
            u = (a - nx) - 0.5 * (ny - 1);
        } else {
            nc = dirs[3 * dq + 2];
            u = (a - nx - ny) - 0.5 * (nz - 1);
        }
        double s, c;
        sincos(-kde * nc * u, &s, &c);
        ffs[t] = z128{c, s};
    }
    __syncthreads();
    // A operand: lane holds row i = lane % 16 (direction), k = lane / 16
    // (dipole of the group of 4); B operand: k = lane / 16, column lane % 16
    const int i = lane & 15, kk = lane >> 4;
    const z128* tx = ffs + i * S;
    const z128* ty = tx + nx;
    const z128* tz = ty + ny;
    const int ntile = min(FF_TILES, (ncols - col0 + 15) / 16);
    const z128* pe = p + int64_t(e) * ncols * n_occ;
    v4d acc_re[FF_TILES], acc_im[FF_TILES];
#pragma unroll
    for (int t = 0; t < FF_TILES; ++t) {
        acc_re[t] = v4d{0.0, 0.0, 0.0, 0.0};
        acc_im[t] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t kb = int64_t(wave) * 4; kb < n_occ; kb += 4 * FF_WAVES) {
        const int64_t j = kb + kk;
        const bool ok = j < n_occ;
        const int pc = coord[ok ? j : 0];
        const z128 ph = tx[pc & 1023] * ty[(pc >> 10) & 1023] * tz[pc >> 20];
        const double are = ok ? ph.x : 0.0, aim = ok ? ph.y : 0.0;
#pragma unroll
        for (int t = 0; t < FF_TILES; ++t) {
            if (t < ntile) {  // uniform over the block
                const int col = col0 + t * 16 + i;
                z128 b{0.0, 0.0};
                if (ok && col < ncols) b = pe[int64_t(col) * n_occ + j];
                acc_re[t] = mfma(are, b.x, acc_re[t]);
                acc_re[t] = mfma(-aim, b.y, acc_re[t]);
                acc_im[t] = mfma(are, b.y, acc_im[t]);
                acc_im[t] = mfma(aim, b.x, acc_im[t]);
            }
        }
    }
    // partial sums of the waves, added in wave order (deterministic); the
    // 16 x 16 result of a tile sits as D[4 r + lane / 16][lane % 16] in
    // element r of the lane (the f64 16x16x4 output layout)
    double* red = reinterpret_cast<double*>(ffs);  // [wave][256][2]
    for (int t = 0; t < ntile; ++t) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 4 * r + (lane >> 4), cl = lane & 15;
            red[(wave * 256 + row * 16 + cl) * 2] = acc_re[t][r];
            red[(wave * 256 + row * 16 + cl) * 2 + 1] = acc_im[t][r];
        }
        __syncthreads();
        const int row = tid >> 4, cl = tid & 15;  // 256 threads: one entry each
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int w = 0; w < FF_WAVES; ++w) {
            sr += red[(w * 256 + tid) * 2];
            si += red[(w * 256 + tid) * 2 + 1];
        }
        const int dir = dir0 + row, col = col0 + t * 16 + cl;
        if (dir < n_dir && col < ncols) {
            const int traj = col / 3, comp = col - (col / 3) * 3;
            const int64_t rhs = int64_t(e) * (ncols / 3) + traj;
            amp[(rhs * n_dir + dir) * 3 + comp] = z128{sr, si};
        }
    }
}

// dP/dOmega per (right-hand side, direction) and its weighted sum per
// right-hand side (one block per right-hand side, fixed summation order).
__global__ __launch_bounds__(256) void k_ff_power(const z128* __restrict__ amp,
                                                  const double* __restrict__ dirs,
                                                  const double* __restrict__ w, int n_dir,
                                                  const double* __restrict__ scale,
                                                  double* __restrict__ dp, double* __restrict__ pcl) {
    __shared__ double sm[256];
    const int64_t rhs = blockIdx.x;
    const double sc = scale[rhs];
    double acc = 0.0;
    for (int q = threadIdx.x; q < n_dir; q += 256) {
        const z128* a = amp + (rhs * n_dir + q) * 3;
        const double nx = dirs[3 * q], ny = dirs[3 * q + 1], nz = dirs[3 * q + 2];
        const z128 na{nx * a[0].x + ny * a[1].x + nz * a[2].x,
                      nx * a[0].y + ny * a[1].y + nz * a[2].y};
        const double v = sc * (norm2(a[0]) + norm2(a[1]) + norm2(a[2]) - norm2(na));
        if (dp) dp[rhs * n_dir + q] = v;
        if (w) acc += w[q] * v;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && pcl) pcl[rhs] = sm[0];
}

}  // namespace

size_t ff_lds_bytes(int nx, int ny, int nz) {
    const size_t tables = size_t(FF_DIRS) * size_t(nx + ny + nz) * sizeof(z128);
    const size_t partial = size_t(FF_WAVES) * 256 * 2 * sizeof(double);
    return std::max(tables, partial);
}

void launch_ff_amp(const z128* p, const int* coord, int64_t n_occ, int nx, int ny, int nz,
                   const double* dirs, int n_dir, const double* kd, int n_energy, int n_traj,
                   z128* amp, hipStream_t s) {
    if (n_energy == 0 || n_traj == 0 || n_dir == 0) return;
    const int ncols = 3 * n_traj;
    dim3 grid((n_dir + FF_DIRS - 1) / FF_DIRS, (ncols + FF_COLS - 1) / FF_COLS, n_energy);
    const size_t lds = ff_lds_bytes(nx, ny, nz);
    if (lds > (size_t(64) << 10)) throw Error(-1, "lattice sides too long for the far-field tables");
    k_ff_amp<<<grid, FF_NT, lds, s>>>(p, coord, n_occ, nx, ny, nz, dirs, n_dir, kd, ncols, amp);
    DDA_LAUNCH_CHECK();
}

void launch_ff_power(const z128* amp, const double* dirs, const double* w, int n_dir,
                     const double* scale, int64_t nrhs, double* dp, double* pcl, hipStream_t s) {
    if (nrhs == 0 || n_dir == 0) return;
    k_ff_power<<<unsigned(nrhs), 256, 0, s>>>(amp, dirs, w, n_dir, scale, dp, pcl);
    DDA_LAUNCH_CHECK();
}

}  // namespace dda

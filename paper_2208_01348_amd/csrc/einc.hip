// Incident field of the fast electron at every dipole (eq. 25), FP64.
//
// e_hat = exp(i omega (z - z0)/v) ( (x-x0)/b K1(k_t b), (y-y0)/b K1(k_t b),
//                                   -(i/gamma_h) K0(k_t b) ),
// k_t = omega/(gamma_h v); gamma_h in the first quadrant (eq. 24) puts
// z = k_t b in the sector -pi/2 <= arg z <= 0 (the imaginary axis is the
// lossless Cherenkov case, where K0 oscillates instead of decaying).
//
// K0 and K1 at complex z are evaluated without a library:
//  * |z| <= 1.5: ascending series (DLMF 10.31.2 and 10.31.1),
//      K0 = -(ln(z/2) + gamma_E) I0(z) + sum_k H_k q^k/(k!)^2,
//      K1 = 1/z + ln(z/2) I1(z) - (z/4) sum_k (psi(k+1) + psi(k+2)) q^k/(k!(k+1)!),
//    q = z^2/4, H_k the harmonic numbers;
//  * |z| > 1.5: the Laplace-type integral (DLMF 10.32.8) with t = s^2,
//      K0 = exp(-z)/sqrt(2z)   int_R exp(-s^2) (1 + s^2/(2z))^(-1/2) ds,
//      K1 = 2 exp(-z)/sqrt(2z) int_R s^2 exp(-s^2) (1 + s^2/(2z))^(+1/2) ds,
//    by the trapezoidal rule with step 0.2 on |s| <= 6.4.  The integrands are
//    analytic in the strip |Im s| < sqrt(|z|) (the branch point is at
//    s^2 = -2z), so the rule converges geometrically; both functions share
//    the one square root per node.  Relative error < 1e-15 over
//    1e-4 <= |z| <= 60, -pi/2 <= arg z <= 0.
#include <mutex>

#include "kernels.h"

namespace dda {

namespace {

__device__ __forceinline__ z128 csqrt_right(z128 q) {
    // principal square root for Re q >= 0
    const double r = hypot(q.x, q.y);
    const double t = sqrt(0.5 * (r + q.x));
    return z128{t, q.y / (2.0 * t)};
}

__device__ __forceinline__ z128 crecip(z128 a) {
    const double s = 1.0 / (a.x * a.x + a.y * a.y);
    return z128{a.x * s, -a.y * s};
}

constexpr double EULER_GAMMA = 0.57721566490153286061;
constexpr double TRAP_H = 0.2;
constexpr int TRAP_N = 32;

}  // namespace

__device__ void besselk01(z128 z, z128& K0, z128& K1) {
    const double r = hypot(z.x, z.y);
    if (r <= 1.5) {
        const z128 q = 0.25 * (z * z);
        z128 t0{1.0, 0.0};  // q^k/(k!)^2
        z128 t1{1.0, 0.0};  // q^k/(k!(k+1)!)
        z128 I0 = t0, S0{0.0, 0.0}, I1s = t1;
        double H = 0.0;                    // H_k
        double psi = 1.0 - 2.0 * EULER_GAMMA;  // psi(k+1) + psi(k+2) at k = 0
        z128 S1 = psi * t1;
#pragma unroll 1
        for (int k = 1; k <= 18; ++k) {
            const double kd = double(k);
            t0 = (1.0 / (kd * kd)) * (t0 * q);
            t1 = (1.0 / (kd * (kd + 1.0))) * (t1 * q);
            H += 1.0 / kd;
            psi = 2.0 * (H - EULER_GAMMA) + 1.0 / (kd + 1.0);
            I0 = I0 + t0;
            S0 = S0 + H * t0;
            I1s = I1s + t1;
            S1 = S1 + psi * t1;
        }
        const z128 lg{log(0.5 * r), atan2(z.y, z.x)};  // ln(z/2)
        const z128 I1 = 0.5 * (z * I1s);
        K0 = S0 - (lg + z128{EULER_GAMMA, 0.0}) * I0;
        K1 = crecip(z) + lg * I1 - 0.25 * (z * S1);
        return;
    }
    if (z.x > 700.0) {  // exp(-z) underflows; both functions are below 1e-300
        K0 = z128{0.0, 0.0};
        K1 = z128{0.0, 0.0};
        return;
    }
    const z128 u = crecip(2.0 * z);  // 1/(2z)
    z128 a0{0.0, 0.0}, a1{0.0, 0.0};
    // node 0 (s = 0): weight h, f0 = 1, f1 = 0
    a0.x = 1.0;
#pragma unroll 4
    for (int j = 1; j <= TRAP_N; ++j) {
        const double s = TRAP_H * j;
        const double s2 = s * s;
        const double w = 2.0 * exp(-s2);
        const z128 qv{1.0 + s2 * u.x, s2 * u.y};
        const z128 sq = csqrt_right(qv);
        a0 = a0 + w * crecip(sq);
        a1 = a1 + (w * s2) * sq;
    }
    // prefactor exp(-z)/sqrt(2z)
    double sn, cs;
    sincos(z.y, &sn, &cs);
    const double m = exp(-z.x);
    const z128 ez{m * cs, -m * sn};
    const z128 pre = ez * crecip(csqrt_right(2.0 * z));
    K0 = TRAP_H * (pre * a0);
    K1 = (2.0 * TRAP_H) * (pre * a1);
}

__global__ __launch_bounds__(256) void k_einc(z128* __restrict__ einc,
                                              const int* __restrict__ occ_lin, Geo g, double d,
                                              double beta, const EincSys* __restrict__ sys,
                                              const double* __restrict__ r0, int n_traj,
                                              int64_t blocks_per_rhs) {
    const int64_t rhs = blockIdx.x / blocks_per_rhs;
    const int64_t i = (blockIdx.x - rhs * blocks_per_rhs) * 256 + threadIdx.x;
    if (i >= g.n_occ) return;
    const int e = int(rhs / n_traj);
    const int t = int(rhs - int64_t(e) * n_traj);
    const EincSys S = sys[e];
    const int lin = occ_lin[i];
    const int plane = g.nx * g.ny;
    const int iz = lin / plane;
    const int rem = lin - iz * plane;
    const int iy = rem / g.nx;
    const int ix = rem - iy * g.nx;
    const double px = d * (ix - 0.5 * g.nx + 0.5);
    const double py = d * (iy - 0.5 * g.ny + 0.5);
    const double pz = d * (iz - 0.5 * g.nz + 0.5);
    const double dx = px - r0[3 * t], dy = py - r0[3 * t + 1], dz = pz - r0[3 * t + 2];
    const double b = hypot(dx, dy);
    z128 K0, K1;
    besselk01(z128{S.kt_re * b, S.kt_im * b}, K0, K1);
    double sn, cs;
    sincos(S.k0 * dz / beta, &sn, &cs);
    const z128 ph{cs, sn};
    const z128 pk1 = ph * K1;
    const double ib = 1.0 / b;
    z128* out = einc + rhs * 3 * g.n_occ + i;
    out[0] = (dx * ib) * pk1;
    out[g.n_occ] = (dy * ib) * pk1;
    out[2 * g.n_occ] = ph * (z128{S.ig_re, S.ig_im} * K0);
}

void launch_einc(z128* einc, const int* occ_lin, const Geo& g, double d, double beta,
                 const EincSys* sys, const double* r0, int n_energy, int n_traj, hipStream_t s) {
    if (g.n_occ == 0 || n_energy == 0 || n_traj == 0) return;
    const int64_t bpr = (g.n_occ + 255) / 256;
    const int64_t nrhs = int64_t(n_energy) * n_traj;
    k_einc<<<dim3(unsigned(bpr * nrhs)), 256, 0, s>>>(einc, occ_lin, g, d, beta, sys, r0, n_traj,
                                                      bpr);
    DDA_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_einc_prep(const double* __restrict__ energy,
                                                   EincSys* __restrict__ sys, int n, double hbar_c,
                                                   z128 inv_bg, z128 ig) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const double k0 = energy[e] / hbar_c;
    sys[e] = EincSys{k0, k0 * inv_bg.x, k0 * inv_bg.y, ig.x, ig.y};
}

void launch_einc_prep(const double* energy, EincSys* sys, int n, double hbar_c, z128 inv_bg,
                      z128 ig, hipStream_t s) {
    if (n <= 0) return;
    k_einc_prep<<<unsigned((n + 255) / 256), 256, 0, s>>>(energy, sys, n, hbar_c, inv_bg, ig);
    DDA_LAUNCH_CHECK();
}

// Staging area of dda_einc_electron_noalloc.  In host code `scratch` names a
// host-side stand-in, not the device array: host code uses only the address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kEincScratchBytes =
    einc_stage_bytes(kEincNoallocMaxEnergies, kEincNoallocMaxTraj);
static __device__ __align__(256) unsigned char scratch[kEincScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void einc_scratch_init() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        throw Error(-3, "einc scratch: no current device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        throw Error(-3, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
}

void* einc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

__global__ void k_besselk01(const z128* __restrict__ z, z128* __restrict__ k0,
                            z128* __restrict__ k1, int64_t n) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) besselk01(z[i], k0[i], k1[i]);
}

void launch_besselk01(const z128* z, z128* k0, z128* k1, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_besselk01<<<unsigned((n + 255) / 256), 256, 0, s>>>(z, k0, k1, n);
    DDA_LAUNCH_CHECK();
}

}  // namespace dda

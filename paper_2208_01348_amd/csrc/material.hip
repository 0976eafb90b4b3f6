// Per-dipole material terms on the device, FP64: the inverse polarizability
// 1/alpha_i(E) that the matvec diagonal needs, and the absorption weight of
// the loss reduction, from the absolute permittivity of every dipole at every
// energy of a batch.
//
// Polarizabilities (relative index m^2 = eps / m_h^2, cell volume d^3):
//   CM:  alpha = 3 d^3/(4 pi) (m^2 - 1)/(m^2 + 2)
//   RR:  alpha_CM / (1 - (2/3) i k^3 alpha_CM)
//   LDR: alpha_CM / (1 + (alpha_CM/d^3) [(b1 + m^2 b2) (kd)^2 - (2/3) i (kd)^3])
//        (Draine & Goodman 1993 with S = 0 for propagation along z)
// with k = m_h omega/c the host wavenumber; m_h and k are per system.
// Absorption weight w_i, used as P_abs ~ sum_i w_i |p_i|^2 / |m_h|^4: eq. (18)
// with the cell field of eq. (7), E_i = 4 pi p_i / ((m^2 - 1) d^3), plus the
// change the polarizability prescription makes to the exciting field's work
// on the dipole and less the nominal self-radiated power,
//   w = 4 pi Im(m_h^2 m^2) / (|m^2 - 1|^2 d^3)
//       + Im(m_h^2 conj(1/alpha - 1/alpha_CM)) - Re(m_h^2) (2/3) Re(k)^3,
// one formula for every host (in a real host it is m_h^2 times Draine's
// discrete absorption -Im(1/alpha) - (2/3) k^3).
#include <algorithm>

#include "kernels.h"

namespace dda {

namespace {

__device__ __forceinline__ z128 cdiv(z128 a, z128 b) {
    // Smith's algorithm: no overflow for large |b|
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, den = b.x + b.y * r;
        return z128{(a.x + a.y * r) / den, (a.y - a.x * r) / den};
    }
    const double r = b.x / b.y, den = b.x * r + b.y;
    return z128{(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kB1 = -1.8915316, kB2 = 0.1648469;

__global__ __launch_bounds__(256) void k_material(const z128* __restrict__ eps,
                                                  const MatSys* __restrict__ sys, int64_t n,
                                                  int64_t total, MatParams mp,
                                                  const int* __restrict__ out_row,
                                                  z128* __restrict__ ainv128,
                                                  z64* __restrict__ ainv64,
                                                  double* __restrict__ w, int* __restrict__ err) {
    const double d3 = mp.d * mp.d * mp.d;
    for (int64_t t = blockIdx.x * int64_t(256) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * 256) {
        const int64_t s = t / n;
        const z128 mh{sys[s].mh_re, sys[s].mh_im};
        const z128 mh2 = mh * mh;
        const int64_t o = out_row ? int64_t(out_row[s]) * n + (t - s * n) : t;
        const z128 ep = eps[t];
        if (!isfinite(ep.x) || !isfinite(ep.y)) {
            err[s] = 1;  // non-finite permittivity
            continue;
        }
        const z128 m2 = cdiv(ep, mh2);
        const z128 one{1.0, 0.0};
        const z128 acm = (3.0 * d3 / (4.0 * kPi)) * cdiv(m2 - one, m2 + z128{2.0, 0.0});
        const z128 k{sys[s].k_re, sys[s].k_im};
        z128 a = acm;
        if (mp.kind == 2) {  // RR
            const z128 k3 = k * k * k;
            a = cdiv(acm, one - (2.0 / 3.0) * (z128{0.0, 1.0} * k3 * acm));
        } else if (mp.kind == 0) {  // LDR
            const z128 kd = mp.d * k;
            const z128 kd2 = kd * kd;
            const z128 corr = (z128{kB1, 0.0} + kB2 * m2) * kd2 -
                              (2.0 / 3.0) * (z128{0.0, 1.0} * kd2 * kd);
            a = cdiv(acm, one + (1.0 / d3) * (acm * corr));
        }
        const double an = a.x * a.x + a.y * a.y;
        if (!(an > 0.0) || !isfinite(an)) {
            err[s] = 2;  // zero or infinite polarizability
            continue;
        }
        const z128 ai = cdiv(one, a);
        if (ainv128) ainv128[o] = ai;
        if (ainv64) ainv64[o] = cvt<float>(ai);
        if (w) {
            const z128 dm = m2 - one;
            const double w18 = 4.0 * kPi * (mh2 * m2).y / ((dm.x * dm.x + dm.y * dm.y) * d3);
            const z128 aicm = (4.0 * kPi / (3.0 * d3)) * cdiv(m2 + z128{2.0, 0.0}, dm);
            const z128 dc{ai.x - aicm.x, aicm.y - ai.y};  // conj(1/alpha - 1/alpha_CM)
            const double kr = k.x;
            w[o] = w18 + (mh2 * dc).y - mh2.x * (2.0 / 3.0) * kr * kr * kr;
        }
    }
}

}  // namespace

void launch_material(const z128* eps, const MatSys* sys, int64_t n, int ns, MatParams mp,
                     const int* out_row, z128* ainv128, z64* ainv64, double* w, int* err,
                     hipStream_t s) {
    const int64_t total = n * ns;
    if (total == 0) return;
    const unsigned b = unsigned(std::min<int64_t>((total + 255) / 256, 8192));
    k_material<<<b, 256, 0, s>>>(eps, sys, n, total, mp, out_row, ainv128, ainv64, w, err);
    DDA_LAUNCH_CHECK();
}

}  // namespace dda

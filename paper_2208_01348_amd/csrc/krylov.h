// Krylov (BiCGStab) building blocks and FP64 loss reductions on gfx950.
#pragma once

#include "kernels.h"

namespace dda {

enum SlotStatus : int {
    SLOT_ACTIVE = 0,
    SLOT_CONVERGED = 1,
    SLOT_HALF = 2,       // ||s|| met the tolerance inside an iteration
    SLOT_BREAKDOWN = 3,  // rho, <rhat, v> or omega vanished
};

// Per right-hand-side scalars, resident on the device.
struct BicgSlot {
    z128 rho, rho_old, alpha, omega;
    z128 rv, ts;          // <rhat, v>, <t, s>
    double tt;            // <t, t>
    double bnorm2;        // ||b||^2
    double rnorm2;        // ||r||^2 (recursive, or true after a residual pass)
    double tol2;          // tol^2
    int status;
    int iters;
};

// Reduction scratch: per slot, up to `max_blocks` partial rows of up to 8
// doubles, and one arrival counter per slot (zero between kernels).
struct RedScratch {
    double* partial;      // [max_slots][max_blocks][8]
    unsigned* counters;   // [max_slots]
    int max_blocks;
};

// Vectors are [slot][nv] (nv = 3 n_occ); `act` lists the slots to process
// (n_act of them).  Each launcher is one kernel.
template <typename T>
void bicg_norm_b(const cx<T>* b, BicgSlot* st, const int* act, int n_act, int64_t nv,
                 double tol2, RedScratch red, hipStream_t s);
template <typename T>
void bicg_reset(const cx<T>* r, cx<T>* rhat, cx<T>* p, cx<T>* v, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s);
template <typename T>
void bicg_update_p(const cx<T>* r, cx<T>* p, const cx<T>* v, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, hipStream_t s);
template <typename T>
void bicg_alpha(const cx<T>* rhat, const cx<T>* v, BicgSlot* st, const int* act, int n_act,
                int64_t nv, RedScratch red, hipStream_t s);
template <typename T>
void bicg_update_s(const cx<T>* r, const cx<T>* v, cx<T>* sv, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, hipStream_t s);
template <typename T>
void bicg_omega(const cx<T>* t, const cx<T>* sv, BicgSlot* st, const int* act, int n_act,
                int64_t nv, RedScratch red, hipStream_t s);
template <typename T>
void bicg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* rhat, const cx<T>* p, const cx<T>* sv,
                    const cx<T>* t, BicgSlot* st, const int* act, int n_act, int64_t nv,
                    RedScratch red, hipStream_t s);
// r = b - y, rnorm2 = ||r||^2 (true residual after y = A x)
template <typename T>
void residual(const cx<T>* b, const cx<T>* y, cx<T>* r, BicgSlot* st, const int* act, int n_act,
              int64_t nv, RedScratch red, hipStream_t s);

// Mixed precision helpers: r32 = r64 / sqrt(rnorm2); x64 += sqrt(rnorm2) * d32.
void scale_down(const z128* r, z64* r32, const BicgSlot* st, const int* act, int n_act,
                int64_t nv, hipStream_t s);
void accumulate_up(z128* x, const z64* d32, const BicgSlot* st, const int* act, int n_act,
                   int64_t nv, hipStream_t s);

// FP64 sums for the loss probabilities, per slot (8 doubles each):
//   [0,1] sum g_i . p_i          (g: auxiliary field of eq. 34 from e_hat)
//   [2,3] sum conj(e_i) . p_i
//   [4]   sum w_i |p_i|^2        (w: per-dipole absorption weight)
//   [5,6] sum conj(p_i) . y_i    (y = G_off p)
//   [7]   sum |p_i|^2
// einc and p are indexed by global right-hand side (slot s is rhs0 + s);
// y, w and kv are chunk-local (system = slot / n_traj).
void loss_sums(const z128* einc, const z128* p, const z128* y, const double* w /*[sys][n_occ]*/,
               const int* occ_lin, const Geo& g, double d, const double* kv /*[sys] omega/v*/,
               const double* r0 /*[n_traj][3]*/, int n_traj, int64_t rhs0, int nslots,
               double* out /*[nslots][8]*/, RedScratch red, hipStream_t s);

}  // namespace dda

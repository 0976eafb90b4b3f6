// Krylov (BiCGStab) building blocks and FP64 loss reductions on gfx950.
#pragma once

#include "kernels.h"
#include "slots.h"

namespace dda {

// Vectors are [slot][nv] (nv = 3 n_occ); `act` lists the slots to process
// (n_act of them).  Each launcher is one kernel.
// bnorm2 = ||b||^2; also sets tol2, upd2, maxit and zeroes the counters
template <typename T>
void bicg_norm_b(const cx<T>* b, BicgSlot* st, const int* act, int n_act, int64_t nv,
                 double tol2, double upd2, int maxit, RedScratch red, hipStream_t s);
template <typename T>
void bicg_reset(const cx<T>* r, cx<T>* rhat, cx<T>* p, cx<T>* v, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s);
// One iteration: update_p, v = A p (pack mode PACK_AX_DOTW with w = rhat),
// update_s, t = A s (PACK_AX_TS), update_xr.  Each kernel takes the scalar
// it needs from the partial rows of the one before (nblk_mv: the matvec
// pack kernel's rows per slot); update_p with fin_prev closes the previous
// iteration, and bicg_finish closes the last one of a sequence (before the
// host reads the slot states).
template <typename T>
void bicg_update_p(const cx<T>* r, cx<T>* p, const cx<T>* v, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, bool fin_prev, hipStream_t s);
template <typename T>
void bicg_update_s(const cx<T>* r, const cx<T>* v, cx<T>* sv, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, int nblk_mv, hipStream_t s);
// nblk_s: rows of ||s||^2 (0: those of bicg_update_s; the folded s update
// writes one per block of its x kernel)
template <typename T>
void bicg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* rhat, const cx<T>* p, const cx<T>* sv,
                    const cx<T>* t, BicgSlot* st, const int* act, int n_act, int64_t nv,
                    RedScratch red, int nblk_mv, int nblk_s, hipStream_t s);
void bicg_finish(BicgSlot* st, const int* act, int n_act, int64_t nv, RedScratch red,
                 hipStream_t s);
// r = b - y, rnorm2 = ||r||^2 (true residual after y = A x)
template <typename T>
void residual(const cx<T>* b, const cx<T>* y, cx<T>* r, BicgSlot* st, const int* act, int n_act,
              int64_t nv, RedScratch red, hipStream_t s);

// COCG (conjugate-orthogonal CG for complex-symmetric A, bilinear products
// x^T y).  The matvec's pack kernel writes the partial rows of mu = p^T q.
// alpha = rho / mu from the partial rows the fused pack kernel wrote
// (nblk_mu rows per slot; mu == 0 or not finite: SLOT_BREAKDOWN), then
// x += alpha p; r -= alpha q and the rows of rho' = r^T r, ||r||^2; with
// finish, then rho' (into copy 0), beta = rho'/rho and the convergence,
// reliable-update, breakdown and iteration-limit flags (slots in SLOT_ACTIVE
// only).  Without finish that last step is left to the next direction update
// (CocgFold over cocg_rows(nv) rows).  par: parity of the iteration in its
// interval (its rho is copy par).
template <typename T>
void cocg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* p, const cx<T>* q, BicgSlot* st,
                    const int* act, int n_act, int64_t nv, RedScratch red, int nblk_mu,
                    int par, bool finish, hipStream_t s);
int cocg_rows(int64_t nv, int max_blocks);
// FP64 residual passes: r = b - y (FP64; y == NULL stands for 0), r_lo = r
// rounded to T, rho = r_lo^T r_lo, rnorm2 = rmax2 = ||r||^2.
//   cocg_start: every listed slot, from x0 = 0 (y = 0); p = r on the first
//     direction update; SLOT_DONE if b already meets the tolerance.
//   cocg_check: only slots with needs_check(); decides SLOT_DONE,
//     SLOT_FAIL_NOCONV, SLOT_FAIL_BREAKDOWN (after max_restarts restarts) or
//     a restart / reliable update that returns the slot to SLOT_ACTIVE.
template <typename T>
void cocg_start(const z128* b, const z128* y, cx<T>* r_lo, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s);
template <typename T>
void cocg_check(const z128* b, const z128* y, cx<T>* r_lo, BicgSlot* st, const int* act,
                int n_act, int64_t nv, int max_restarts, RedScratch red, hipStream_t s,
                bool always_reset = false);

// QMR for complex-symmetric A (Freund 1992), on the same driver as COCG:
// qmr_start begins a cycle (v_1 = r / ||r||, v_0 = p_{-1} = p_0 = 0 and the
// scalars of step 1) on the listed slots whose reset_p is set; qmr_step is
// one Lanczos step after the matvec u = A vc (pack mode PACK_AX_COCG: rows of
// vc^T u), with the roles of the vectors and of the two scalar copies given
// by the step's parity `par` in its interval (vc, vo: v_n and v_{n-1}; p1,
// p2: p_{n-1} and p_{n-2}; p_n is written over p2 and v_{n+1} over vo).
// x accumulates in T.  The slot status becomes SLOT_CONVERGED when
// sqrt(n+1) |tau| meets the tolerance (an FP64 check then decides),
// SLOT_BREAKDOWN or SLOT_MAXIT.
// A cycle ends when its residual bound falls to max(tol ||b||, inner ||r_0||).
template <typename T>
void qmr_start(const cx<T>* r, cx<T>* va, cx<T>* vb, cx<T>* p1, cx<T>* p2, BicgSlot* st,
               const int* act, int n_act, int64_t nv, double inner, hipStream_t s);
template <typename T>
void qmr_step(cx<T>* x, const cx<T>* u, cx<T>* vc, cx<T>* vo, cx<T>* p1, cx<T>* p2,
              BicgSlot* st, const int* act, int n_act, int64_t nv, RedScratch red, int nblk_mu,
              int par, hipStream_t s);
// x = 0 and x_lo = 0 (if not NULL) on the listed slots
void cocg_zero(z128* x, z64* x_lo, const int* act, int n_act, int64_t nv, hipStream_t s);
// slot act[i] becomes SLOT_FAIL_INVALID where err[i] != 0 (i < n)
void mark_invalid(BicgSlot* st, const int* act, const int* err, int n, hipStream_t s);
// x64 += x_lo; x_lo = 0 (slots the filter accepts)
void accumulate_lo(z128* x, z64* x_lo, const int* act, int n_act, int64_t nv, SlotFilter f,
                   hipStream_t s);

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

// Krylov solvers over many right-hand sides at once (BiCGStab, van der Vorst
// 1992; COCG, the conjugate-orthogonal CG for complex-symmetric matrices,
// van der Vorst & Melissen 1990), with every scalar resident on the device,
// and the FP64 loss reductions.
//
// One grid covers every active slot: blockIdx.y picks the slot from the
// active list, blockIdx.x a contiguous piece of its vector.  Each dot product
// is a work kernel that writes one partial row per block; the rows are summed
// in index order, by a finalize kernel (one block per slot) or by every block
// of the next kernel, which then updates the slot's scalars: deterministic,
// without atomics or fences.  The host never synchronises inside an
// iteration.
#include "krylov.h"

namespace dda {

namespace {

constexpr int NT = 256;
constexpr int EPB = 1024;  // vector elements per block

inline int blocks_for(int64_t nv, int max_blocks) {
    int64_t b = (nv + EPB - 1) / EPB;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return int(b);
}

// conj(a) * b accumulated in double
template <typename T>
__device__ __forceinline__ void acc_cdot(double& re, double& im, cx<T> a, cx<T> b) {
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    re += ax * bx + ay * by;
    im += ax * by - ay * bx;
}
// a * b (bilinear) accumulated in double
template <typename T>
__device__ __forceinline__ void acc_bdot(double& re, double& im, cx<T> a, cx<T> b) {
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    re += ax * bx - ay * by;
    im += ax * by + ay * bx;
}

#define SLOT_PROLOGUE                                                   \
    const int slot = act[blockIdx.y];                                   \
    const int64_t base = int64_t(slot) * nv;                            \
    const int64_t i0 = int64_t(blockIdx.x) * NT + threadIdx.x;          \
    const int64_t stride = int64_t(gridDim.x) * NT;

// Finalize kernels: one block per listed slot.
#define FIN_PROLOGUE(K)                                                 \
    const int slot = act[blockIdx.x];                                   \
    double tot[K];                                                      \
    sum_rows<K, NT>(red, slot, nblk, tot);                              \
    if (threadIdx.x != 0) return;                                       \
    BicgSlot& S = st[slot];

__device__ __forceinline__ bool all_finite(const double* t, int k) {
    for (int i = 0; i < k; ++i)
        if (!isfinite(t[i])) return false;
    return true;
}

// The slot status as one thread of the block read it, for every wave of the
// block.  Kernels whose block 0 may change the status while other blocks run
// take their decisions from this single read, so the waves of a block cannot
// disagree and reach different barriers.  Every thread must call it.
__device__ __forceinline__ int block_status(const BicgSlot& S) {
    __shared__ int sh;
    if (threadIdx.x == 0) sh = S.status;
    __syncthreads();
    return sh;
}

// ------------------------------------------------------------- ||b||^2 ----
template <typename T>
__global__ __launch_bounds__(NT) void k_norm_b(const cx<T>* __restrict__ b,
                                               const int* __restrict__ act, int64_t nv,
                                               RedScratch red) {
    SLOT_PROLOGUE
    double v[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) v[0] += double(norm2(b[base + i]));
    block_partial<1, NT>(v, red, slot, blockIdx.x);
}
__global__ __launch_bounds__(NT) void k_fin_norm_b(BicgSlot* st, const int* act, RedScratch red,
                                                   int nblk, double tol2, double upd2, int maxit) {
    FIN_PROLOGUE(1)
    S.bnorm2 = tot[0];
    S.tol2 = tol2;
    S.upd2 = upd2;
    S.iters = 0;
    S.want_update = 0;
    S.matvecs = 0;
    S.restarts = 0;
    S.reset_p = 0;
    S.maxit = maxit;
}

// ------------------------------------------------------------ BiCGStab ----
template <typename T>
__global__ __launch_bounds__(NT) void k_reset(const cx<T>* __restrict__ r, cx<T>* __restrict__ rhat,
                                              cx<T>* __restrict__ p, cx<T>* __restrict__ v,
                                              const int* __restrict__ act, int64_t nv,
                                              RedScratch red) {
    SLOT_PROLOGUE
    double s[1] = {0.0};
    const cx<T> zero{T(0), T(0)};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> ri = r[base + i];
        rhat[base + i] = ri;
        p[base + i] = zero;
        v[base + i] = zero;
        s[0] += double(norm2(ri));
    }
    block_partial<1, NT>(s, red, slot, blockIdx.x);
}
__global__ __launch_bounds__(NT) void k_fin_reset(BicgSlot* st, const int* act, RedScratch red,
                                                  int nblk) {
    FIN_PROLOGUE(1)
    S.rho = z128{tot[0], 0.0};
    S.rho_old = z128{1.0, 0.0};
    S.alpha = z128{1.0, 0.0};
    S.omega = z128{1.0, 0.0};
    S.rnorm2 = tot[0];
    S.status = (tot[0] <= S.tol2 * S.bnorm2) ? SLOT_CONVERGED : SLOT_ACTIVE;
}

// One BiCGStab iteration is three vector kernels around the two matvecs,
// whose pack kernels write the dot products of their output:
//   update_p  [FIN: sums the rows at 0..2 of the previous update_xr]
//   v = A p   (pack rows of <rhat, v> at 0..1)
//   update_s  (sums those rows -> alpha; writes ||s||^2 rows at 6)
//   t = A s   (pack rows of <t, s>, ||t||^2 at 3..5)
//   update_xr (sums row 6 -> the half-step test, rows 3..5 -> omega; writes
//              <rhat, r>, ||r||^2 rows at 0..2)
// and k_fin_xr closes the last iteration of an interval.  For small batches
// update_p and update_s are folded into the x kernels of the two matvecs
// (BicgFold), which sum the same rows in the same order.  A kernel that
// needs a scalar sums the rows itself in every block (the same fixed order,
// so every block gets the same value); block 0 stores it in the slot state.
// Rows read and rows written by one kernel never overlap, and no block reads
// a state field that another block of the same kernel writes, except the
// status: it is read once per block (block_status), and a block that sees
// the status another block just set takes the decision that block took.

// Sums K rows at OFF for `slot` and returns the totals in every thread.
template <int K, int OFF>
__device__ __forceinline__ void slot_totals(RedScratch red, int slot, int nblk, double (&v)[K]) {
    __shared__ double sh[K];
    double tot[K];
    sum_rows<K, NT, OFF>(red, slot, nblk, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) sh[k] = tot[k];
    __syncthreads();
    for (int k = 0; k < K; ++k) v[k] = sh[k];
}

template <typename T, bool FIN>
__global__ __launch_bounds__(NT) void k_update_p(const cx<T>* __restrict__ r, cx<T>* __restrict__ p,
                                                 const cx<T>* __restrict__ v, BicgSlot* st,
                                                 const int* __restrict__ act, int64_t nv,
                                                 RedScratch red, int nblk) {
    SLOT_PROLOGUE
    BicgSlot& S = st[slot];
    const int status = block_status(S);
    z128 rho;
    if constexpr (FIN) {
        if (status != SLOT_ACTIVE && status != SLOT_HALF) return;  // uniform per block
        double tot[3];
        slot_totals<3, 0>(red, slot, nblk, tot);
        const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
        if (finish_iteration(S, status, tot, lead) != SLOT_ACTIVE) return;
        rho = z128{tot[0], tot[1]};
    } else {
        if (status != SLOT_ACTIVE) return;
        rho = S.rho;
    }
    const z128 beta = zdiv(rho, S.rho_old) * zdiv(S.alpha, S.omega);
    const cx<T> bt{T(beta.x), T(beta.y)};
    const cx<T> om{T(S.omega.x), T(S.omega.y)};
    for (int64_t i = i0; i < nv; i += stride)
        p[base + i] = bicg_p_of(r[base + i], bt, p[base + i], om, v[base + i]);
}
static_assert(NT == kBicgUpdateThreads, "the folded p update sums like this kernel");

template <typename T>
__global__ __launch_bounds__(NT) void k_update_s(const cx<T>* __restrict__ r,
                                                 const cx<T>* __restrict__ v, cx<T>* __restrict__ sv,
                                                 BicgSlot* st, const int* __restrict__ act,
                                                 int64_t nv, RedScratch red, int nblk_mv) {
    SLOT_PROLOGUE
    BicgSlot& S = st[slot];
    if (block_status(S) != SLOT_ACTIVE) return;
    double rv[2];
    slot_totals<2, 0>(red, slot, nblk_mv, rv);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if ((rv[0] == 0.0 && rv[1] == 0.0) || !all_finite(rv, 2)) {
        if (lead) {
            S.rv = z128{rv[0], rv[1]};
            S.status = SLOT_BREAKDOWN;
        }
        return;
    }
    const z128 al = zdiv(S.rho, z128{rv[0], rv[1]});
    if (lead) {
        S.rv = z128{rv[0], rv[1]};
        S.alpha = al;
    }
    const cx<T> a{T(al.x), T(al.y)};
    double s[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> si = bicg_s_of(r[base + i], a, v[base + i]);
        sv[base + i] = si;
        s[0] += bicg_norm2(si);
    }
    block_partial<1, NT, 6>(s, red, slot, blockIdx.x);
}
static_assert(NT == kBicgUpdateThreads, "the folded s update sums like this kernel");

template <typename T>
__global__ __launch_bounds__(NT) void k_update_xr(cx<T>* __restrict__ x, cx<T>* __restrict__ r,
                                                  const cx<T>* __restrict__ rhat,
                                                  const cx<T>* __restrict__ p,
                                                  const cx<T>* __restrict__ sv,
                                                  const cx<T>* __restrict__ t, BicgSlot* st,
                                                  const int* __restrict__ act, int64_t nv,
                                                  RedScratch red, int nblk_mv, int nblk_s) {
    SLOT_PROLOGUE
    BicgSlot& S = st[slot];
    const int status = block_status(S);
    if (status != SLOT_ACTIVE && status != SLOT_HALF) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    z128 om{0.0, 0.0};
    if (status == SLOT_ACTIVE) {
        double ss[1];
        slot_totals<1, 6>(red, slot, nblk_s, ss);
        if (ss[0] <= S.tol2 * S.bnorm2) {  // ||s|| met the tolerance: x += alpha p ends the solve
            if (lead) {
                S.omega = om;
                S.status = SLOT_HALF;
            }
        } else {
            double ts[3];
            slot_totals<3, 3>(red, slot, nblk_mv, ts);
            if (ts[2] > 0.0) om = z128{ts[0] / ts[2], ts[1] / ts[2]};
            if (lead) {
                S.ts = z128{ts[0], ts[1]};
                S.tt = ts[2];
                S.omega = om;
            }
        }
    }
    if (lead) S.rho_old = S.rho;
    const z128 al = S.alpha;
    const cx<T> a{T(al.x), T(al.y)}, o{T(om.x), T(om.y)};
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> si = sv[base + i];
        x[base + i] = x[base + i] + a * p[base + i] + o * si;
        const cx<T> ri = si - o * t[base + i];
        r[base + i] = ri;
        acc_cdot(s[0], s[1], rhat[base + i], ri);
        s[2] += double(norm2(ri));
    }
    block_partial<3, NT, 0>(s, red, slot, blockIdx.x);
}
__global__ __launch_bounds__(NT) void k_fin_xr(BicgSlot* st, const int* act, RedScratch red,
                                               int nblk) {
    const int status = st[act[blockIdx.x]].status;
    if (status != SLOT_ACTIVE && status != SLOT_HALF) return;
    FIN_PROLOGUE(3)
    finish_iteration(S, status, tot, true);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_residual(const cx<T>* __restrict__ b,
                                                 const cx<T>* __restrict__ y, cx<T>* __restrict__ r,
                                                 const int* __restrict__ act, int64_t nv,
                                                 RedScratch red) {
    SLOT_PROLOGUE
    double s[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> ri = b[base + i] - y[base + i];
        r[base + i] = ri;
        s[0] += double(norm2(ri));
    }
    block_partial<1, NT>(s, red, slot, blockIdx.x);
}
__global__ __launch_bounds__(NT) void k_fin_residual(BicgSlot* st, const int* act, RedScratch red,
                                                     int nblk) {
    FIN_PROLOGUE(1)
    S.rnorm2 = tot[0];
}

__global__ __launch_bounds__(NT) void k_scale_down(const z128* __restrict__ r, z64* __restrict__ r32,
                                                   const BicgSlot* st, const int* __restrict__ act,
                                                   int64_t nv) {
    SLOT_PROLOGUE
    const double rn = st[slot].rnorm2;
    const double sc = rn > 0.0 ? 1.0 / sqrt(rn) : 0.0;
    for (int64_t i = i0; i < nv; i += stride) r32[base + i] = cvt<float>(sc * r[base + i]);
}

__global__ __launch_bounds__(NT) void k_accumulate_up(z128* __restrict__ x,
                                                      const z64* __restrict__ d32,
                                                      const BicgSlot* st,
                                                      const int* __restrict__ act, int64_t nv) {
    SLOT_PROLOGUE
    const double sc = sqrt(st[slot].rnorm2);
    for (int64_t i = i0; i < nv; i += stride)
        x[base + i] = x[base + i] + sc * cvt<double>(d32[base + i]);
}

// ---------------------------------------------------------------- COCG ----
// alpha = rho / mu from the pack kernel's partial rows (doubles 0, 1 of each
// row; every block sums them in the same fixed order, block 0 records the
// result or the breakdown, and counts the iteration), then x += alpha p,
// r -= alpha q and the partial rows of r^T r and ||r||^2 (doubles 4..6, so
// the mu rows stay intact while other blocks of the slot still read them).
// rho is copy `par` (the parity of the iteration in its interval).
template <typename T>
__global__ __launch_bounds__(NT) void k_cocg_xr(cx<T>* __restrict__ x, cx<T>* __restrict__ r,
                                                const cx<T>* __restrict__ p,
                                                const cx<T>* __restrict__ q, BicgSlot* st,
                                                const int* __restrict__ act, int64_t nv,
                                                RedScratch red, int nblk_mu, int par) {
    SLOT_PROLOGUE
    if (block_status(st[slot]) != SLOT_ACTIVE) return;
    __shared__ double mu_sh[2];
    {
        double mu[2];
        sum_rows<2, NT>(red, slot, nblk_mu, mu);
        if (threadIdx.x == 0) {
            mu_sh[0] = mu[0];
            mu_sh[1] = mu[1];
        }
    }
    __syncthreads();
    const z128 rv{mu_sh[0], mu_sh[1]};
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if ((rv.x == 0.0 && rv.y == 0.0) || !isfinite(rv.x) || !isfinite(rv.y)) {
        if (lead) {
            st[slot].rv = rv;
            st[slot].status = SLOT_BREAKDOWN;
        }
        return;
    }
    const z128 al = zdiv(par ? st[slot].rho1 : st[slot].rho, rv);
    if (lead) {
        st[slot].rv = rv;
        st[slot].alpha = al;
        // the iteration is counted here, and the direction reset (if any) is
        // spent: the next direction update may be folded into a kernel whose
        // blocks must all read the same values
        st[slot].iters += 1;
        st[slot].matvecs += 1;
        st[slot].reset_p = 0;
    }
    const cx<T> a{T(al.x), T(al.y)};
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        x[base + i] = x[base + i] + a * p[base + i];
        const cx<T> ri = r[base + i] - a * q[base + i];
        r[base + i] = ri;
        acc_bdot(s[0], s[1], ri, ri);
        s[2] += double(norm2(ri));
    }
    block_partial<3, NT, 4>(s, red, slot, blockIdx.x);
}
// The end of the last iteration of an interval (parity par), as a kernel of
// its own: rho goes to copy 0, where the next interval starts.  Inside an
// interval the same step is folded into the next direction update
// (cocg_fold), which sums the rows in this kernel's order.
static_assert(NT == kCocgFinThreads, "the folded finalizer sums like this kernel");
__global__ __launch_bounds__(NT) void k_fin_cocg_xr(BicgSlot* st, const int* act, RedScratch red,
                                                    int nblk, int par) {
    if (st[act[blockIdx.x]].status != SLOT_ACTIVE) return;
    const int slot = act[blockIdx.x];
    double tot[3];
    sum_rows<3, NT, 4>(red, slot, nblk, tot);
    if (threadIdx.x != 0) return;
    BicgSlot& S = st[slot];
    z128 beta;
    const int status = cocg_next(S, tot, par ? S.rho1 : S.rho, beta);
    cocg_record(S, tot, status, beta, 0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_true_residual(const z128* __restrict__ b,
                                                      const z128* __restrict__ y,
                                                      cx<T>* __restrict__ r_lo,
                                                      const int* __restrict__ act, int64_t nv,
                                                      SlotFilter f, RedScratch red) {
    SLOT_PROLOGUE
    if (!slot_live(f, slot)) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const z128 ri = y ? b[base + i] - y[base + i] : b[base + i];
        const cx<T> rl = cvt<T>(ri);
        r_lo[base + i] = rl;
        acc_bdot(s[0], s[1], rl, rl);
        s[2] += ri.x * ri.x + ri.y * ri.y;
    }
    block_partial<3, NT>(s, red, slot, blockIdx.x);
}
// Start of COCG from x0 = 0 (r = b): rho = r^T r, p = r on the first
// direction update, done at once if b meets the tolerance.
__global__ __launch_bounds__(NT) void k_fin_cocg_start(BicgSlot* st, const int* act,
                                                       RedScratch red, int nblk) {
    FIN_PROLOGUE(3)
    S.rho = z128{tot[0], tot[1]};
    S.beta = z128{0.0, 0.0};
    S.rnorm2 = tot[2];
    S.rmax2 = tot[2];
    S.want_update = 0;
    S.reset_p = 1;
    S.best2 = tot[2];
    S.stall = 0;
    S.status = (tot[2] <= S.tol2 * S.bnorm2) ? SLOT_DONE : SLOT_ACTIVE;
}

// Mixed precision: the recursion runs on the FP32 operator, and near a
// resonance (large condition number) its directions can lose conjugacy with
// respect to the FP64 one; the FP64 residual then stalls while the recursive
// one keeps falling.  A slot whose FP64 residual has not halved over
// kStallChecks checks restarts its recursion from the FP64 residual.
constexpr double kStallDrop = 0.5;
constexpr int kStallChecks = 8;

// FP64 residual check of a slot that asked for one (needs_check): the FP64
// residual decides convergence; otherwise the iteration limit ends the slot, a
// breakdown restarts the recursion from the true residual (p = r), and a
// reliable update continues it with the recomputed residual (p, beta kept).
__global__ __launch_bounds__(NT) void k_fin_check(BicgSlot* st, const int* act, RedScratch red,
                                                  int nblk, int max_restarts, int always_reset) {
    if (!needs_check(st[act[blockIdx.x]])) return;
    FIN_PROLOGUE(3)
    S.matvecs += 1;
    S.rnorm2 = tot[2];
    S.rmax2 = tot[2];
    S.want_update = 0;
    if (!all_finite(tot, 3)) {
        S.status = SLOT_FAIL_BREAKDOWN;
        return;
    }
    if (tot[2] <= S.tol2 * S.bnorm2) {
        S.status = SLOT_DONE;
        return;
    }
    if (S.status == SLOT_MAXIT || S.iters >= S.maxit) {
        S.status = SLOT_FAIL_NOCONV;
        return;
    }
    if (S.status == SLOT_BREAKDOWN) {
        if (S.restarts >= max_restarts) {
            S.status = SLOT_FAIL_BREAKDOWN;
            return;
        }
        S.restarts += 1;
        S.reset_p = 1;
        S.beta = z128{0.0, 0.0};
    } else if (S.upd2 > 0.0) {
        if (tot[2] < kStallDrop * S.best2) {
            S.best2 = tot[2];
            S.stall = 0;
        } else if (++S.stall >= kStallChecks) {
            S.stall = 0;
            S.best2 = tot[2];
            S.reset_p = 1;
            S.beta = z128{0.0, 0.0};
        }
    }
    S.rho = z128{tot[0], tot[1]};
    S.status = SLOT_ACTIVE;
    if (always_reset) S.reset_p = 1;  // QMR restarts its Lanczos process from the new residual
}

__global__ __launch_bounds__(NT) void k_cocg_zero(z128* __restrict__ x, z64* __restrict__ x_lo,
                                                  const int* __restrict__ act, int64_t nv) {
    SLOT_PROLOGUE
    for (int64_t i = i0; i < nv; i += stride) {
        x[base + i] = z128{0.0, 0.0};
        if (x_lo) x_lo[base + i] = z64{0.f, 0.f};
    }
}

// err[i] != 0 (per listed position) ends slot act[i] as invalid.
__global__ __launch_bounds__(NT) void k_mark_invalid(BicgSlot* st, const int* __restrict__ act,
                                                     const int* __restrict__ err, int n) {
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i < n && err[i] != 0) st[act[i]].status = SLOT_FAIL_INVALID;
}

__global__ __launch_bounds__(NT) void k_accumulate_lo(z128* __restrict__ x, z64* __restrict__ x_lo,
                                                      const int* __restrict__ act, int64_t nv,
                                                      SlotFilter f) {
    SLOT_PROLOGUE
    if (!slot_live(f, slot)) return;
    for (int64_t i = i0; i < nv; i += stride) {
        x[base + i] = x[base + i] + cvt<double>(x_lo[base + i]);
        x_lo[base + i] = z64{0.f, 0.f};
    }
}

// ----------------------------------------------------------------- QMR ----
// QMR for complex-symmetric matrices (Freund 1992): the Lanczos process of
// the bilinear form x^T y with vectors of unit 2-norm, and the quasi-minimal
// residual iterate from Givens rotations of its tridiagonal matrix H (column
// n: beta_n, alpha_n, rho_{n+1}).  Per step, around the matvec u = A v_n
// (whose pack kernel writes the partial rows of v_n^T u at 0..1):
//   k_qmr_lanczos  alpha_n = v_n^T u / delta_n, beta_n = rho_n delta_n /
//                  delta_{n-1}; w = u - alpha_n v_n - beta_n v_{n-1} (into
//                  the v_{n-1} buffer); rows of ||w||^2 at 4, w^T w at 5..6
//   k_qmr_update   rho_{n+1}, delta_{n+1}; the column through G_{n-2},
//                  G_{n-1} and the new rotation G_n; p_n = (v_n - d2 p_{n-1}
//                  - eps p_{n-2}) / r_n (into the p_{n-2} buffer); x += c_n
//                  tau_n p_n; v_{n+1} = w / rho_{n+1}; tau_{n+1} = -conj(s_n)
//                  tau_n; the scalars for step n+1 into the other copy
//   k_qmr_fin      the copy's flag becomes the slot status (converged when
//                  sqrt(n+1) |tau_{n+1}|, which bounds the residual, meets
//                  the cycle's threshold: the tolerance, or in FP32 a fixed
//                  fraction of the cycle's starting residual, since the
//                  FP32 recursion cannot resolve more; breakdown when delta
//                  or r_n vanishes)
// Both vector kernels take the step's scalars from the same sums in every
// block; only block 0 stores them.

constexpr int kQmrStagSteps = 256;

__device__ __forceinline__ z128 zmul(z128 a, z128 b) {
    return z128{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ z128 zconj(z128 a) { return z128{a.x, -a.y}; }

// alpha_n and beta_n of step `Q` from the mu rows; false on a breakdown
// (delta_n = 0, or a non-finite product), which every block detects alike.
__device__ __forceinline__ bool qmr_ab(const QmrScalars& Q, const double (&mu)[2], z128& a,
                                       z128& b) {
    if (!isfinite(mu[0]) || !isfinite(mu[1])) return false;
    if (Q.delta.x == 0.0 && Q.delta.y == 0.0) return false;
    a = zdiv(z128{mu[0], mu[1]}, Q.delta);
    b = Q.n > 1 ? Q.rho * zdiv(Q.delta, Q.delta_prev) : z128{0.0, 0.0};
    return isfinite(a.x) && isfinite(a.y) && isfinite(b.x) && isfinite(b.y);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_qmr_lanczos(const cx<T>* __restrict__ vc,
                                                    cx<T>* __restrict__ vo,
                                                    const cx<T>* __restrict__ u, BicgSlot* st,
                                                    const int* __restrict__ act, int64_t nv,
                                                    RedScratch red, int nblk_mu, int par) {
    SLOT_PROLOGUE
    BicgSlot& S = st[slot];
    if (block_status(S) != SLOT_ACTIVE) return;
    double mu[2];
    slot_totals<2, 0>(red, slot, nblk_mu, mu);
    z128 a, b;
    if (!qmr_ab(S.qmr[par], mu, a, b)) return;  // k_qmr_update flags it
    const cx<T> at{T(a.x), T(a.y)}, bt{T(b.x), T(b.y)};
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> w = u[base + i] - at * vc[base + i] - bt * vo[base + i];
        vo[base + i] = w;
        s[0] += double(norm2(w));
        acc_bdot(s[1], s[2], w, w);
    }
    block_partial<3, NT, 4>(s, red, slot, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_qmr_update(cx<T>* __restrict__ x,
                                                   const cx<T>* __restrict__ vc,
                                                   cx<T>* __restrict__ vo,
                                                   const cx<T>* __restrict__ p1,
                                                   cx<T>* __restrict__ p2, BicgSlot* st,
                                                   const int* __restrict__ act, int64_t nv,
                                                   RedScratch red, int nblk_mu, int par) {
    SLOT_PROLOGUE
    BicgSlot& S = st[slot];
    if (block_status(S) != SLOT_ACTIVE) return;
    const QmrScalars& Q = S.qmr[par];
    QmrScalars& N = S.qmr[par ^ 1];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    double mu[2];
    slot_totals<2, 0>(red, slot, nblk_mu, mu);
    z128 a, b;
    if (!qmr_ab(Q, mu, a, b)) {
        if (lead) {
            N = Q;
            N.flag = QMR_BREAKDOWN;
        }
        return;
    }
    double ws[3];
    slot_totals<3, 4>(red, slot, gridDim.x, ws);
    const double rho1 = sqrt(ws[0]);
    // column n of H through G_{n-2} and G_{n-1}; no entry above the diagonal
    // in the first column of a cycle
    const z128 th = Q.n > 1 ? b : z128{0.0, 0.0};
    const z128 eps = zmul(Q.s2, th);
    const z128 th2 = Q.c2 * th;
    const z128 d2 = Q.c1 * th2 + zmul(Q.s1, a);
    const z128 gam = Q.c1 * a - zmul(zconj(Q.s1), th2);
    // G_n zeroes rho_{n+1} below gam: c real, r = (gam/|gam|) nu
    double c;
    z128 sn, r;
    const double ag = hypot(gam.x, gam.y);
    if (ag == 0.0) {
        c = 0.0;
        sn = z128{1.0, 0.0};
        r = z128{rho1, 0.0};
    } else {
        const double nu = hypot(ag, rho1);
        const z128 ph{gam.x / ag, gam.y / ag};
        c = ag / nu;
        sn = (rho1 / nu) * ph;
        r = nu * ph;
    }
    const bool bad = !(r.x != 0.0 || r.y != 0.0) || !isfinite(r.x) || !isfinite(r.y) ||
                     !isfinite(ws[0]) || !isfinite(ws[1]) || !isfinite(ws[2]);
    if (bad) {
        if (lead) {
            N = Q;
            N.flag = QMR_BREAKDOWN;
        }
        return;
    }
    const z128 phi = c * Q.tau;
    const z128 ri = zdiv(z128{1.0, 0.0}, r);
    const cx<T> rit{T(ri.x), T(ri.y)}, d2t{T(d2.x), T(d2.y)}, et{T(eps.x), T(eps.y)};
    const cx<T> pht{T(phi.x), T(phi.y)};
    const T iw = rho1 > 0.0 ? T(1.0 / rho1) : T(0);
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> pn = rit * (vc[base + i] - d2t * p1[base + i] - et * p2[base + i]);
        p2[base + i] = pn;
        x[base + i] = x[base + i] + pht * pn;
        vo[base + i] = iw * vo[base + i];
    }
    if (lead) {
        const z128 tau1 = -1.0 * zmul(zconj(sn), Q.tau);
        const z128 del1 = rho1 > 0.0 ? (1.0 / ws[0]) * z128{ws[1], ws[2]} : z128{0.0, 0.0};
        N.delta_prev = Q.delta;
        N.delta = del1;
        N.s2 = Q.s1;
        N.c2 = Q.c1;
        N.s1 = sn;
        N.c1 = c;
        N.tau = tau1;
        N.rho = rho1;
        N.stop2 = Q.stop2;
        N.n = Q.n + 1;
        const double t2 = tau1.x * tau1.x + tau1.y * tau1.y;
        const double est2 = double(Q.n + 1) * t2;
        // FP32 cycles: a quasi-residual that fell by less than a tenth over
        // kQmrStagSteps steps has stagnated (the FP32 Lanczos vectors lost
        // their bi-orthogonality); the cycle ends and restarts from the
        // FP64 residual
        bool stagnated = false;
        N.mark2 = Q.mark2;
        N.mark = Q.mark;
        if (Q.mark2 > 0.0 && N.n - Q.mark >= kQmrStagSteps) {
            stagnated = t2 > 0.81 * Q.mark2;
            N.mark2 = t2;
            N.mark = N.n;
        }
        S.iters += 1;
        S.matvecs += 1;
        S.rnorm2 = est2;
        N.flag = (rho1 == 0.0 || est2 <= Q.stop2 || stagnated) ? QMR_CONVERGED
                 : (del1.x == 0.0 && del1.y == 0.0)         ? QMR_BREAKDOWN
                 : (S.iters >= S.maxit)                     ? QMR_MAXIT
                                                            : QMR_GO;
    }
}

// The flag of the copy just written becomes the slot status.
__global__ __launch_bounds__(NT) void k_qmr_fin(BicgSlot* st, const int* act, int par) {
    if (threadIdx.x != 0) return;
    BicgSlot& S = st[act[blockIdx.x]];
    if (S.status != SLOT_ACTIVE) return;
    const int fl = S.qmr[par].flag;
    if (fl == QMR_CONVERGED) S.status = SLOT_CONVERGED;
    else if (fl == QMR_BREAKDOWN) S.status = SLOT_BREAKDOWN;
    else if (fl == QMR_MAXIT) S.status = SLOT_MAXIT;
}

// Start of a QMR cycle from the residual r (the T vector the FP64 check or
// the start wrote; rho_1 = sqrt(rnorm2), delta_1 = r^T r / rho_1^2): v_1 =
// r / rho_1 into va, zero vb, p1, p2.  Only slots with reset_p set.
template <typename T>
__global__ __launch_bounds__(NT) void k_qmr_start(const cx<T>* __restrict__ r,
                                                  cx<T>* __restrict__ va, cx<T>* __restrict__ vb,
                                                  cx<T>* __restrict__ p1, cx<T>* __restrict__ p2,
                                                  const BicgSlot* st, const int* __restrict__ act,
                                                  int64_t nv) {
    SLOT_PROLOGUE
    const BicgSlot& S = st[slot];
    if (S.status != SLOT_ACTIVE || !S.reset_p) return;  // not changed by this kernel
    const double rn = sqrt(S.rnorm2);
    const T sc = rn > 0.0 ? T(1.0 / rn) : T(0);
    const cx<T> zero{T(0), T(0)};
    for (int64_t i = i0; i < nv; i += stride) {
        va[base + i] = sc * r[base + i];
        vb[base + i] = zero;
        p1[base + i] = zero;
        p2[base + i] = zero;
    }
}
__global__ __launch_bounds__(NT) void k_qmr_start_fin(BicgSlot* st, const int* act,
                                                       double inner2) {
    if (threadIdx.x != 0) return;
    BicgSlot& S = st[act[blockIdx.x]];
    if (S.status != SLOT_ACTIVE || !S.reset_p) return;
    const double rn = sqrt(S.rnorm2);
    QmrScalars& Q = S.qmr[0];
    Q.rho = rn;
    Q.delta = rn > 0.0 ? (1.0 / S.rnorm2) * S.rho : z128{0.0, 0.0};
    Q.delta_prev = z128{1.0, 0.0};
    Q.s1 = Q.s2 = z128{0.0, 0.0};
    Q.c1 = Q.c2 = 1.0;
    Q.tau = z128{rn, 0.0};
    Q.stop2 = fmax(S.tol2 * S.bnorm2, inner2 * S.rnorm2);
    Q.mark2 = inner2 > 0.0 ? S.rnorm2 : 0.0;
    Q.mark = 1;
    Q.n = 1;
    Q.flag = rn > 0.0 ? QMR_GO : QMR_CONVERGED;
    S.reset_p = 0;
    if (rn == 0.0) S.status = SLOT_CONVERGED;
}

// --------------------------------------------------------- loss sums ------
// Slot s is right-hand side rhs0 + s; einc and p are indexed by the global
// right-hand side, y, w and kv by the chunk (system = slot / n_traj).
__global__ __launch_bounds__(NT) void k_loss_sums(const z128* __restrict__ einc,
                                                  const z128* __restrict__ p,
                                                  const z128* __restrict__ y,
                                                  const double* __restrict__ w,
                                                  const int* __restrict__ occ_lin, Geo g, double d,
                                                  const double* __restrict__ kv,
                                                  const double* __restrict__ r0, int n_traj,
                                                  int64_t rhs0, RedScratch red) {
    const int slot = blockIdx.y;
    const int64_t rhs = rhs0 + slot;
    const int sys = slot / n_traj;
    const int t = slot - sys * n_traj;
    const double z0 = r0[3 * t + 2];
    const double kvs = kv[sys];
    const int64_t n = g.n_occ;
    const z128* E = einc + rhs * 3 * n;
    const z128* P = p + rhs * 3 * n;
    const z128* Y = y + int64_t(slot) * 3 * n;
    const double* W = w + int64_t(sys) * n;
    const int plane = g.nx * g.ny;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
        const int iz = occ_lin[i] / plane;
        const double z = d * (iz - 0.5 * g.nz + 0.5);
        double sn, cs;
        sincos(-2.0 * kvs * (z - z0), &sn, &cs);  // exp(-2 i omega (z - z0)/v)
        const z128 ph{cs, sn};
        double p2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const z128 e = E[c * n + i], pc = P[c * n + i], yc = Y[c * n + i];
            z128 gq = ph * e;  // auxiliary field of eq. (34)
            if (c < 2) gq = -gq;
            acc_bdot(s[0], s[1], gq, pc);  // bilinear, eq. (32)
            acc_cdot(s[2], s[3], e, pc);
            acc_cdot(s[5], s[6], pc, yc);
            p2 += norm2(pc);
        }
        s[4] += W[i] * p2;
        s[7] += p2;
    }
    block_partial<8, NT>(s, red, slot, blockIdx.x);
}
__global__ __launch_bounds__(NT) void k_fin_loss(double* __restrict__ out, RedScratch red,
                                                 int nblk) {
    const int slot = blockIdx.x;
    double tot[8];
    sum_rows<8, NT>(red, slot, nblk, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) out[slot * 8 + k] = tot[k];
}

}  // namespace

// ---------------------------------------------------------------- launchers

#define GRID(nv) dim3(blocks_for(nv, red.max_blocks), n_act)
#define FIN(kernel, ...)                                                          \
    do {                                                                          \
        kernel<<<n_act, NT, 0, s>>>(st, act, red, blocks_for(nv, red.max_blocks), \
                                    ##__VA_ARGS__);                               \
        DDA_LAUNCH_CHECK();                                                       \
    } while (0)

template <typename T>
void bicg_norm_b(const cx<T>* b, BicgSlot* st, const int* act, int n_act, int64_t nv, double tol2,
                 double upd2, int maxit, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_norm_b<T><<<GRID(nv), NT, 0, s>>>(b, act, nv, red);
    DDA_LAUNCH_CHECK();
    FIN(k_fin_norm_b, tol2, upd2, maxit);
}
template <typename T>
void bicg_reset(const cx<T>* r, cx<T>* rhat, cx<T>* p, cx<T>* v, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_reset<T><<<GRID(nv), NT, 0, s>>>(r, rhat, p, v, act, nv, red);
    DDA_LAUNCH_CHECK();
    FIN(k_fin_reset);
}
template <typename T>
void bicg_update_p(const cx<T>* r, cx<T>* p, const cx<T>* v, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, bool fin_prev, hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    const int nblk = blocks_for(nv, red.max_blocks);
    if (fin_prev) k_update_p<T, true><<<grid, NT, 0, s>>>(r, p, v, st, act, nv, red, nblk);
    else k_update_p<T, false><<<grid, NT, 0, s>>>(r, p, v, st, act, nv, red, nblk);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_update_s(const cx<T>* r, const cx<T>* v, cx<T>* sv, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, int nblk_mv, hipStream_t s) {
    if (n_act == 0) return;
    if (nblk_mv < 1 || nblk_mv > red.max_blocks) throw Error(-3, "bad matvec row count");
    k_update_s<T><<<GRID(nv), NT, 0, s>>>(r, v, sv, st, act, nv, red, nblk_mv);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* rhat, const cx<T>* p, const cx<T>* sv,
                    const cx<T>* t, BicgSlot* st, const int* act, int n_act, int64_t nv,
                    RedScratch red, int nblk_mv, int nblk_s, hipStream_t s) {
    if (n_act == 0) return;
    if (nblk_mv < 1 || nblk_mv > red.max_blocks) throw Error(-3, "bad matvec row count");
    if (nblk_s == 0) nblk_s = blocks_for(nv, red.max_blocks);  // rows of k_update_s
    if (nblk_s < 1 || nblk_s > red.max_blocks) throw Error(-3, "bad s row count");
    k_update_xr<T><<<GRID(nv), NT, 0, s>>>(x, r, rhat, p, sv, t, st, act, nv, red, nblk_mv,
                                           nblk_s);
    DDA_LAUNCH_CHECK();
}
void bicg_finish(BicgSlot* st, const int* act, int n_act, int64_t nv, RedScratch red,
                 hipStream_t s) {
    if (n_act == 0) return;
    FIN(k_fin_xr);
}
template <typename T>
void residual(const cx<T>* b, const cx<T>* y, cx<T>* r, BicgSlot* st, const int* act, int n_act,
              int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_residual<T><<<GRID(nv), NT, 0, s>>>(b, y, r, act, nv, red);
    DDA_LAUNCH_CHECK();
    FIN(k_fin_residual);
}
template <typename T>
void cocg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* p, const cx<T>* q, BicgSlot* st,
                    const int* act, int n_act, int64_t nv, RedScratch red, int nblk_mu,
                    int par, bool finish, hipStream_t s) {
    if (n_act == 0) return;
    if (nblk_mu < 1 || nblk_mu > red.max_blocks) throw Error(-1, "bad partial row count");
    k_cocg_xr<T><<<GRID(nv), NT, 0, s>>>(x, r, p, q, st, act, nv, red, nblk_mu, par & 1);
    DDA_LAUNCH_CHECK();
    if (finish) FIN(k_fin_cocg_xr, par & 1);
}
int cocg_rows(int64_t nv, int max_blocks) { return blocks_for(nv, max_blocks); }
template <typename T>
void cocg_start(const z128* b, const z128* y, cx<T>* r_lo, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_true_residual<T><<<GRID(nv), NT, 0, s>>>(b, y, r_lo, act, nv, SlotFilter{st, FILTER_ALL},
                                               red);
    DDA_LAUNCH_CHECK();
    FIN(k_fin_cocg_start);
}
template <typename T>
void cocg_check(const z128* b, const z128* y, cx<T>* r_lo, BicgSlot* st, const int* act,
                int n_act, int64_t nv, int max_restarts, RedScratch red, hipStream_t s,
                bool always_reset) {
    if (n_act == 0) return;
    k_true_residual<T><<<GRID(nv), NT, 0, s>>>(b, y, r_lo, act, nv,
                                               SlotFilter{st, FILTER_CHECK}, red);
    DDA_LAUNCH_CHECK();
    FIN(k_fin_check, max_restarts, always_reset ? 1 : 0);
}
template <typename T>
void qmr_start(const cx<T>* r, cx<T>* va, cx<T>* vb, cx<T>* p1, cx<T>* p2, BicgSlot* st,
               const int* act, int n_act, int64_t nv, double inner, hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_qmr_start<T><<<grid, NT, 0, s>>>(r, va, vb, p1, p2, st, act, nv);
    DDA_LAUNCH_CHECK();
    k_qmr_start_fin<<<n_act, NT, 0, s>>>(st, act, inner * inner);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void qmr_step(cx<T>* x, const cx<T>* u, cx<T>* vc, cx<T>* vo, cx<T>* p1, cx<T>* p2,
              BicgSlot* st, const int* act, int n_act, int64_t nv, RedScratch red, int nblk_mu,
              int par, hipStream_t s) {
    if (n_act == 0) return;
    if (nblk_mu < 1 || nblk_mu > red.max_blocks) throw Error(-1, "bad partial row count");
    k_qmr_lanczos<T><<<GRID(nv), NT, 0, s>>>(vc, vo, u, st, act, nv, red, nblk_mu, par);
    DDA_LAUNCH_CHECK();
    k_qmr_update<T><<<GRID(nv), NT, 0, s>>>(x, vc, vo, p1, p2, st, act, nv, red, nblk_mu, par);
    DDA_LAUNCH_CHECK();
    k_qmr_fin<<<n_act, NT, 0, s>>>(st, act, par ^ 1);
    DDA_LAUNCH_CHECK();
}
void cocg_zero(z128* x, z64* x_lo, const int* act, int n_act, int64_t nv, hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_cocg_zero<<<grid, NT, 0, s>>>(x, x_lo, act, nv);
    DDA_LAUNCH_CHECK();
}
void mark_invalid(BicgSlot* st, const int* act, const int* err, int n, hipStream_t s) {
    if (n == 0) return;
    k_mark_invalid<<<(n + NT - 1) / NT, NT, 0, s>>>(st, act, err, n);
    DDA_LAUNCH_CHECK();
}
void accumulate_lo(z128* x, z64* x_lo, const int* act, int n_act, int64_t nv, SlotFilter f,
                   hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_accumulate_lo<<<grid, NT, 0, s>>>(x, x_lo, act, nv, f);
    DDA_LAUNCH_CHECK();
}
void scale_down(const z128* r, z64* r32, const BicgSlot* st, const int* act, int n_act, int64_t nv,
                hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_scale_down<<<grid, NT, 0, s>>>(r, r32, st, act, nv);
    DDA_LAUNCH_CHECK();
}
void accumulate_up(z128* x, const z64* d32, const BicgSlot* st, const int* act, int n_act,
                   int64_t nv, hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_accumulate_up<<<grid, NT, 0, s>>>(x, d32, st, act, nv);
    DDA_LAUNCH_CHECK();
}

void loss_sums(const z128* einc, const z128* p, const z128* y, const double* w, const int* occ_lin,
               const Geo& g, double d, const double* kv, const double* r0, int n_traj, int64_t rhs0,
               int nslots, double* out, RedScratch red, hipStream_t s) {
    if (nslots == 0) return;
    const int nb = blocks_for(g.n_occ, red.max_blocks);
    k_loss_sums<<<dim3(nb, nslots), NT, 0, s>>>(einc, p, y, w, occ_lin, g, d, kv, r0, n_traj, rhs0,
                                                red);
    DDA_LAUNCH_CHECK();
    k_fin_loss<<<nslots, NT, 0, s>>>(out, red, nb);
    DDA_LAUNCH_CHECK();
}

#define DDA_INST(T)                                                                              \
    template void bicg_norm_b<T>(const cx<T>*, BicgSlot*, const int*, int, int64_t, double,      \
                                 double, int, RedScratch, hipStream_t);                          \
    template void bicg_reset<T>(const cx<T>*, cx<T>*, cx<T>*, cx<T>*, BicgSlot*, const int*, int, \
                                int64_t, RedScratch, hipStream_t);                               \
    template void bicg_update_p<T>(const cx<T>*, cx<T>*, const cx<T>*, BicgSlot*, const int*,    \
                                   int, int64_t, RedScratch, bool, hipStream_t);                 \
    template void bicg_update_s<T>(const cx<T>*, const cx<T>*, cx<T>*, BicgSlot*, const int*,    \
                                   int, int64_t, RedScratch, int, hipStream_t);                  \
    template void bicg_update_xr<T>(cx<T>*, cx<T>*, const cx<T>*, const cx<T>*, const cx<T>*,    \
                                    const cx<T>*, BicgSlot*, const int*, int, int64_t,           \
                                    RedScratch, int, int, hipStream_t);                          \
    template void residual<T>(const cx<T>*, const cx<T>*, cx<T>*, BicgSlot*, const int*, int,    \
                              int64_t, RedScratch, hipStream_t);                                 \
    template void cocg_update_xr<T>(cx<T>*, cx<T>*, const cx<T>*, const cx<T>*, BicgSlot*,       \
                                    const int*, int, int64_t, RedScratch, int, int, bool,        \
                                    hipStream_t);                                                \
    template void cocg_start<T>(const z128*, const z128*, cx<T>*, BicgSlot*, const int*, int,    \
                                int64_t, RedScratch, hipStream_t);                               \
    template void cocg_check<T>(const z128*, const z128*, cx<T>*, BicgSlot*, const int*, int,    \
                                int64_t, int, RedScratch, hipStream_t, bool);                    \
    template void qmr_start<T>(const cx<T>*, cx<T>*, cx<T>*, cx<T>*, cx<T>*, BicgSlot*,          \
                               const int*, int, int64_t, double, hipStream_t);                   \
    template void qmr_step<T>(cx<T>*, const cx<T>*, cx<T>*, cx<T>*, cx<T>*, cx<T>*, BicgSlot*,   \
                              const int*, int, int64_t, RedScratch, int, int, hipStream_t);
DDA_INST(double)
DDA_INST(float)

}  // namespace dda

// Per right-hand-side solver state resident on the device, and the
// deterministic block reduction shared by the Krylov and the fused FFT
// kernels.
#pragma once

#include "common.h"

namespace dda {

enum SlotStatus : int {
    SLOT_ACTIVE = 0,
    SLOT_CONVERGED = 1,  // the recursive residual met the tolerance
    SLOT_HALF = 2,       // BiCGStab: ||s|| met the tolerance inside an iteration
    SLOT_BREAKDOWN = 3,  // a Krylov scalar vanished or went non-finite
    SLOT_MAXIT = 4,      // the iteration limit was reached
    // terminal states, set by the FP64 residual check of the COCG driver
    SLOT_DONE = 5,              // the FP64 residual met the tolerance
    SLOT_FAIL_NOCONV = 6,       // iteration limit reached above the tolerance
    SLOT_FAIL_BREAKDOWN = 7,    // breakdowns beyond the restart budget
    SLOT_FAIL_INVALID = 8,      // the system's permittivity was rejected
};

// QMR for complex-symmetric systems: the scalars one Lanczos step reads.
// Every step reads one copy and writes the other (by the parity of its index
// in the interval), so the blocks of a launch never see a value another block
// of the same launch has just written.
struct QmrScalars {
    z128 delta, delta_prev;  // v_n^T v_n and v_{n-1}^T v_{n-1} (bilinear)
    z128 s1, s2;             // sines of the rotations G_{n-1}, G_{n-2}
    z128 tau;                // quasi-residual
    double rho;              // ||w_n||: v_n = w_n / rho_n
    double c1, c2;           // cosines of G_{n-1}, G_{n-2}
    double stop2;            // the cycle ends when (n+1)|tau|^2 falls to this
    double mark2;            // |tau|^2 at step `mark` (stagnation test; 0: off)
    int mark;
    int n;                   // Lanczos step of the cycle (1-based)
    int flag;                // QMR_GO, QMR_CONVERGED, QMR_BREAKDOWN, QMR_MAXIT
};
enum QmrFlag : int { QMR_GO = 0, QMR_CONVERGED = 1, QMR_BREAKDOWN = 2, QMR_MAXIT = 3 };

struct BicgSlot {
    z128 rho, rho_old, alpha, omega;  // BiCGStab; COCG uses rho and alpha
    z128 rv, ts;                      // BiCGStab <rhat, v>, <t, s>; COCG: rv = p^T q
    z128 beta;                        // COCG: p <- r + beta p
    z128 rho1;                        // COCG: r^T r of the odd iterations of an interval
                                      // (rho holds the even ones; see CocgFold)
    double tt;                        // <t, t>
    double bnorm2;                    // ||b||^2
    double rnorm2;                    // ||r||^2 (recursive, or true after a residual pass)
    double rmax2;                     // largest ||r||^2 since the last FP64 residual
    double best2;                     // smallest FP64 ||r||^2 of the mixed-precision checks
    double tol2;                      // tol^2
    double upd2;                      // reliable update when rnorm2 < upd2 * rmax2 (0: never)
    int status;
    int iters;
    int want_update;                  // set by the device, cleared by the FP64 residual pass
    int matvecs;                      // matrix-vector products spent on this slot
    int restarts;                     // breakdown restarts so far
    int reset_p;                      // COCG: the next direction update takes p = r
    int maxit;                        // iteration limit
    int stall;                        // FP64 checks since best2 last halved
    QmrScalars qmr[2];                // QMR: the two alternating copies
};

__host__ __device__ inline bool slot_terminal(int status) { return status >= SLOT_DONE; }

// COCG: a slot waits for the FP64 residual check when its recursive residual
// converged, a scalar broke down, the iteration limit was hit, or the
// residual fell far enough below its running maximum for a reliable update.
__device__ __forceinline__ bool needs_check(const BicgSlot& S) {
    return S.status == SLOT_CONVERGED || S.status == SLOT_BREAKDOWN || S.status == SLOT_MAXIT ||
           (S.status == SLOT_ACTIVE && S.want_update);
}

// Which listed slots a kernel processes: all of them, only those still
// iterating, or only those waiting for the FP64 check.  A block whose slot is
// filtered out returns before touching memory, so converged slots cost one
// load of their status until the host drops them from the list.
enum FilterMode : int { FILTER_ALL = 0, FILTER_ACTIVE = 1, FILTER_CHECK = 2 };
struct SlotFilter {
    const BicgSlot* st;
    int mode;
};
__device__ __forceinline__ bool slot_live(SlotFilter f, int64_t slot) {
    if (f.mode == FILTER_ALL) return true;
    const BicgSlot& S = f.st[slot];
    return f.mode == FILTER_ACTIVE ? S.status == SLOT_ACTIVE : needs_check(S);
}

// Reduction scratch: per slot, up to `max_blocks` partial rows of up to 8
// doubles.  A reduction is two kernels: the work kernel writes one row per
// block (block_partial), then a finalize kernel with one block per slot sums
// the rows in index order (sum_rows) and updates the slot's scalars.  No
// atomics and no fences; the result does not depend on block scheduling.
struct RedScratch {
    double* partial;  // [max_slots][max_blocks][8]
    int max_blocks;
};

__device__ __forceinline__ z128 zdiv(z128 a, z128 b) {
    const double s = 1.0 / (b.x * b.x + b.y * b.y);
    return z128{(a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s};
}

template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_down(v[k], off, 64);
    }
}

// Block-reduces K values (blockDim.x == NT) and stores them as partial row
// `blk` of `slot`.  Must be called by every thread of the block.
template <int K, int NT, int OFF = 0>
__device__ __forceinline__ void block_partial(double (&v)[K], RedScratch red, int slot, int blk) {
    static_assert(OFF + K <= 8, "a partial row holds 8 doubles");
    __shared__ double sm[NT / 64][K];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    wave_sum<K>(v);
    if (lane == 0)
        for (int k = 0; k < K; ++k) sm[w][k] = v[k];
    __syncthreads();
    if (tid == 0) {
        double* row = red.partial + (int64_t(slot) * red.max_blocks + blk) * 8;
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sm[q][k];
            row[OFF + k] = s;
        }
    }
}

// Sums rows 0..nblk-1 of `slot` in a fixed order; the totals are valid in
// thread 0.  Must be called by every thread of the block.
template <int K, int NT, int OFF = 0>
__device__ __forceinline__ void sum_rows(RedScratch red, int slot, int nblk, double (&tot)[K]) {
    __shared__ double sm[NT / 64][K];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double* rows = red.partial + int64_t(slot) * red.max_blocks * 8;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = tid; b < nblk; b += NT) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += rows[int64_t(b) * 8 + OFF + k];
    }
    wave_sum<K>(acc);
    if (lane == 0)
        for (int k = 0; k < K; ++k) sm[w][k] = acc[k];
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sm[q][k];
            tot[k] = s;
        }
    }
}

// Sums rows 0..nblk-1 of `slot` exactly as sum_rows<K, NTS, OFF> does
// (same grouping of rows by thread, same order) in a block of NTB >= NTS
// threads, so that a value summed by a kernel of another block size is
// bit-identical.  Totals valid in thread 0; every thread must call it.
template <int K, int NTS, int OFF, int NTB>
__device__ __forceinline__ void sum_rows_as(RedScratch red, int slot, int nblk, double (&tot)[K]) {
    static_assert(NTB >= NTS && NTS % 64 == 0, "block too small");
    __shared__ double sm[NTS / 64][K];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double* rows = red.partial + int64_t(slot) * red.max_blocks * 8;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    if (tid < NTS) {
        for (int b = tid; b < nblk; b += NTS) {
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += rows[int64_t(b) * 8 + OFF + k];
        }
    }
    wave_sum<K>(acc);
    if (lane == 0 && w < NTS / 64)
        for (int k = 0; k < K; ++k) sm[w][k] = acc[k];
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < NTS / 64; ++q) s += sm[q][k];
            tot[k] = s;
        }
    }
}

// ----------------------------------------------------------- COCG step ----
// The end of a COCG iteration: from tot = (r^T r re, im, ||r||^2) of the
// updated residual, the next status (SLOT_ACTIVE to go on) and
// beta = rho_new / rho_old.  It reads only fields that no kernel of the
// iteration writes, so every block evaluating it decides alike.
__device__ __forceinline__ int cocg_next(const BicgSlot& S, const double (&tot)[3], z128 rho_old,
                                         z128& beta) {
    beta = z128{0.0, 0.0};
    if (!(isfinite(tot[0]) && isfinite(tot[1]) && isfinite(tot[2]))) return SLOT_BREAKDOWN;
    const z128 rho_new{tot[0], tot[1]};
    const bool rho0 = rho_old.x == 0.0 && rho_old.y == 0.0;
    const bool rhon0 = rho_new.x == 0.0 && rho_new.y == 0.0;
    if (!rho0) beta = zdiv(rho_new, rho_old);
    if (tot[2] <= S.tol2 * S.bnorm2) return SLOT_CONVERGED;
    if (rho0 || rhon0) return SLOT_BREAKDOWN;
    if (S.iters >= S.maxit) return SLOT_MAXIT;
    return SLOT_ACTIVE;
}
// Its bookkeeping, by one thread: residual norms for the FP64 check, the
// reliable-update flag, beta, rho (into copy `dst`: 0 = rho, 1 = rho1) and a
// terminal status.
__device__ __forceinline__ void cocg_record(BicgSlot& S, const double (&tot)[3], int status,
                                            z128 beta, int dst) {
    S.rnorm2 = tot[2];
    if (!(isfinite(tot[0]) && isfinite(tot[1]) && isfinite(tot[2]))) {
        S.status = SLOT_BREAKDOWN;
        return;
    }
    S.beta = beta;
    if (dst) S.rho1 = z128{tot[0], tot[1]};
    else S.rho = z128{tot[0], tot[1]};
    if (tot[2] > S.rmax2) S.rmax2 = tot[2];
    if (S.upd2 > 0.0 && tot[2] < S.upd2 * S.rmax2) S.want_update = 1;
    if (status != SLOT_ACTIVE) S.status = status;
}

// The end of COCG iteration k - 1 folded into the direction update of
// iteration k (the first kernel of its matvec), instead of a kernel of its
// own: every block sums the rows of r^T r the x, r update left (doubles 4..6,
// nblk rows, in the finalizer's order) and takes beta and the decision
// itself; the slot's first block records them.  Iteration k - 1 has parity
// `par` and read its rho from copy par; the record goes to copy par ^ 1, so
// no block of the launch reads a value another one writes.  nblk == 0: no
// fold (beta and reset_p come from the slot state).
struct CocgFold {
    BicgSlot* st;
    RedScratch red;
    int nblk;
    int par;
};
constexpr int kCocgFinThreads = 256;  // block size of the standalone finalizer

// Every thread of the block calls it (after a block-uniform check that the
// slot is active); returns false when the slot stops here.
template <int NTB>
__device__ __forceinline__ bool cocg_fold(CocgFold fo, int slot, bool lead, z128& beta) {
    double tot[3];
    sum_rows_as<3, kCocgFinThreads, 4, NTB>(fo.red, slot, fo.nblk, tot);
    __shared__ double bc[2];
    __shared__ int go;
    if (threadIdx.x == 0) {
        BicgSlot& S = fo.st[slot];
        z128 b;
        const int status = cocg_next(S, tot, fo.par ? S.rho1 : S.rho, b);
        bc[0] = b.x;
        bc[1] = b.y;
        go = status == SLOT_ACTIVE;
        if (lead) cocg_record(S, tot, status, b, fo.par ^ 1);
    }
    __syncthreads();
    beta = z128{bc[0], bc[1]};
    return go != 0;
}

// --------------------------------------------------- BiCGStab folds ------
// s = r - alpha v and p = r + beta (p - omega v), their complex products
// written out with explicit fma calls so that every kernel built from them
// rounds the same way (each update is done either by a vector kernel or by
// the x kernel of the next matvec).
template <typename T>
__device__ __forceinline__ cx<T> bicg_s_of(cx<T> r, cx<T> a, cx<T> v) {
    return cx<T>{fma(-a.x, v.x, fma(a.y, v.y, r.x)), fma(-a.x, v.y, fma(-a.y, v.x, r.y))};
}
template <typename T>
__device__ __forceinline__ cx<T> bicg_p_of(cx<T> r, cx<T> bt, cx<T> p, cx<T> om, cx<T> v) {
    const cx<T> t{fma(-om.x, v.x, fma(om.y, v.y, p.x)), fma(-om.x, v.y, fma(-om.y, v.x, p.y))};
    return cx<T>{fma(bt.x, t.x, fma(-bt.y, t.y, r.x)), fma(bt.x, t.y, fma(bt.y, t.x, r.y))};
}
template <typename T>
__device__ __forceinline__ double bicg_norm2(cx<T> s) {
    return double(fma(s.x, s.x, s.y * s.y));
}

// End of a BiCGStab iteration from the rows <rhat, r>, ||r||^2: the new rho,
// the residual norm, the iteration count and the status.  Returns the new
// status; the state is stored by `lead` only, and the decision reads no field
// that is written here, so every block evaluating it decides alike.
__device__ __forceinline__ int finish_iteration(BicgSlot& S, int status, const double (&tot)[3],
                                                bool lead) {
    int ns = status;
    if (!(isfinite(tot[0]) && isfinite(tot[1]) && isfinite(tot[2]))) {
        ns = SLOT_BREAKDOWN;
    } else if (status == SLOT_HALF || tot[2] <= S.tol2 * S.bnorm2) {
        ns = SLOT_CONVERGED;
    } else if ((tot[0] == 0.0 && tot[1] == 0.0) || (S.omega.x == 0.0 && S.omega.y == 0.0)) {
        ns = SLOT_BREAKDOWN;
    }
    if (lead) {
        S.iters += 1;
        S.rho = z128{tot[0], tot[1]};
        S.rnorm2 = tot[2];
        if (ns != status) S.status = ns;
    }
    return ns;
}

// A BiCGStab vector update folded into the x kernel of the next matvec
// (kind BICG_FOLD_S: s = r - alpha v before t = A s; BICG_FOLD_P: p = r +
// beta (p - omega v) before v = A p).  Every block sums the rows the vector
// kernel would sum, in its order (nblk rows: <rhat, v> for s; <rhat, r>,
// ||r||^2 for p, or none when the iteration's rho is already in the state),
// forms the scalars itself and updates the elements it gathers in place;
// block 0 records the scalars and the status.  The s update also writes the
// partial rows of ||s||^2 (double 6 of row `blk`).  kind 0: no fold.
enum BicgFoldKind { BICG_FOLD_NONE = 0, BICG_FOLD_S = 1, BICG_FOLD_P = 2 };
struct BicgFold {
    BicgSlot* st;
    RedScratch red;
    int kind;
    int nblk;
    const void* v;  // v = A p, laid out like the input
};
constexpr int kBicgUpdateThreads = 256;  // block size of the vector kernels it stands in for

// s update: every thread of the block calls it for a slot that is iterating
// (status read once per block); returns false on a breakdown (<rhat, v> zero
// or not finite), which block `lead` records.
template <int NTB>
__device__ __forceinline__ bool bicg_sfold(BicgFold fo, int slot, bool lead, z128& alpha) {
    double rv[2];
    sum_rows_as<2, kBicgUpdateThreads, 0, NTB>(fo.red, slot, fo.nblk, rv);
    __shared__ double bc[2];
    __shared__ int go;
    if (threadIdx.x == 0) {
        BicgSlot& S = fo.st[slot];
        const z128 rvz{rv[0], rv[1]};
        const bool bad = (rv[0] == 0.0 && rv[1] == 0.0) || !isfinite(rv[0]) || !isfinite(rv[1]);
        const z128 al = bad ? z128{0.0, 0.0} : zdiv(S.rho, rvz);
        if (lead) {
            S.rv = rvz;
            if (bad) S.status = SLOT_BREAKDOWN;
            else S.alpha = al;
        }
        bc[0] = al.x;
        bc[1] = al.y;
        go = !bad;
    }
    __syncthreads();
    alpha = z128{bc[0], bc[1]};
    return go != 0;
}

// p update: every thread of the block calls it with the block's reading of
// the status; returns false when the slot does not go on (then the x kernel
// transforms the old p, whose product nothing reads).  beta and omega come
// back in every thread.
template <int NTB>
__device__ __forceinline__ bool bicg_pfold(BicgFold fo, int slot, int status, bool lead,
                                           z128& beta, z128& omega) {
    const bool fin = fo.nblk > 0;
    if (!(status == SLOT_ACTIVE || (fin && status == SLOT_HALF))) return false;  // uniform
    double tot[3] = {0.0, 0.0, 0.0};
    if (fin) sum_rows_as<3, kBicgUpdateThreads, 0, NTB>(fo.red, slot, fo.nblk, tot);
    __shared__ double bc[4];
    __shared__ int go;
    if (threadIdx.x == 0) {
        BicgSlot& S = fo.st[slot];
        // the stored rho is read before finish_iteration replaces it, and the
        // choice is made on the values: a choice between the two addresses
        // would put tot in scratch memory behind a flat load
        const z128 rho_st = S.rho;
        int ns = status;
        if (fin) ns = finish_iteration(S, status, tot, lead);
        const z128 rho{fin ? tot[0] : rho_st.x, fin ? tot[1] : rho_st.y};
        const z128 b = zdiv(rho, S.rho_old) * zdiv(S.alpha, S.omega);
        bc[0] = b.x;
        bc[1] = b.y;
        bc[2] = S.omega.x;
        bc[3] = S.omega.y;
        go = ns == SLOT_ACTIVE;
    }
    __syncthreads();
    beta = z128{bc[0], bc[1]};
    omega = z128{bc[2], bc[3]};
    return go != 0;
}

}  // namespace dda

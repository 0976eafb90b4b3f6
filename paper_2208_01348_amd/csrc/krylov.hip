// BiCGStab (van der Vorst 1992) over many right-hand sides at once, with all
// scalars resident on the device, and the FP64 loss reductions.
//
// One grid covers every active slot: blockIdx.y picks the slot from the
// active list, blockIdx.x a contiguous piece of its vector.  Dot products are
// reduced deterministically: each block writes its partial sums to a fixed
// row, and the last block of a slot to arrive (counted with an atomic) sums the
// rows in index order and updates that slot's scalars.  The host never
// synchronises inside an iteration.
#include "krylov.h"

namespace dda {

namespace {

constexpr int NT = 256;
constexpr int EPB = 2048;  // vector elements per block

inline int blocks_for(int64_t nv, int max_blocks) {
    int64_t b = (nv + EPB - 1) / EPB;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return int(b);
}

template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_down(v[k], off, 64);
    }
}

// Block-reduces K values, stores them as this block's partial row, and
// returns true in the (single) last block of the slot, where `tot` then
// holds the slot totals summed in fixed order (valid in thread 0).
template <int K>
__device__ bool reduce_last(double (&v)[K], double (&tot)[K], RedScratch red, int slot,
                            int nblk) {
    __shared__ double sm[NT / 64][K];
    __shared__ bool is_last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    wave_sum<K>(v);
    if (lane == 0)
        for (int k = 0; k < K; ++k) sm[w][k] = v[k];
    __syncthreads();
    double* rows = red.partial + (int64_t(slot) * red.max_blocks) * 8;
    if (tid == 0) {
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sm[q][k];
            rows[blockIdx.x * 8 + k] = s;
        }
        __threadfence();
        const unsigned prev = atomicAdd(&red.counters[slot], 1u);
        is_last = (prev == unsigned(nblk - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = tid; b < nblk; b += NT) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += __builtin_nontemporal_load(&rows[b * 8 + k]);
    }
    wave_sum<K>(acc);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < K; ++k) sm[w][k] = acc[k];
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sm[q][k];
            tot[k] = s;
        }
        red.counters[slot] = 0u;
    }
    return true;
}

__device__ __forceinline__ z128 zdiv(z128 a, z128 b) {
    const double s = 1.0 / (b.x * b.x + b.y * b.y);
    return z128{(a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s};
}

template <typename T>
__device__ __forceinline__ z128 up(cx<T> a) { return z128{double(a.x), double(a.y)}; }

// conj(a) * b accumulated in double
template <typename T>
__device__ __forceinline__ void acc_cdot(double& re, double& im, cx<T> a, cx<T> b) {
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    re += ax * bx + ay * by;
    im += ax * by - ay * bx;
}

#define SLOT_PROLOGUE                                                   \
    const int slot = act[blockIdx.y];                                   \
    const int64_t base = int64_t(slot) * nv;                            \
    const int64_t i0 = int64_t(blockIdx.x) * NT + threadIdx.x;          \
    const int64_t stride = int64_t(gridDim.x) * NT;

// ---------------------------------------------------------------- kernels

template <typename T>
__global__ __launch_bounds__(NT) void k_norm_b(const cx<T>* __restrict__ b, BicgSlot* st,
                                               const int* __restrict__ act, int64_t nv,
                                               double tol2, RedScratch red) {
    SLOT_PROLOGUE
    double v[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) v[0] += double(norm2(b[base + i]));
    double tot[1];
    if (reduce_last<1>(v, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        st[slot].bnorm2 = tot[0];
        st[slot].tol2 = tol2;
        st[slot].iters = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_reset(const cx<T>* __restrict__ r, cx<T>* __restrict__ rhat,
                                              cx<T>* __restrict__ p, cx<T>* __restrict__ v,
                                              BicgSlot* st, const int* __restrict__ act,
                                              int64_t nv, RedScratch red) {
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
    double tot[1];
    if (reduce_last<1>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        BicgSlot& S = st[slot];
        S.rho = z128{tot[0], 0.0};
        S.rho_old = z128{1.0, 0.0};
        S.alpha = z128{1.0, 0.0};
        S.omega = z128{1.0, 0.0};
        S.rnorm2 = tot[0];
        S.status = (tot[0] <= S.tol2 * S.bnorm2) ? SLOT_CONVERGED : SLOT_ACTIVE;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_update_p(const cx<T>* __restrict__ r, cx<T>* __restrict__ p,
                                                 const cx<T>* __restrict__ v, const BicgSlot* st,
                                                 const int* __restrict__ act, int64_t nv) {
    SLOT_PROLOGUE
    const BicgSlot& S = st[slot];
    if (S.status != SLOT_ACTIVE) return;
    const z128 beta = zdiv(S.rho, S.rho_old) * zdiv(S.alpha, S.omega);
    const cx<T> bt{T(beta.x), T(beta.y)};
    const cx<T> om{T(S.omega.x), T(S.omega.y)};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> pi = p[base + i];
        p[base + i] = r[base + i] + bt * (pi - om * v[base + i]);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_alpha(const cx<T>* __restrict__ rhat,
                                              const cx<T>* __restrict__ v, BicgSlot* st,
                                              const int* __restrict__ act, int64_t nv,
                                              RedScratch red) {
    SLOT_PROLOGUE
    if (st[slot].status != SLOT_ACTIVE) return;
    double s[2] = {0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) acc_cdot(s[0], s[1], rhat[base + i], v[base + i]);
    double tot[2];
    if (reduce_last<2>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        BicgSlot& S = st[slot];
        S.rv = z128{tot[0], tot[1]};
        if (tot[0] == 0.0 && tot[1] == 0.0) {
            S.status = SLOT_BREAKDOWN;
        } else {
            S.alpha = zdiv(S.rho, S.rv);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_update_s(const cx<T>* __restrict__ r,
                                                 const cx<T>* __restrict__ v, cx<T>* __restrict__ sv,
                                                 BicgSlot* st, const int* __restrict__ act,
                                                 int64_t nv, RedScratch red) {
    SLOT_PROLOGUE
    if (st[slot].status != SLOT_ACTIVE) return;
    const z128 al = st[slot].alpha;
    const cx<T> a{T(al.x), T(al.y)};
    double s[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> si = r[base + i] - a * v[base + i];
        sv[base + i] = si;
        s[0] += double(norm2(si));
    }
    double tot[1];
    if (reduce_last<1>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        BicgSlot& S = st[slot];
        if (tot[0] <= S.tol2 * S.bnorm2) S.status = SLOT_HALF;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_omega(const cx<T>* __restrict__ t,
                                              const cx<T>* __restrict__ sv, BicgSlot* st,
                                              const int* __restrict__ act, int64_t nv,
                                              RedScratch red) {
    SLOT_PROLOGUE
    const int status = st[slot].status;
    if (status == SLOT_HALF) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st[slot].omega = z128{0.0, 0.0};
        return;
    }
    if (status != SLOT_ACTIVE) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> ti = t[base + i];
        acc_cdot(s[0], s[1], ti, sv[base + i]);
        s[2] += double(norm2(ti));
    }
    double tot[3];
    if (reduce_last<3>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        BicgSlot& S = st[slot];
        S.ts = z128{tot[0], tot[1]};
        S.tt = tot[2];
        S.omega = tot[2] > 0.0 ? z128{tot[0] / tot[2], tot[1] / tot[2]} : z128{0.0, 0.0};
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_update_xr(cx<T>* __restrict__ x, cx<T>* __restrict__ r,
                                                  const cx<T>* __restrict__ rhat,
                                                  const cx<T>* __restrict__ p,
                                                  const cx<T>* __restrict__ sv,
                                                  const cx<T>* __restrict__ t, BicgSlot* st,
                                                  const int* __restrict__ act, int64_t nv,
                                                  RedScratch red) {
    SLOT_PROLOGUE
    const int status = st[slot].status;
    if (status != SLOT_ACTIVE && status != SLOT_HALF) return;
    const z128 al = st[slot].alpha, om = st[slot].omega;
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
    double tot[3];
    if (reduce_last<3>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) {
        BicgSlot& S = st[slot];
        S.iters += 1;
        S.rho_old = S.rho;
        S.rho = z128{tot[0], tot[1]};
        S.rnorm2 = tot[2];
        if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2])) {
            S.status = SLOT_BREAKDOWN;
        } else if (status == SLOT_HALF || tot[2] <= S.tol2 * S.bnorm2) {
            S.status = SLOT_CONVERGED;
        } else if ((tot[0] == 0.0 && tot[1] == 0.0) || (S.omega.x == 0.0 && S.omega.y == 0.0)) {
            S.status = SLOT_BREAKDOWN;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_residual(const cx<T>* __restrict__ b,
                                                 const cx<T>* __restrict__ y, cx<T>* __restrict__ r,
                                                 BicgSlot* st, const int* __restrict__ act,
                                                 int64_t nv, RedScratch red) {
    SLOT_PROLOGUE
    double s[1] = {0.0};
    for (int64_t i = i0; i < nv; i += stride) {
        const cx<T> ri = b[base + i] - y[base + i];
        r[base + i] = ri;
        s[0] += double(norm2(ri));
    }
    double tot[1];
    if (reduce_last<1>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0) st[slot].rnorm2 = tot[0];
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
    for (int64_t i = i0; i < nv; i += stride) x[base + i] = x[base + i] + sc * cvt<double>(d32[base + i]);
}

// Loss sums (see krylov.h).  Slot s is right-hand side rhs0 + s.
__global__ __launch_bounds__(NT) void k_loss_sums(const z128* __restrict__ einc,
                                                  const z128* __restrict__ p,
                                                  const z128* __restrict__ y,
                                                  const double* __restrict__ w,
                                                  const int* __restrict__ occ_lin, Geo g, double d,
                                                  const double* __restrict__ kv,
                                                  const double* __restrict__ r0, int n_traj,
                                                  int64_t rhs0, double* __restrict__ out,
                                                  RedScratch red) {
    const int slot = blockIdx.y;
    const int64_t rhs = rhs0 + slot;
    const int sys = slot / n_traj;  // chunk-local system (chunks hold whole energies)
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
            z128 gq = ph * e;
            if (c < 2) gq = -gq;
            const z128 gp = gq * pc;  // bilinear, eq. (32)
            s[0] += gp.x;
            s[1] += gp.y;
            acc_cdot(s[2], s[3], e, pc);
            acc_cdot(s[5], s[6], pc, yc);
            p2 += norm2(pc);
        }
        s[4] += W[i] * p2;
        s[7] += p2;
    }
    double tot[8];
    if (reduce_last<8>(s, tot, red, slot, gridDim.x) && threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) out[slot * 8 + k] = tot[k];
}

}  // namespace

// ---------------------------------------------------------------- launchers

#define GRID(nv) dim3(blocks_for(nv, red.max_blocks), n_act)

template <typename T>
void bicg_norm_b(const cx<T>* b, BicgSlot* st, const int* act, int n_act, int64_t nv, double tol2,
                 RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_norm_b<T><<<GRID(nv), NT, 0, s>>>(b, st, act, nv, tol2, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_reset(const cx<T>* r, cx<T>* rhat, cx<T>* p, cx<T>* v, BicgSlot* st, const int* act,
                int n_act, int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_reset<T><<<GRID(nv), NT, 0, s>>>(r, rhat, p, v, st, act, nv, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_update_p(const cx<T>* r, cx<T>* p, const cx<T>* v, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, hipStream_t s) {
    if (n_act == 0) return;
    dim3 grid(blocks_for(nv, 1 << 20), n_act);
    k_update_p<T><<<grid, NT, 0, s>>>(r, p, v, st, act, nv);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_alpha(const cx<T>* rhat, const cx<T>* v, BicgSlot* st, const int* act, int n_act,
                int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_alpha<T><<<GRID(nv), NT, 0, s>>>(rhat, v, st, act, nv, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_update_s(const cx<T>* r, const cx<T>* v, cx<T>* sv, BicgSlot* st, const int* act,
                   int n_act, int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_update_s<T><<<GRID(nv), NT, 0, s>>>(r, v, sv, st, act, nv, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_omega(const cx<T>* t, const cx<T>* sv, BicgSlot* st, const int* act, int n_act,
                int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_omega<T><<<GRID(nv), NT, 0, s>>>(t, sv, st, act, nv, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void bicg_update_xr(cx<T>* x, cx<T>* r, const cx<T>* rhat, const cx<T>* p, const cx<T>* sv,
                    const cx<T>* t, BicgSlot* st, const int* act, int n_act, int64_t nv,
                    RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_update_xr<T><<<GRID(nv), NT, 0, s>>>(x, r, rhat, p, sv, t, st, act, nv, red);
    DDA_LAUNCH_CHECK();
}
template <typename T>
void residual(const cx<T>* b, const cx<T>* y, cx<T>* r, BicgSlot* st, const int* act, int n_act,
              int64_t nv, RedScratch red, hipStream_t s) {
    if (n_act == 0) return;
    k_residual<T><<<GRID(nv), NT, 0, s>>>(b, y, r, st, act, nv, red);
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
    dim3 grid(blocks_for(g.n_occ, red.max_blocks), nslots);
    k_loss_sums<<<grid, NT, 0, s>>>(einc, p, y, w, occ_lin, g, d, kv, r0, n_traj, rhs0, out, red);
    DDA_LAUNCH_CHECK();
}

#define DDA_INST(T)                                                                              \
    template void bicg_norm_b<T>(const cx<T>*, BicgSlot*, const int*, int, int64_t, double,      \
                                 RedScratch, hipStream_t);                                       \
    template void bicg_reset<T>(const cx<T>*, cx<T>*, cx<T>*, cx<T>*, BicgSlot*, const int*, int, \
                                int64_t, RedScratch, hipStream_t);                               \
    template void bicg_update_p<T>(const cx<T>*, cx<T>*, const cx<T>*, BicgSlot*, const int*,    \
                                   int, int64_t, hipStream_t);                                   \
    template void bicg_alpha<T>(const cx<T>*, const cx<T>*, BicgSlot*, const int*, int, int64_t, \
                                RedScratch, hipStream_t);                                        \
    template void bicg_update_s<T>(const cx<T>*, const cx<T>*, cx<T>*, BicgSlot*, const int*,    \
                                   int, int64_t, RedScratch, hipStream_t);                       \
    template void bicg_omega<T>(const cx<T>*, const cx<T>*, BicgSlot*, const int*, int, int64_t, \
                                RedScratch, hipStream_t);                                        \
    template void bicg_update_xr<T>(cx<T>*, cx<T>*, const cx<T>*, const cx<T>*, const cx<T>*,    \
                                    const cx<T>*, BicgSlot*, const int*, int, int64_t,           \
                                    RedScratch, hipStream_t);                                    \
    template void residual<T>(const cx<T>*, const cx<T>*, cx<T>*, BicgSlot*, const int*, int,    \
                              int64_t, RedScratch, hipStream_t);
DDA_INST(double)
DDA_INST(float)

}  // namespace dda

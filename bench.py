"""Benchmark: EELS spectrum points/s of the DDA EELS/CL path on one MI355X.

A step is one whole spectrum of the nanorod workload (capped rod 20 x 20 x 80
nm on 96 x 24 x 24 dipoles, 39,464 dipoles; Drude permittivity; host 1.45;
beta 0.55; 128 loss energies over 1-3 eV): the electron field at every dipole,
the interaction spectra D(k) of all 128 energies (rebuilt every step), the
batched Krylov solves to a relative residual of 1e-10 and the loss/CL
reductions.  Inputs are synthetic and resident in HBM before the timed region.

Printed as one JSON line, with the per-kernel roofline of the dominant FFT
kernel (HIP events on the library's stream), the FFT matvec bandwidth at the
64^3 lattice, single-solve latency percentiles, and the FP64 CPU oracle's
throughput on the same workload as a reported baseline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6  # MI355X dense FP64 matrix peak
KERNELS = ["unpack_xfft", "yfft", "zconv", "iyfft", "ixfft_pack", "yzconv", "xyfft", "ixyfft_pack"]
# the costliest kernel of the matvec chain: the fused yz kernel on lattices
# whose padded yz plane fits in LDS, the z pass otherwise (profiles/)
CONV_KERNELS = ["yzconv", "zconv"]


def kernel_bytes(name: str, nx, ny, nz, mx, my, mz, n_occ, c: int, nrhs: float = 1.0,
                 n_d: float = None) -> float:
    """Algorithmic HBM bytes of one launch of a matvec kernel over nrhs
    right-hand sides that use n_d distinct interaction spectra D (n_d = nrhs
    when every right-hand side has its own energy; a D shared by a batch is
    read once).  Complex size c; the index map is 4-byte ints.  The
    zero-padded rows the kernels never touch are not counted."""
    if n_d is None:
        n_d = nrhs
    N = nx * ny * nz
    row_x = 3 * nz * ny * mx            # x-transformed rows (y < ny, z < nz)
    full_y = 3 * nz * my * mx           # after the y pass
    if name == "unpack_xfft":
        return (3 * n_occ * c + 4 * N + row_x * c) * nrhs
    if name == "yfft":
        return (row_x + full_y) * c * nrhs
    if name == "zconv":
        # D is stored as its [0, M/2] corner per axis (even/odd symmetry)
        return 2 * full_y * c * nrhs + 6 * (mz // 2 + 1) * (my // 2 + 1) * (mx // 2 + 1) * c * n_d
    if name == "iyfft":
        return (full_y + row_x) * c * nrhs
    if name == "ixfft_pack":
        return (row_x * c + 4 * N + (3 + 1 + 3) * n_occ * c) * nrhs
    if name == "xyfft":  # the gather, x and y passes of one (component, z) plane
        return (3 * n_occ * c + 4 * N + full_y * c) * nrhs
    if name == "ixyfft_pack":
        return (full_y * c + 4 * N + (3 + 1 + 3) * n_occ * c) * nrhs
    if name == "yzconv":
        # T[kx][3][nz][ny] in and out, D as kx slabs of its [0, L/2]^2 corner
        return 2 * row_x * c * nrhs + 6 * (mx // 2 + 1) * (my // 2 + 1) * (mz // 2 + 1) * c * n_d
    raise KeyError(name)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ["fft_core.h", "quad_fft.h", "matvec.hip", "matvec_yz.hip", "matvec_xy.hip"]:
        with open(os.path.join(ROOT, "paper_2208_01348_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str, precision: str, rhs_per_launch: float):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary (bytes per
    right-hand side times the right-hand sides per launch), if the summary was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    with open(p) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash():
        return None
    try:
        return round(float(vals["hbm_bytes_per_rhs"]) * rhs_per_launch)
    except (KeyError, ValueError):
        return None


def cpu_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--solver", choices=["cocg", "bicgstab"], default="cocg")
    ap.add_argument("--n-energy", type=int, default=128)
    ap.add_argument("--check-every", type=int, default=48,
                    help="Krylov iterations per interval (device-side FP64 checks between); "
                         "a converged system waits for the next check idle, so longer "
                         "intervals cost no matvecs (12 ... 64 swept on the nanorod spectrum)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch the COCG kernels one by one instead of replaying captured "
                         "HIP graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the seeded serving stream to replay (0: skip)")
    ap.add_argument("--serve-window", type=float, default=75.0,
                    help="seconds the server runs on the replayed stream")
    ap.add_argument("--c4-energies", type=int, default=8,
                    help="energies of the impact-map workload (x 256 impacts; 0: skip); the "
                         "full configuration has 32")
    ap.add_argument("--c3-energies", type=int, default=64,
                    help="energies of the Cherenkov 64^3 workload (x 2 trajectories; 0: skip); "
                         "the full configuration has 64")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed steps of the plain FP64 nanorod spectrum (COCG and BiCGStab, "
                         "complex128 throughout) reported beside the headline; 0: skip")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (for scaling rocprofv3 "
                         "FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--latency-only", action="store_true",
                    help="only the c1 single-solve latency lines (FP64 BiCGStab and COCG)")
    ap.add_argument("--matvec64-only", action="store_true",
                    help="measure only the 64^3 FFT matvec (one JSON line) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve shards by "
              "energy across GPUs with no communication; only the one-GPU path exists.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2208_01348_amd.solver import DDASolver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.latency_only:
        log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
        print(json.dumps(measure_latency(torch, W, DDASolver, log)), flush=True)
        return
    if args.matvec64_only:
        log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
        if args.calibrate_copy:
            a = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
            del a
        print(json.dumps({"matvec_64cubed": measure_matvec64(torch, W, DDASolver, log)}),
              flush=True)
        return

    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    w = W.c2_nanorod_spectrum(args.n_energy)
    n = w.n_occ
    E = w.energies
    # inputs resident in HBM before the timed region
    eps = torch.from_numpy(np.repeat(w.eps_table()[:, None], n, axis=1)).to(dev)
    solver = DDASolver(w.mask, w.d, w.m_h, precision=args.precision, tol=w.tol, maxit=50000,
                       solver=args.solver, check_every=args.check_every,
                       use_graphs=not args.no_graphs)
    mx, my, mz = solver.grid
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    log(f"workload {w.name}: n_occ={n} grid={solver.grid} energies={E.size} "
        f"precision={args.precision} solver={args.solver}")

    def step():
        solver.drop_cache()  # interaction spectra are part of every step
        return solver.spectrum(E, w.beta, eps, w.r0)

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.3f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        P, info = step()
        log(f"step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = t1 - t0
    value = args.steps * E.size * w.n_traj / T
    iters = [x.iters for x in info]
    mvs = [x.matvecs for x in info]
    log(f"matvecs min/median/max {min(mvs)}/{int(np.median(mvs))}/{max(mvs)}")
    log(f"timed {args.steps} steps in {T:.3f} s -> {value:.2f} points/s; iterations "
        f"min/median/max {min(iters)}/{int(np.median(iters))}/{max(iters)}")
    statuses = sorted(set(x.status for x in info))

    # roofline of the dominant kernel: HIP events on the library's stream
    # around every launch of the convolution kernels, over one more step of the
    # same workload (with timing on the library launches kernel by kernel:
    # events recorded inside a replayed graph carry no timestamps).  In the
    # mixed path the launches mix FP32 (iterations) and FP64 (checks); the
    # algorithmic bytes use the FP32 size, which dominates.
    solver.set_timing(True, kernels=CONV_KERNELS)
    t2 = time.perf_counter()
    _, info_t = step()
    torch.cuda.synchronize()
    log(f"instrumented step: {time.perf_counter() - t2:.3f} s")
    c = 8 if args.precision == "mixed" else 16
    dom = max(CONV_KERNELS, key=lambda k: solver.kernel_time(k)[1])
    ms, launches, slots = solver.kernel_time(dom)
    # A launch covers every slot of the active list, but a system that has met
    # the tolerance waits idle for the next FP64 check and its blocks return at
    # once.  The right-hand sides a launch works on are counted from the
    # systems' matvec counts (each matvec passes the convolution kernel once).
    rhs = sum(x.matvecs for x in info_t) / max(launches, 1)
    per_launch = kernel_bytes(dom, w.nx, w.ny, w.nz, mx, my, mz, n, c, nrhs=rhs)  # one D each
    achieved = per_launch / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(dom, "c2", args.precision, rhs),
                "avg_launch_ms": round(ms, 5), "launches": launches,
                "timing": "HIP events per launch, one instrumented step after the timed ones",
                "rhs_per_launch": round(rhs, 2), "slots_per_launch": round(slots, 2),
                "bytes_per_launch": round(per_launch)}
    solver.set_timing(False)
    from paper_2208_01348_amd import _lib as L
    tuning = {"fp32": L.dda_tuning(solver.ctx, L.DDA_PREC_MIXED),
              "fp64": L.dda_tuning(solver.ctx, L.DDA_PREC_FP64)}
    log(f"autotuned tiles: {tuning}")

    extras = {}
    if args.fp64_steps > 0 and args.precision == "mixed":
        extras["c2_plain_fp64"] = measure_plain_fp64(torch, W, DDASolver, w, eps, P, info,
                                                     args.fp64_steps, args.check_every, log)
    if not args.no_extras:
        extras.update(measure_extras(torch, W, DDASolver, log))
        if args.serve_requests > 0:
            extras["serving_c5"] = measure_serving(torch, W, DDASolver, args.serve_requests, log,
                                                   window_s=args.serve_window)
        if args.c4_energies > 0:
            extras["impact_map_c4"] = measure_batch(torch, W, DDASolver, "c4",
                                                    args.c4_energies, log)
        if args.c3_energies > 0:
            extras["cherenkov_c3"] = measure_batch(torch, W, DDASolver, "c3",
                                                   args.c3_energies, log)
        extras["far_field_cl"] = measure_farfield(torch, W, DDASolver, log)
        extras["richardson_series"] = measure_series(torch, W, log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, [x.matvecs for x in info], log)

    out = {
        "metric": "EELS spectrum points/s + matvec HBM GB/s at 64^3; p50/p99 solve latency",
        "value": round(value, 3),
        "unit": "spectrum points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * T / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 matvec + f64 refinement" if args.precision == "mixed" else "c128",
        "data": "synthetic (Drude nanorod, seeded; no optical data or measured spectra)",
        "check_every": args.check_every,
        "graphs": not args.no_graphs,
        "config": {"workload": "c2 nanorod spectrum: capped rod 20x20x80 nm on 96x24x24 dipoles "
                               f"(n_occ={n}), host 1.45, beta 0.55, {E.size} energies over 1-3 eV, "
                               f"tol {w.tol}, LDR",
                   "solver": args.solver, "precision": args.precision, "fft_grid": [mx, my, mz],
                   "parallelism": "1 GPU, energies batched as right-hand sides"},
        "solve": {"iterations_min": min(iters), "iterations_median": int(np.median(iters)),
                  "iterations_max": max(iters), "iterations_total": int(sum(iters)),
                  "matvecs_total": int(sum(mvs)),
                  "max_rel_residual": max(x.rel_residual for x in info), "statuses": statuses},
        "roofline": roofline,
        "autotune": tuning,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def rel_err_per_point(P, R):
    """|P - R| per value relative to max(|R|, 1e-3 max of the point's four values)
    (the per-point reading of a relative error where a probability is near 0)."""
    P, R = np.asarray(P), np.asarray(R)
    scale = np.maximum(np.abs(R), 1e-3 * np.max(np.abs(R), axis=1, keepdims=True))
    return np.abs(P - R) / scale


def measure_plain_fp64(torch, W, DDASolver, w, eps, P_mixed, info_mixed, steps, check_every,
                       log):
    """The same nanorod spectrum through the plain FP64 path (complex128
    matvecs and vectors, no refinement), COCG, BiCGStab and QMR, timed like the
    headline; and the largest per-point difference between the mixed
    spectrum and the FP64 one.  Both meet the FP64 residual tolerance for
    every point; the FP64 path matches the FP64 CPU oracle to 1e-9 in the
    GPU parity tests."""
    out = {}
    P_ref = None
    for solver in ("cocg", "bicgstab", "qmr"):
        s = DDASolver(w.mask, w.d, w.m_h, precision="fp64", tol=w.tol, maxit=50000,
                      solver=solver, check_every=check_every if solver != "bicgstab" else 16)

        def step():
            s.drop_cache()
            return s.spectrum(w.energies, w.beta, eps, w.r0)

        step()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            P, info = step()
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        s.close()
        rate = steps * len(info) / T
        mvs = [i.matvecs for i in info]
        its = [i.iters for i in info]
        res = {"points_per_s": round(rate, 3), "steps": steps, "ms_per_step": round(1e3 * T / steps, 2),
               "matvecs_total": int(sum(mvs)), "matvecs_max": int(max(mvs)),
               "iterations_median": int(np.median(its)), "iterations_max": int(max(its)),
               "max_rel_residual": max(i.rel_residual for i in info),
               "all_converged": all(i.status == 0 for i in info)}
        if P_ref is None:
            P_ref = P
        else:
            e = rel_err_per_point(P, P_ref)
            res["max_rel_diff_vs_fp64_cocg"] = float(e.max())
        out[solver] = res
        log(f"plain FP64 {solver}: {rate:.2f} points/s ({T / steps:.3f} s per spectrum), "
            f"matvecs {sum(mvs)}")
    e = rel_err_per_point(P_mixed, P_ref)
    out["mixed_vs_fp64"] = {
        "max_rel_diff": float(e.max()),
        "max_rel_diff_per_quantity": {k: float(e[:, j].max()) for j, k in
                                      enumerate(["p_eels", "p_ext", "p_abs", "p_cl"])},
        "median_rel_diff_p_eels": float(np.median(e[:, 0])),
        "points": int(e.shape[0]),
        "max_rel_residual_mixed": max(i.rel_residual for i in info_mixed),
        "note": "per point: |P_mixed - P_fp64| / max(|P_fp64|, 1e-3 max of the point's four "
                "values); both solves end on an FP64 residual <= tol"}
    log(f"mixed vs FP64: max per-point relative difference {e.max():.2e}")
    return out


def measure_matvec64(torch, W, DDASolver, log):
    """FFT matvec GB/s on the 64^3 lattice: FP64 (five-pass chain) and FP32
    (the fused xy chain), one and eight right-hand sides, and 64 in FP32."""
    w3 = W.c3_cherenkov()
    n3 = w3.n_occ
    Em = float(w3.energies[len(w3.energies) // 2])
    eps3 = np.full(n3, w3.eps_table()[len(w3.energies) // 2])
    s3 = DDASolver(w3.mask, w3.d, w3.m_h)
    mx, my, mz = s3.grid
    N = w3.nx * w3.ny * w3.nz
    mv = {}
    for prec, dt, c in [("fp64", torch.complex128, 16), ("fp32", torch.complex64, 8)]:
        # the autotuner times its candidates on the first batch it sees
        for nrhs in ((8, 1, 64) if prec == "fp32" else (8, 1)):
            x = torch.randn((nrhs, 3, n3), dtype=dt, device="cuda")
            y = torch.empty_like(x)
            p = "fp64" if prec == "fp64" else "mixed"
            s3.matvec(Em, eps3, x, precision=p, out=y)
            torch.cuda.synchronize()
            reps = 20
            s3.set_timing(True)
            for _ in range(reps):
                s3.matvec(Em, eps3, x, precision=p, out=y)
            # device time of the kernel chain (HIP events per kernel)
            kt = {k: s3.kernel_time(k)[0] for k in KERNELS if s3.kernel_time(k)[1] > 0}
            dt_s = sum(kt.values()) * 1e-3
            s3.set_timing(False)
            per_launch = sum(kernel_bytes(k, w3.nx, w3.ny, w3.nz, mx, my, mz, n3, c, nrhs, 1)
                             for k in kt)
            d_red = 6 * (mz // 2 + 1) * (my // 2 + 1) * (mx // 2 + 1)
            # the chain that ran: the fused xy kernels stream the y-transformed
            # grid (12N on this cube) once each way, the five-pass chain also
            # the x-transformed rows (6N) twice each way
            xy = "xyfft" in kt
            per_n = 48 if xy else 72
            model = ((per_n * N + 10 * n3) * nrhs + d_red) * c  # one D shared by the batch
            five = ((72 * N + 10 * n3) * nrhs + d_red) * c
            mv[f"{prec}_nrhs{nrhs}"] = {
                "chain": "xyfft, zconv, ixyfft_pack" if xy else "five-pass",
                "ms": round(dt_s * 1e3, 4),
                "model_bytes_per_matvec": int(model),
                "GBps_model": round(model / dt_s / 1e9, 1),
                # the five-pass chain's bytes over this time: the rate that chain
                # would need to match it (not a measured bandwidth)
                "five_pass_bytes_over_time_GBps": round(five / dt_s / 1e9, 1),
                "GBps_kernels": round(per_launch / dt_s / 1e9, 1),
                "frac_of_hbm_peak": round(model / dt_s / 1e9 / HBM_PEAK_GBS, 4),
                "kernels_GBps": {k: round(kernel_bytes(k, w3.nx, w3.ny, w3.nz, mx, my, mz, n3, c,
                                                       nrhs, 1) / (kt[k] * 1e-3) / 1e9, 1)
                                 for k in kt},
                "kernels_ms": {k: round(kt[k], 4) for k in kt}}
            log(f"matvec 64^3 {prec} nrhs={nrhs}: {dt_s * 1e3:.3f} ms, "
                f"{model / dt_s / 1e9:.0f} GB/s (model)")
    s3.close()
    return mv


def measure_extras(torch, W, DDASolver, log):
    """FFT matvec GB/s on the 64^3 lattice and single-solve latency (c1)."""
    res = {"matvec_64cubed": measure_matvec64(torch, W, DDASolver, log)}
    res.update(measure_latency(torch, W, DDASolver, log))
    return res


def measure_latency(torch, W, DDASolver, log):
    """Single-solve latency percentiles on c1 (16^3 sphere, one energy, FP64
    to 1e-10): BiCGStab as specified, and COCG."""
    res = {}
    # single-solve latency, c1 (FP64 BiCGStab to 1e-10), 10 solves
    w1 = W.c1_single_solve()
    s1 = DDASolver(w1.mask, w1.d, w1.m_h, tol=w1.tol, solver="bicgstab")
    eps1 = w1.eps_dipoles(0)[None, :]
    lat = []
    for i in range(11):
        s1.drop_cache()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info1 = s1.spectrum(w1.energies, w1.beta, eps1, w1.r0)
        torch.cuda.synchronize()
        if i:
            lat.append(time.perf_counter() - t)
    s1.close()
    it = info1[0].iters
    res["solve_latency_c1_ms"] = {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                                  "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                                  "solves": len(lat), "precision": "fp64", "solver": "bicgstab",
                                  "iterations": it,
                                  "us_per_iteration": round(1e6 * float(np.median(lat)) / it, 2)}
    log(f"c1 latency p50 {res['solve_latency_c1_ms']['p50']} ms")
    # the same solve with FP64 COCG (device-driven intervals, captured graphs)
    s1 = DDASolver(w1.mask, w1.d, w1.m_h, tol=w1.tol, solver="cocg")
    lat = []
    for i in range(11):
        s1.drop_cache()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info1 = s1.spectrum(w1.energies, w1.beta, eps1, w1.r0)
        torch.cuda.synchronize()
        if i:
            lat.append(time.perf_counter() - t)
    s1.close()
    it = info1[0].iters
    res["solve_latency_c1_cocg_ms"] = {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                                       "solves": len(lat), "precision": "fp64", "solver": "cocg",
                                       "iterations": it,
                                       "us_per_iteration": round(1e6 * float(np.median(lat)) / it,
                                                                 2)}
    log(f"c1 COCG latency p50 {res['solve_latency_c1_cocg_ms']['p50']} ms")
    return res


def measure_serving(torch, W, DDASolver, n_req, log, window_s=75.0, plain_req=12,
                    plain_window_s=45.0, max_inflight=16):
    """The seeded Poisson stream (mean 200 requests/s; sphere / capped rod /
    ellipsoid on 24-96 cells per side; host 1-2; beta 0.4-0.8; 8-64
    energies; tol 1e-8): n_req requests submitted at their arrival times to
    the continuous-batching server (mixed precision, one engine per box of
    cells shared by every lattice and request in it, at most max_inflight
    requests in the engines, the rest first come first served), served for
    window_s seconds from the first arrival with the queue depth sampled;
    then the first plain_req requests through the plain FP64 path (one
    dda_solve per request, COCG, in arrival order on one stream) for at most
    plain_window_s.  The stream arrives far faster than one GPU serves it, so
    the window measures the sustained rate and the backlog; the arrival rate
    one GPU sustains with bounded latency is the sustained points/s over the
    stream's mean points per request."""
    from paper_2208_01348_amd.serving import Server, replay_window, requests_from_stream
    reqs = requests_from_stream(W.c5_request_stream(n_requests=n_req))
    points = sum(len(r.energies) for r in reqs)
    mean_pts = points / len(reqs)
    srv = Server(hbm_budget_bytes=180 << 30, slots=64, precision="mixed", tol=1e-8,
                 check_every=8, max_inflight=max_inflight)
    t = time.perf_counter()
    rep = replay_window(srv, reqs, window_s, progress=lambda snap: log(f"  serving {snap}"))
    lat = np.array(sorted(rep.latency.values())) if rep.latency else np.array([np.nan])
    ok = all(i[3] == 0 for c in rep.completions for i in c.info)
    rate = rep.systems_solved / rep.window_s
    # the second half of the window, once every request has arrived and the
    # engines are busy: points solved in it per second
    mid = min(rep.samples, key=lambda smp: abs(smp["t"] - rep.window_s / 2))
    rate_late = (rep.systems_solved - mid["systems_solved"]) / max(rep.window_s - mid["t"], 1e-9)
    step = max(1, len(rep.samples) // 16)
    served = {
        "requests_arrived": int(sum(1 for v in rep.waited.values() if v > 0) + len(rep.completions)),
        "requests_completed": len(rep.completions), "points_completed": rep.points_done,
        "points_solved": rep.systems_solved,
        "window_s": round(rep.window_s, 2), "points_per_s": round(rate, 2),
        "points_per_s_second_half": round(rate_late, 2),
        "p50_s": round(float(np.percentile(lat, 50)), 3),
        "p99_s": round(float(np.percentile(lat, 99)), 3),
        "max_wait_unfinished_s": round(max(rep.waited.values()), 2) if rep.waited else 0.0,
        "all_converged": bool(ok),
        "lattices_completed": len(set(c.lattice for c in rep.completions)),
        "engines_used": len(set(c.engine for c in rep.completions)),
        "queue_depth": [{k: v for k, v in smp.items()} for smp in rep.samples[::step]],
        "sustainable_requests_per_s": round(rate / mean_pts, 3),
        "max_inflight_requests": max_inflight}
    log(f"serving: {len(rep.completions)}/{n_req} requests ({rep.systems_solved} points solved) in "
        f"{rep.window_s:.1f} s, {rate:.1f} points/s; p50 {served['p50_s']} s p99 "
        f"{served['p99_s']} s of the completed; backlog {len(rep.waited)} requests "
        f"({time.perf_counter() - t:.1f} s wall)")
    # plain FP64: the first plain_req requests one after another in arrival order
    first = sorted(reqs, key=lambda r: r.arrival)[:plain_req]
    t0 = time.perf_counter()
    lat64, pts64 = [], 0
    for r in first:
        if time.perf_counter() - t0 > plain_window_s:
            break
        wait = t0 + r.arrival - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        s = DDASolver(r.mask, r.d, r.m_h, solver="cocg", precision="fp64", tol=1e-8,
                      maxit=50000, check_every=8)
        n = s.n_occ
        s.spectrum(r.energies, r.beta, np.repeat(r.eps[:, None], n, axis=1), r.r0.reshape(1, 3))
        s.close()
        lat64.append(time.perf_counter() - (t0 + r.arrival))
        pts64 += len(r.energies)
    span64 = time.perf_counter() - t0
    L64 = np.array(lat64)
    plain = {"requests_completed": len(lat64), "points_completed": pts64,
             "p50_s": round(float(np.percentile(L64, 50)), 3),
             "p99_s": round(float(np.percentile(L64, 99)), 3),
             "points_per_s": round(pts64 / span64, 2), "seconds": round(span64, 2)}
    log(f"plain FP64 per request: {len(lat64)} requests, {pts64} points in {span64:.1f} s")
    # the served path on the same first requests alone, for a like-for-like rate
    srv2 = Server(hbm_budget_bytes=180 << 30, slots=64, precision="mixed", tol=1e-8,
                  check_every=8)
    rep2 = replay_window(srv2, first[:len(lat64)], plain_window_s)
    L2 = np.array(sorted(rep2.latency.values())) if rep2.latency else np.array([np.nan])
    served_first = {"requests_completed": len(rep2.completions), "points_completed": rep2.points_done,
                    "p50_s": round(float(np.percentile(L2, 50)), 3),
                    "p99_s": round(float(np.percentile(L2, 99)), 3),
                    "points_per_s": round(rep2.points_done / rep2.window_s, 2),
                    "seconds": round(rep2.window_s, 2)}
    log(f"served, same {len(lat64)} requests: {rep2.window_s:.1f} s")
    return {"requests": n_req, "points": points, "arrival_rate_per_s": 200.0,
            "stream_seconds": round(max(r.arrival for r in reqs), 3),
            "mean_points_per_request": round(mean_pts, 2),
            "served_mixed": served, "plain_fp64_first_requests": plain,
            "served_mixed_first_requests": served_first,
            "note": "seeded stream (default_rng(5)); tol 1e-8; latencies of completed requests "
                    "only (the unfinished ones had waited at least max_wait_unfinished_s)"}


def measure_batch(torch, W, DDASolver, which, n_energy, log):
    """Points/s of a multi-right-hand-side batch: the impact map (48^3
    ellipsoid, 16 x 16 impacts per energy sharing one D) or the Cherenkov
    sphere (64^3, absorbing host 2 + 0.01i, two trajectories), mixed COCG."""
    w = W.c4_impact_map(n_energy=n_energy) if which == "c4" else W.c3_cherenkov(n_energy=n_energy)
    n = w.n_occ
    eps = np.repeat(w.eps_table()[:, None], n, axis=1)
    s = DDASolver(w.mask, w.d, w.m_h, precision="mixed", tol=w.tol, maxit=50000, solver="cocg",
                  check_every=16)
    s.spectrum(w.energies[:1], w.beta, eps[:1], w.r0[:1])  # warm-up (builds, first launches)
    s.drop_cache()
    torch.cuda.synchronize()
    t = time.perf_counter()
    P, info = s.spectrum(w.energies, w.beta, eps, w.r0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    from paper_2208_01348_amd import _lib as L
    tuning = {"fp32": L.dda_tuning(s.ctx, L.DDA_PREC_MIXED),
              "fp64": L.dda_tuning(s.ctx, L.DDA_PREC_FP64)}
    s.close()
    pts = len(info)
    its = [i.iters for i in info]
    log(f"{which}: {pts} points in {dt:.2f} s ({pts / dt:.1f} points/s), iterations "
        f"median {int(np.median(its))} max {max(its)}")
    full = (32 if which == "c4" else 64) * w.r0.shape[0]
    return {"points": pts, "points_full_config": full,
            "measured_fraction_of_full_config": round(pts / full, 4),
            "projected_full_config_s": None if pts == full else round(full * dt / pts, 1),
            "seconds": round(dt, 3), "points_per_s": round(pts / dt, 2),
            "n_occ": n, "fft_grid": list(s.grid), "iterations_median": int(np.median(its)),
            "iterations_max": max(its), "tol": w.tol, "precision": "mixed",
            "all_converged": all(i.status == 0 for i in info), "autotune": tuning}


def _sphere_directions(n_theta, n_phi):
    """Gauss-Legendre in cos(theta) x equispaced phi: unit directions and
    solid-angle weights (sum 4 pi)."""
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - x * x)
    d = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(x, np.ones(n_phi))], axis=-1).reshape(-1, 3)
    return d, np.outer(wx, np.full(n_phi, 2.0 * np.pi / n_phi)).reshape(-1)


def measure_farfield(torch, W, DDASolver, log):
    """CL over 2,048 directions on the FP64 matrix cores: the impact-map
    lattice (48^3 ellipsoid) with its 256 trajectories at one energy (one
    product of 2,048 x n_occ phases by n_occ x 768 moments), and the nanorod
    spectrum (128 energies x 1 trajectory).  Seeded random moments stand in
    for solutions (the arithmetic does not depend on their values)."""
    out = {}
    dirs, wts = _sphere_directions(32, 64)
    for name, w, E, nt in [("impact_map_c4", W.c4_impact_map(n_energy=1), None, 256),
                           ("spectrum_c2", W.c2_nanorod_spectrum(), None, 1)]:
        n = w.n_occ
        energies = w.energies[:1] if nt > 1 else w.energies
        nrhs = len(energies) * nt
        g = torch.Generator(device="cuda").manual_seed(5)
        p = torch.randn((nrhs, 3, n), dtype=torch.complex128, device="cuda", generator=g)
        s = DDASolver(w.mask, w.d, w.m_h)
        s.cl_directions(energies, w.beta, nt, p, dirs[:64], wts[:64], want_dp=False)  # warm-up
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            s.cl_directions(energies, w.beta, nt, p, dirs, wts, want_dp=False)
            times.append(time.perf_counter() - t)
        s.close()
        dt = min(times)
        flops = 8.0 * dirs.shape[0] * n * 3 * nrhs
        tf = flops / dt / 1e12
        log(f"far field {name}: {nrhs} rhs x {dirs.shape[0]} directions in {dt * 1e3:.2f} ms, "
            f"{tf:.1f} TFLOP/s FP64 matrix ({tf / FP64_MFMA_PEAK_TFS:.1%} of peak)")
        out[name] = {"rhs": nrhs, "directions": int(dirs.shape[0]), "n_occ": n,
                     "ms": round(dt * 1e3, 3), "tflops": round(tf, 2),
                     "frac_of_fp64_matrix_peak": round(tf / FP64_MFMA_PEAK_TFS, 4),
                     "note": "whole call: phase tables, matrix-core product, |A_perp|^2 and "
                             "the weighted sum; 8 flops per complex multiply-add"}
    return out


def measure_series(torch, W, log):
    """Richardson series (section 3.2) at a reduced scale: a sphere of radius
    10 nm on n_x = 48, 40, 34, 28, 24 (the ratios of the paper's 128 ... 64),
    4 energies, one trajectory 4 nm outside, mixed COCG tol 1e-8."""
    from paper_2208_01348_amd.series import lattice_series
    n_list = [48, 40, 34, 28, 24]
    E = np.linspace(2.0, 3.5, 4)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ds, P, ext, ci, infos = lattice_series(lambda n, d: W.sphere_mask(n, d, 10.0), 20.0, n_list,
                                           1.45, 0.55, E, lambda e: W.drude_eps(e),
                                           np.array([[14.0, 0.0, 0.0]]), tol=1e-8)
    dt = time.perf_counter() - t
    pts = sum(len(i) for i in infos)
    log(f"series: {len(n_list)} lattices x {len(E)} energies in {dt:.2f} s; extrapolated "
        f"P_EELS {ext[:, 0].round(8).tolist()} +- {ci[:, 0].round(8).tolist()}")
    return {"lattices": n_list, "energies": E.tolist(), "seconds": round(dt, 3),
            "points": pts, "p_eels_extrapolated": ext[:, 0].tolist(),
            "p_eels_ci95": ci[:, 0].tolist(), "p_eels_finest": P[0, :, 0].tolist(),
            "all_converged": all(i.status == 0 for info in infos for i in info)}


def cpu_baseline(w, gpu_matvecs, log):
    """The FP64 oracle (dense on-the-fly matvec, OpenMP) on the same spectrum,
    on a bounded sample: two dense matvecs at full size are timed, and the
    spectrum time is extrapolated with the matvec counts the GPU needed
    (plus the loss reduction's one per point)."""
    from oracle import cdense
    from oracle.dda import system
    e_mid = len(w.energies) // 2
    c, alpha, k, _ = system(w.mask, w.d, np.full(w.n_occ, w.eps_table()[e_mid]), w.m_h,
                            float(w.energies[e_mid]))
    x = np.random.default_rng(0).standard_normal((w.n_occ, 3)) + 0j
    reps = 2
    t = time.perf_counter()
    for _ in range(reps):
        cdense.matvec(c, alpha, k, x)
    t_mv = (time.perf_counter() - t) / reps
    total_matvecs = sum(gpu_matvecs) + len(gpu_matvecs)  # + the G_off p of the losses
    t_spec = total_matvecs * t_mv
    log(f"oracle dense matvec at full size: {t_mv:.2f} s; spectrum extrapolated to {t_spec:.0f} s")
    return {"value": round(len(gpu_matvecs) / t_spec, 6), "unit": "spectrum points/s",
            "cores": cdense.num_threads(), "kind": "oracle",
            "sample": f"{reps} dense FP64 matvecs at full size (n_occ={w.n_occ}), "
                      f"{t_mv:.2f} s each, extrapolated with the GPU's iteration counts "
                      f"({total_matvecs} matvecs for the {len(gpu_matvecs)}-point spectrum)"}


if __name__ == "__main__":
    main()

/*
 * libdda -- discrete-dipole-approximation solve for fast-electron EELS and
 * cathodoluminescence of a particle in an arbitrary (possibly absorbing,
 * possibly Cherenkov) host medium, on AMD Instinct MI355X (gfx950).
 *
 * Method: Kichigin & Yurkin, "Simulating electron energy-loss spectroscopy
 * and cathodoluminescence for particles in arbitrary host medium using the
 * discrete dipole approximation" (arXiv 2208.01348).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: lengths in nm, loss energies in eV, electron speed as beta = v/c,
 * probabilities per unit loss energy in 1/eV (section 2.5, eq. 37).
 *
 * Lattice: nx x ny x nz cubic cells of size d, centred on the origin; cell
 * (i, j, l) has its centre at d*(i - nx/2 + 1/2, j - ny/2 + 1/2, l - nz/2 + 1/2).
 * The mask is uint8 [nz][ny][nx] (x fastest); a non-zero entry marks an
 * occupied cell, i.e. a dipole.  Occupied cells are numbered 0..n_occ-1 in
 * increasing linear index l*ny*nx + j*nx + i; every per-dipole array follows
 * that order.
 *
 * Electron: point charge moving along +z with speed beta*c through the point
 * r0 = (x0, y0, z0) (eqs. 20-21).  A trajectory is given as 3 doubles (nm).
 *
 * Host: refractive index m_h = mh_re + i mh_im with 0 <= arg m_h < pi/2
 * (section 2.1); k = m_h * E / (hbar c) is the host wavenumber.
 *
 * Device vectors ("field" layout): complex128 (two doubles, re then im),
 * [nrhs][3][n_occ] -- right-hand side, then Cartesian component, then dipole.
 * Right-hand sides of a batch are numbered rhs = e * n_traj + t for energy e
 * and trajectory t.  Device pointers are borrowed, never freed by the
 * library, and used in stream order on the stream given to dda_setup: the
 * caller keeps them alive until that stream has passed the call.  Host
 * arrays are read before the call returns.
 *
 * Unknowns: dda_solve returns p_hat with A p_hat = e_hat (below), the dipole
 * moments in the normalisation p_hat = p_SI / (4 pi eps0 m_h^2 C), C the
 * amplitude of eq. (25).  e_hat is the dimensionless shape of eq. (25).
 *
 * Errors: every call returns a dda_status.  Nothing throws across the ABI.
 * On an error the outputs are left untouched, except DDA_ENOCONV and
 * DDA_EBREAKDOWN, which leave the best iterate in p and fill `info`.
 * dda_last_error() then describes the failure (thread-local, valid until the
 * next call on the same thread).
 *
 * Threads: a context must not be used by two threads at once.
 */
#ifndef DDA_H
#define DDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dda_ctx dda_ctx;

typedef enum {
    DDA_OK = 0,
    DDA_EINVAL = -1,      /* bad argument (sizes, NaN, non-passive host, ...)  */
    DDA_ENOMEM = -2,      /* device allocation failed                          */
    DDA_EDEVICE = -3,     /* HIP runtime error                                  */
    DDA_ENOCONV = -4,     /* iteration limit reached before the tolerance       */
    DDA_EBREAKDOWN = -5,  /* Krylov breakdown that a restart could not cure     */
    DDA_ESINGULAR = -6    /* beta_h = 1 (eq. 24) or a trajectory through a dipole */
} dda_status;

enum { DDA_POL_LDR = 0, DDA_POL_CM = 1, DDA_POL_RR = 2 };
enum { DDA_SOLVER_BICGSTAB = 0, DDA_SOLVER_COCG = 1, DDA_SOLVER_QMR = 2 };
enum { DDA_PREC_FP64 = 0, DDA_PREC_MIXED = 1 };
enum { DDA_INT_POINT = 0, DDA_INT_IGT = 1 };

typedef struct {
    int polarizability;   /* DDA_POL_*; lattice dispersion relation by default      */
    int solver;           /* DDA_SOLVER_BICGSTAB (two matvecs per iteration),
                             DDA_SOLVER_COCG: conjugate-orthogonal CG for the
                             complex-symmetric DDA matrix (reciprocity, section
                             2.4), one matvec per iteration, or
                             DDA_SOLVER_QMR: QMR for complex-symmetric matrices
                             (the solver family of section S5; Lanczos of the
                             bilinear form with unit-norm vectors, quasi-minimal
                             residual by Givens rotations), one matvec per
                             iteration; it restarts from the FP64 residual when
                             its residual bound sqrt(n+1)|tau| meets tol but the
                             FP64 residual does not (in MIXED precision, the
                             FP32 cycles are refined this way)              */
    int precision;        /* DDA_PREC_FP64: complex128 throughout.
                             DDA_PREC_MIXED: complex64 FFT matvecs and Krylov vectors
                             with FP64 refinement: BiCGStab restarts from the FP64
                             residual; COCG keeps iterating and periodically
                             replaces its residual by the FP64 one while the
                             solution accumulates in FP64 (reliable updates)       */
    double tol;           /* stopping threshold on ||e - A p|| / ||e|| (unscaled)    */
    int maxit;            /* iteration limit (matvec pairs for BiCGStab)              */
    int check_every;      /* BiCGStab: the host polls convergence every this many
                             iterations.  COCG: iterations per interval; each
                             interval starts with the FP64 residual check of the
                             right-hand sides that asked for one, and the host
                             reads the solver states two intervals behind without
                             stalling the stream                                    */
    int use_graphs;       /* COCG on a non-default stream: send each interval as a
                             captured HIP graph (replayed while the set of active
                             right-hand sides keeps its size); 0 launches kernels
                             one by one, and so does a context whose kernel timing
                             is on (dda_set_timing).  Results are identical.       */
    int interaction;      /* DDA_INT_POINT: the point-dipole Green's tensor G(R)
                             between every pair of dipoles.  DDA_INT_IGT: the
                             interaction the paper recommends (section S5),
                             read as the Green's tensor of eq. (5) integrated
                             over the source cell (the VIE of eqs. 4 and 8 with
                             the polarization constant in each cell):
                             for |R| <= 3 d the cell average
                             d^-3 int_cube G(R + s) d^3 s (24-point Gauss-
                             Legendre rule per axis, FP64), beyond it G(R).
                             The self term stays with the polarizability.     */
} dda_options;

typedef struct {
    int iters;            /* Krylov iterations taken (inner ones for MIXED)           */
    int matvecs;          /* FFT matvecs applied to this right-hand side              */
    double rel_residual;  /* final true ||e - A p|| / ||e|| in FP64                   */
    int status;           /* dda_status of this right-hand side                        */
} dda_solve_info;

typedef struct {
    double p_eels;  /* particle-induced loss probability, eqs. (32), (34), (37)   */
    double p_ext;   /* extinction probability, eqs. (17), (48)                    */
    double p_abs;   /* absorption probability, eq. (18) in discrete form          */
    double p_cl;    /* cathodoluminescence probability, eq. (42)                  */
} dda_result;

/* Default options: LDR, BiCGStab, FP64, tol 1e-10, maxit 100000, check 16. */
void dda_default_options(dda_options* opt);

/* Relativistic v/c of an electron of the given kinetic energy (keV). */
double dda_beta_from_keV(double kinetic_keV);

/*
 * Free-space loss of the electron per unit path length and energy, eq. (29)
 * through eq. (36) (Frank-Tamm): d Gamma_0/dz = alpha_fs (1 - 1/beta_h^2) /
 * (hbar c) in eV^-1 nm^-1 when beta_h = beta m_h > 1, else 0.  Host only.
 * Errors: DDA_EINVAL for beta outside (0, 1), Re m_h <= 0, non-finite input,
 * or an absorbing host (Im m_h != 0), where W_0 is undefined (section 2.3).
 */
int dda_free_space_loss(double beta, double mh_re, double mh_im, double* dgamma_dz);

/*
 * Richardson extrapolation to zero dipole size (section 3.2): a weighted
 * least-squares quadratic a + b d + c d^2 through (d_nm[i], value[i]), i < n,
 * the errors of the points taken to scale as d^3 (weights d^-6).  at_zero =
 * a; ci95 (may be NULL) = twice the standard error of a, the residual
 * variance estimated from the n - 3 degrees of freedom (NaN for n = 3).  Host
 * only.  Errors: DDA_EINVAL for n < 3, d <= 0, non-finite values, or sizes
 * that do not determine a quadratic (fewer than three distinct).
 */
int dda_richardson(const double* d_nm, const double* value, int n, double* at_zero,
                   double* ci95);

/*
 * Total particle-related CL probability, eq. (41): out[i] = P_EELS - P_ext +
 * P_CL of res[i] (the cross sections C_enh - C_ext + C_sca share the
 * prefactor of eqs. 37, 42, 48); equal to P_CL when beta_h < 1.  Host only;
 * res and out are host arrays of n.  Errors: DDA_EINVAL for bad arguments or
 * an absorbing host (Im m_h != 0), where the far-field powers it rests on are
 * not defined (section 2.6).
 */
int dda_cl_total(const dda_result* res, int n, double mh_im, double* out);

/*
 * Spectrum convolved with a Gaussian point-spread function of unit area and
 * full width at half maximum fwhm_eV (the instrumental broadening applied to
 * measured spectra, section 3.4): out_i = sum_j p_j g(E_i - E_j) dE on a
 * uniform energy grid, the spectrum taken as zero outside the grid.  Host
 * arrays of n; out may alias p.  Errors: DDA_EINVAL for n < 1, fwhm <= 0, or
 * energies that are not an increasing uniform grid.
 */
int dda_psf_gauss(const double* energy_eV, const double* p, int n, double fwhm_eV,
                  double* out);

/*
 * Builds a context for one lattice and host medium.  Copies the mask, builds
 * the index maps on the host and uploads them.  `hip_stream` is a hipStream_t
 * (NULL = the default stream) on which every later call is ordered.
 * Errors: DDA_EINVAL for sizes < 1, d <= 0, a lattice side above 256, a
 * non-passive or non-finite m_h, bad options; DDA_ENOMEM / DDA_EDEVICE.
 * An empty mask is allowed (n_occ = 0: every later call is a no-op).
 */
int dda_setup(const uint8_t* mask, int nx, int ny, int nz, double d_nm,
              double mh_re, double mh_im, const dda_options* opt,
              void* hip_stream, dda_ctx** out);

/*
 * A non-blocking HIP stream of default priority, for a context of its own:
 * graph capture on it (see use_graphs) cannot collide with work other
 * threads put on the legacy default stream.  Destroy it after the contexts
 * that use it.
 */
int dda_stream_create(void** stream);
int dda_stream_destroy(void* stream);

/*
 * Changes the host index of a context (passive: Re m_h > 0, Im m_h >= 0).
 * Later calls use it; the cached interaction spectra stay valid (they are
 * keyed by the wavenumber m_h omega/c), and systems already submitted to the
 * engine keep the host index they were submitted with.
 */
int dda_set_host(dda_ctx* ctx, double mh_re, double mh_im);

/* Number of occupied cells (dipoles). */
int dda_n_occ(const dda_ctx* ctx, int64_t* n_occ);

/* FFT grid of the block-Toeplitz embedding: the smallest 2^a 3^b sizes
 * (b <= 1) that are >= 2n - 1 per axis. */
int dda_grid_dims(const dda_ctx* ctx, int* mx, int* my, int* mz);

/*
 * Incident field shape of the electron (eq. 25) at every dipole, for
 * n_energy energies x n_traj trajectories:
 *   e_hat = exp(i omega (z - z0)/v) ((x-x0)/b K1(k_t b), (y-y0)/b K1(k_t b),
 *                                    -(i/gamma_h) K0(k_t b)),
 *   k_t = omega/(gamma_h v), gamma_h on the first-quadrant branch of eq. (24).
 * energy_eV [n_energy] host; r0_nm [n_traj][3] host; einc_dev complex128
 * [n_energy*n_traj][3][n_occ], caller-owned.  FP64 throughout.
 * Errors: DDA_ESINGULAR if |beta_h^2 - 1| < 1e-12 or a trajectory passes
 * within 1e-9 d of a dipole centre (eq. 25 is singular at b = 0);
 * DDA_EINVAL for beta outside (0, 1) or non-positive energies.
 */
int dda_einc_electron(dda_ctx* ctx, int n_energy, const double* energy_eV, double beta,
                      const double* r0_nm, int n_traj, void* einc_dev);

/*
 * dda_einc_electron for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and result, bit for bit: the energies
 * and trajectory points are staged in a device array the library holds on
 * every GPU it runs on (288 KiB, set up once per device by dda_setup, kept
 * until the process ends) instead of a buffer of the context, and the call
 * makes no device allocation, free or allocating library call.
 * Limits: n_energy <= DDA_EINC_NOALLOC_MAX_ENERGIES and n_traj <=
 * DDA_EINC_NOALLOC_MAX_TRAJ per call, else DDA_EINVAL.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (from several threads) race on it and must be serialised by the caller.
 * Like dda_einc_electron it returns after the context's stream has passed the
 * call.
 */
#define DDA_EINC_NOALLOC_MAX_ENERGIES 4096
#define DDA_EINC_NOALLOC_MAX_TRAJ 4096
int dda_einc_electron_noalloc(dda_ctx* ctx, int n_energy, const double* energy_eV, double beta,
                              const double* r0_nm, int n_traj, void* einc_dev);

/*
 * Solves A p_hat = e_hat for every right-hand side of a batch:
 *   (A p)_i = p_i / alpha_i - sum_{j != i} G(r_i - r_j) p_j,
 *   G(R) = (k^2 I + grad grad) exp(ikR)/R (eq. 5 times 4 pi k^2),
 * with the matvec done as a zero-padded 3D FFT convolution (block-Toeplitz
 * embedding) and alpha_i from m_i^2 = eps_i / m_h^2 (eq. 2) by the chosen
 * polarizability.  eps_dipole [n_energy][n_occ][2]: absolute particle
 * permittivity per dipole per energy, in host memory (copied in stream order)
 * or device memory (read in place; the runtime's pointer attributes decide).  einc_dev as written by
 * dda_einc_electron; p_dev complex128 [n_energy*n_traj][3][n_occ] out;
 * info [n_energy*n_traj] host out (may be NULL).
 * Returns DDA_OK when every right-hand side met the tolerance, else the
 * first failing status (per-RHS statuses are in info).
 */
int dda_solve(dda_ctx* ctx, int n_energy, const double* energy_eV, const double* eps_dipole,
              const void* einc_dev, int n_traj, void* p_dev, dda_solve_info* info);

/*
 * Loss and emission probabilities for every right-hand side (FP64 sums):
 *   P_EELS = -Pi Im[ sum_i g_i . p_i / (m_h gamma_h)^2 ],  g the auxiliary
 *            field of the conjugate source, eq. (34), built on the fly;
 *   P_ext  =  Pi Im[ m_h^2 sum_i conj(e_i) . p_i ] / (|m_h|^4 |gamma_h|^2);
 *   P_abs  =  Pi/(|m_h|^4|gamma_h|^2) sum_i w_i |p_i|^2, one formula for every host:
 *             w_i = 4 pi Im(m_h^2 m_i^2)/(|m_i^2 - 1|^2 d^3)      (eq. 18 with the
 *                   cell field of eq. 7, E_i = 4 pi p_i/((m_i^2 - 1) d^3))
 *                 + Im(m_h^2 conj(1/alpha_i - 1/alpha_CM,i))  (the polarizability's
 *                   change to the exciting field's work)
 *                 - Re(m_h^2) (2/3) Re(k)^3                   (self-radiated part);
 *             continuous in m_h; in a real host m_h^2 [-Im(1/alpha_i) - 2k^3/3], so
 *             that P_ext = P_abs + P_CL exactly there;
 *   P_CL   =  Pi Re(m_h^2)/(|m_h|^4|gamma_h|^2) [Im(p^H G_off p) + 2 Re(k)^3 ||p||^2/3]
 *             (eq. 42; nominal in an absorbing host),
 *   Pi = 4 alpha_fs k0^2 / (pi hbar c beta^4).
 * Uses one extra FP64 FFT matvec per right-hand side (for G_off p).
 * Arguments as for dda_solve; out [n_energy*n_traj] host.
 */
int dda_eels_cl(dda_ctx* ctx, int n_energy, const double* energy_eV, double beta,
                const double* eps_dipole, const double* r0_nm, int n_traj,
                const void* einc_dev, const void* p_dev, dda_result* out);

/*
 * CL resolved over directions (eq. 42 and section 2.6: a detector collects the
 * scattered light over some solid angle).  For every right-hand side
 * (energy e, trajectory t; p_dev as dda_solve leaves it, [e][t][3][n_occ]
 * complex128, device) and unit direction n_q (dir_xyz [n_dir][3], host):
 *   A_q = sum_j p_j exp(-i k n_q . r_j),  k = m_h k0 (non-absorbing host),
 *   dp_domega[rhs][q] = Pi/(m_h^2 |gamma_h|^2) k^3/(4 pi) |(I - n_q n_q) A_q|^2
 *                       (CL probability per unit solid angle, 1/(eV sr)),
 *   p_cl[rhs] = sum_q weight[q] dp_domega[rhs][q].
 * With weights of a rule exact on the sphere, p_cl equals P_CL of
 * dda_eels_cl (the angular integral of Im G); with weights over a detector's
 * directions it is the collected signal.  The dipole sum runs on the FP64
 * matrix cores, one complex product (directions x dipoles) x (dipoles x
 * 3 n_traj) per energy.  dp_domega and p_cl are host arrays (either may be
 * NULL; p_cl needs weight).  Blocks until the results are on the host.
 * Errors: DDA_EINVAL for an absorbing host, non-unit directions, bad sizes,
 * or lattice sides summing to more than 256.
 */
int dda_cl_directions(dda_ctx* ctx, int n_energy, const double* energy_eV, double beta,
                      int n_traj, const void* p_dev, int n_dir, const double* dir_xyz,
                      const double* weight, double* dp_domega, double* p_cl);

/*
 * One FFT matvec y = A x (or y = sum_{j!=i} G x_j when interaction_only) for
 * nrhs vectors of one energy, in the given precision.  x_dev and y_dev are
 * complex128 [nrhs][3][n_occ]; for DDA_PREC_MIXED they are complex64 and the
 * matvec runs in FP32.  Exposed for testing and benchmarking the kernel chain.
 */
int dda_matvec(dda_ctx* ctx, double energy_eV, const double* eps_dipole, int precision,
               int interaction_only, const void* x_dev, void* y_dev, int nrhs);

/*
 * Continuous batching (COCG only): many systems of one box of lattice cells
 * iterate in the slots of one engine.  The interaction spectrum D depends only
 * on the box, the dipole size and the host wavenumber (the Green's tensor of
 * eq. (5) on the embedding grid), not on which cells are occupied, so every
 * lattice in the box can share the engine: each slot carries its lattice's
 * index map (dda_engine_submit_lattice).
 * Device bytes an engine with n_slots slots holds, counting one interaction
 * spectrum D per slot (the worst case: every slot at a distinct energy):
 * per-slot Krylov vectors, 1/alpha, the FFT work buffer, the slot's index map
 * and D in the context's precision, plus the full-grid scratch of a D build.
 * A server admits engines by this footprint.
 */
int dda_workspace_bytes(const dda_ctx* ctx, int n_slots, size_t* bytes);

/*
 * Opens the context's slot pool (at most one per context; max_slots in
 * [1, 4096]) and allocates everything dda_workspace_bytes counts except the
 * D entries, which come from the context's cache as systems are admitted and
 * stay resident while any slot solves at their wavenumber.
 * Errors: DDA_EINVAL when the solver is not COCG, the lattice is empty or an
 * engine is already open; DDA_ENOMEM.
 */
int dda_engine_open(dda_ctx* ctx, int max_slots);

/*
 * Queues one system at the context's current host index (dda_set_host):
 * energy, eps_dipole [n_occ][2] host (copied), einc_dev
 * complex128 [3][n_occ] (one right-hand side as written by
 * dda_einc_electron) and p_dev complex128 [3][n_occ] for the solution; the
 * device buffers must stay valid until the tag comes back from
 * dda_engine_poll and the caller's later work on the stream has used them.
 * May be called from another thread than the one polling.
 * Errors: DDA_EINVAL for a non-positive energy or a non-finite permittivity.
 */
int dda_engine_submit(dda_ctx* ctx, int64_t tag, double energy_eV, const double* eps_dipole,
                      const void* einc_dev, void* p_dev);

/*
 * dda_engine_submit for a system of another lattice `lat` in the engine
 * context's box: lat must have the same nx, ny, nz, dipole size,
 * polarizability and interaction as ctx and at most as many dipoles (an
 * engine opened on a context whose mask fills the box takes every lattice of
 * that box).  The host index is lat's (dda_set_host on lat); eps_dipole
 * [n][2], einc_dev and p_dev [3][n] with n = lat's dipole count, in lat's
 * ordering.  The slot fills the first n of its entries and keeps the rest
 * zero, so the system's iterates are those of a dda_solve on lat alone.  The
 * call waits for lat's stream (the field written there is read at
 * admission), and lat's stream waits for the copy of the solution into p_dev.
 * lat must stay alive until the tag comes back.
 * Errors: DDA_EINVAL for a lattice that does not fit the engine, as well as
 * dda_engine_submit's.
 */
int dda_engine_submit_lattice(dda_ctx* ctx, dda_ctx* lat, int64_t tag, double energy_eV,
                              const double* eps_dipole, const void* einc_dev, void* p_dev);

/*
 * Runs up to max_intervals COCG intervals.  Before each one it harvests the
 * slots that finished (their p_dev copy is queued on the stream) and admits
 * queued systems into free slots; systems admitted while others are halfway
 * through their iterations join the same kernel launches.  Returns at once
 * when nothing is queued or running.  Up to `capacity` finished systems are
 * returned in tags / info (the rest on later calls); *n_done says how many.
 * A system whose permittivity gives a vanishing or infinite polarizability
 * comes back with status DDA_EINVAL.  Each system's arithmetic does not
 * depend on what shares the slots: its result equals a dda_solve of it alone.
 */
int dda_engine_poll(dda_ctx* ctx, int max_intervals, int64_t* tags, dda_solve_info* info,
                    int capacity, int* n_done);

/* Systems queued, in slots, and finished but not yet returned (the last two
 * as the polling thread last left them); may be called from another thread
 * than the one polling. */
int dda_engine_status(dda_ctx* ctx, int* queued, int* running, int* finished);

/* Waits for the stream and frees the slot pool (queued systems are dropped). */
int dda_engine_close(dda_ctx* ctx);

/*
 * Tile choices of the autotuner for the FFT matvec chain of one precision
 * (DDA_PREC_FP64 or DDA_PREC_MIXED = the FP32 chain).  Before a context's
 * first matvec of a precision (outside any graph capture) the candidates are
 * timed on the actual batch with HIP events: threads per block of the fused
 * yz kernel (three-pass chain), or columns per block of the z-convolution and
 * y passes (five-pass chain); the choice is kept for every context of the
 * process with the same lattice and grid.  The candidates only regroup lines
 * into blocks, so the choice never changes a result.  0 means the default
 * width stood; t_default_ms / t_best_ms time the tuned kernel with the
 * default and the chosen width.  Returns 1 (and zeros) if no matvec of that
 * precision has run yet.
 */
int dda_tuning(const dda_ctx* ctx, int precision, int* zconv_tx, int* mid_tx, int* yz_threads,
               double* t_default_ms, double* t_best_ms);

/*
 * Pins the tile choices of one precision's chain for this context (0 = the
 * default width), bypassing the autotuner.  Errors: DDA_EINVAL for a value
 * that is not a candidate for the context's grid.
 */
int dda_set_tuning(dda_ctx* ctx, int precision, int zconv_tx, int mid_tx, int yz_threads);

/* Per-kernel timing of the matvec chain, measured with HIP events recorded on
 * the context's stream around every launch while timing is enabled
 * (dda_set_timing resets the counters).  enabled: 0 off, 1 all kernels,
 * otherwise a bit mask of the kernels to time, bit k for the k-th name of
 * "unpack_xfft", "yfft", "zconv", "iyfft", "ixfft_pack", "yzconv", "xyfft",
 * "ixyfft_pack" (fewer events, less host work per launch).  Lattices whose
 * padded yz plane fits in LDS run a three-pass chain timed as "unpack_xfft",
 * "yzconv", "ixfft_pack"; FP32 matvecs on cubic x-y grids of 96 or 128 (the
 * padded xy plane of one component fits in LDS) the chain "xyfft", "zconv",
 * "ixyfft_pack"; the others the five-pass chain of the first five names.
 * dda_kernel_time gives, for one kernel: average device time per launch (ms),
 * number of launches, and average right-hand sides per launch. */
int dda_set_timing(dda_ctx* ctx, int enabled);
int dda_kernel_time(dda_ctx* ctx, const char* name, double* avg_ms, int64_t* launches,
                    double* avg_rhs);

/* Frees the cached interaction spectra D(k) (they are rebuilt on demand),
 * except those a system in the context's engine still solves with.  The
 * context keeps one D per host wavenumber it has seen, up to a memory limit;
 * callers that sweep many energies once can release them here. */
int dda_drop_cache(dda_ctx* ctx);

int dda_destroy(dda_ctx* ctx);

/* Test hook: the device K0/K1 routine of dda_einc_electron at n complex
 * points.  z: [n][2] host (re, im); k0k1: [n][4] host out (K0 re, im, K1 re,
 * im).  Arguments are expected in Re z >= 0 (eq. 25 only needs
 * -pi/2 <= arg z <= 0).  Synchronous; uses the default stream. */
int dda_debug_besselk01(const double* z, int64_t n, double* k0k1);

/* Thread-local description of the last failure on this thread. */
const char* dda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDA_H */

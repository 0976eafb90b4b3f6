"""Plain FP64 CPU oracle for the DDA EELS/CL solve (Kichigin & Yurkin,
arXiv 2208.01348).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything here; the product
path (the HIP library and its Python binding) never does, and shares no code,
tables or constants with it.

What it computes, step by step, each function citing the passage it follows:

* electron.py      -- beta from kinetic energy and its host rescaling
                      (eq. 47), beta_h and gamma_h (eq. 24), the incident
                      field of the electron (eq. 25) and the auxiliary field of
                      the conjugate source (eq. 34).  K0/K1 come from scipy's
                      AMOS routines (a library primitive).
* lattice.py       -- dipole centres of the cubic lattice.
* polarizability.py-- Clausius-Mossotti, radiative-reaction and
                      lattice-dispersion polarizabilities (DDA literature; the
                      paper only names the option, section S5).
* interaction.py   -- the free-space Green's tensor of eq. (5) as a
                      dipole-dipole interaction, and the dense system matrix.
* dense_matvec.c   -- the same dense matrix-vector product in plain C with
                      OpenMP, evaluated on the fly (no FFT), for lattices too
                      large to store the matrix.
* solve.py         -- dense LU for small systems, BiCGStab otherwise.
* losses.py        -- P_EELS (eqs. 32, 34, 37, 38), P_ext (eqs. 17, 48),
                      P_abs (eq. 18 with the cell field, in the discrete
                      form that closes the real-host budget) and P_CL
                      (eq. 42).
* dda.py           -- the whole path for one (energy, trajectory).

Pinned by the CPU tests in tests/test_oracle_*.py: mpmath Bessel values and
the integral representation of eq. (S8); numerical derivatives of eq. (23)
against eq. (25); a numerical Hessian against the closed-form Green's tensor;
reciprocity (A = A^T); dense LU against BiCGStab; the single-dipole closed
form; the discrete energy budget; scale invariance (eqs. 43-46); invariance
under a shift of z0 (section S5); the printed beta_h values (section 3.3, 3.4).
The LDR coefficient values are literature constants: parity unpinned for the
values themselves (their limits are pinned).
"""

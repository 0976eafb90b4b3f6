"""Richardson extrapolation to zero dipole size (test infrastructure: only
the tests, the smoke check and the benchmark's CPU leg use this package).

Section 3.2: values computed on a series of lattices are extrapolated to
d = 0 with a quadratic in d, the errors of the points taken to scale as d^3,
and twice the standard error of the fitted value at d = 0 is the nominal 95 %
confidence half-width.  As a weighted least-squares problem: minimise
sum_i w_i (y_i - a - b d_i - c d_i^2)^2 with w_i = d_i^-6; the covariance of
(a, b, c) is s^2 (X^T W X)^-1 with s^2 = sum_i w_i r_i^2 / (n - 3) the
residual variance of the weighted fit.  Solved here by QR of W^(1/2) X.
"""

from __future__ import annotations

import numpy as np


def richardson(d, y):
    """(value at d = 0, 95 % half-width = 2 SE); the half-width is NaN for
    three points (no residual degrees of freedom)."""
    d = np.asarray(d, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if d.size < 3 or np.any(d <= 0):
        raise ValueError("need at least three positive dipole sizes")
    sw = d ** -3.0                       # sqrt of the weights d^-6
    X = np.stack([np.ones_like(d), d, d * d], axis=1)
    Q, R = np.linalg.qr(sw[:, None] * X)
    coef = np.linalg.solve(R, Q.T @ (sw * y))
    if d.size == 3:
        return float(coef[0]), float("nan")
    r = sw * (y - X @ coef)
    s2 = float(r @ r) / (d.size - 3)
    Rinv = np.linalg.inv(R)
    var_a = s2 * float(Rinv[0] @ Rinv[0])   # (X^T W X)^-1 = R^-1 R^-T
    return float(coef[0]), 2.0 * float(np.sqrt(var_a))

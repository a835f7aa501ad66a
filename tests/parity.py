"""Tolerances shared by the GPU parity tests.

FP64 path: |C_gpu - C_oracle| <= max(1e-12 |C_oracle|, kappa 2^-53 A[t]);
FP32-compensated path: |C_gpu - C_oracle| <= kappa 2^-24 A[t];
with A[t] the sum of |Wick terms| (the oracle's permanents) and
kappa = 3 (K(n_u) + K(n_d) + n_q + 3), K(n) = (n - 1) + n (n - 1) / 2 the
number of rounded operations along one monomial's path through the row
Laplace recursion (n - 1 multiplications into the product, n(n-1)/2 additions
across levels), n_q for the weight and leaf/group products, and 3 for the
compensated sums.  The signed sum cancels heavily (|C| / A ~ 1e-3 for D_I and
1e-5 for 3He with i.i.d. propagators), so only a bound relative to A is
meaningful for reduced precision.
"""
import numpy as np


def kappa(nu, nd):
    K = lambda n: (n - 1) + n * (n - 1) // 2  # noqa: E731
    return 3 * (K(nu) + K(nd) + nu + nd + 3)


def tol_f64(C_ref, A, nu, nd):
    return np.maximum(1e-12 * np.abs(C_ref), kappa(nu, nd) * 2.0 ** -53 * A)


def tol_f32c(A, nu, nd):
    return kappa(nu, nd) * 2.0 ** -24 * A


def f64_branch(C_ref, A, nu, nd):
    """Which term of the FP64 bound applied, per entry: 'rel' where
    1e-12 |C| exceeds kappa 2^-53 A, 'abs' otherwise; returns a short report."""
    rel = 1e-12 * np.abs(C_ref)
    ab = kappa(nu, nd) * 2.0 ** -53 * np.asarray(A)
    n_rel = int(np.count_nonzero(rel > ab))
    return f"FP64 bound branch: 1e-12|C| on {n_rel}, kappa 2^-53 A on {rel.size - n_rel} of {rel.size} entries"

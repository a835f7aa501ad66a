"""Euclidean Dirac-basis gamma matrices, exact (Gaussian-integer) entries.

The paper's operators (Sec. 1, eq. "ops" and the single-baryon operators
before it) use C*gamma5 and P+- = (1 +- gamma4)/2 without naming a basis.  The
reading here: the Euclidean Dirac basis

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],  gamma_4 = diag(1, 1, -1, -1),
    gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4,    C = gamma_2 gamma_4,

for which C gamma_mu C^{-1} = -gamma_mu^T holds (checked in the tests).  Every
matrix is returned as a pair of int64 arrays (real part, imaginary part) so
that the operator algebra built on it is exact.
"""
import numpy as np

_SIGMA = {
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def _as_exact(m):
    """Split a complex matrix with integer parts into (re, im) int64 arrays."""
    re = np.rint(m.real)
    im = np.rint(m.imag)
    assert np.array_equal(re, m.real) and np.array_equal(im, m.imag), "non-integer entry"
    return re.astype(np.int64), im.astype(np.int64)


def _complex_gammas():
    z = np.zeros((2, 2), dtype=complex)
    g = {}
    for k in (1, 2, 3):
        g[k] = np.block([[z, -1j * _SIGMA[k]], [1j * _SIGMA[k], z]])
    g[4] = np.diag([1, 1, -1, -1]).astype(complex)
    g[5] = g[1] @ g[2] @ g[3] @ g[4]
    return g


def gamma_matrices():
    """gamma_1..gamma_5 as exact (re, im) pairs, keyed 1..5."""
    return {k: _as_exact(v) for k, v in _complex_gammas().items()}


def charge_conjugation():
    """C = gamma_2 gamma_4 as an exact (re, im) pair."""
    g = _complex_gammas()
    return _as_exact(g[2] @ g[4])


def cg5(projector=0):
    """C gamma_5, or C gamma_5 P_+ (projector=+1) / C gamma_5 P_- (projector=-1).

    P_+- = (1 +- gamma_4)/2 (Sec. 1, below the single-baryon operators).  In
    the Dirac basis P_+- is diagonal with 0/1 entries, so the product stays
    integral.
    """
    g = _complex_gammas()
    m = g[2] @ g[4] @ g[5]
    if projector:
        p = (np.eye(4) + projector * g[4]) / 2
        m = m @ p
    return _as_exact(m)


def complex_of(pair):
    """Exact (re, im) pair -> complex128 matrix (for numeric checks only)."""
    return pair[0].astype(float) + 1j * pair[1].astype(float)

"""Seeded synthetic quark propagators (NumPy PCG64 ``default_rng``).

This module only draws random numbers; it holds none of the correlator's
arithmetic, so the GPU path and the FP64 oracle can both be fed from it.

Layout: arrays [T, V, 12, 12] complex128 with V = L^3 sites per timeslice in
[z][y][x] order and the 12 = 4*colour + spin index, rows sink and columns
source.  The paper's propagators (point-source solves on 64^3 gauge
configurations) are not available; these recipes stand in for them:

iid(T, V, seed)
    every entry complex Gaussian with E|S_ab|^2 = 1/12 (real and imaginary
    parts each N(0, 1/24)); draw order: Re S_u, Im S_u, Re S_d, Im S_d.
su3_spin(T, V, seed)
    S = U (x) (I_4 + 0.3 N) per site and flavour: U a Haar-random SU(3)
    colour matrix (QR of a complex Ginibre matrix, phase-fixed, divided by the
    cube root of its determinant), N a 4x4 complex Gaussian with E|N_ab|^2 = 1;
    draw order: U_u, N_u, U_d, N_d (real parts before imaginary parts).
"""
import numpy as np


def _cgauss(rng, shape, var):
    s = np.sqrt(var / 2.0)
    re = rng.standard_normal(shape) * s
    im = rng.standard_normal(shape) * s
    return re + 1j * im


def iid(T, V, seed):
    """(S_u, S_d), i.i.d. complex Gaussian entries with variance 1/12."""
    rng = np.random.default_rng(seed)
    shape = (T, V, 12, 12)
    S_u = _cgauss(rng, shape, 1.0 / 12.0)
    S_d = _cgauss(rng, shape, 1.0 / 12.0)
    return S_u, S_d


def _haar_su3(rng, shape):
    z = _cgauss(rng, shape + (3, 3), 1.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


def _colour_spin(U, M):
    """Kronecker product per site: out[4c+s, 4c'+s'] = U[c, c'] M[s, s']."""
    out = U[..., :, None, :, None] * M[..., None, :, None, :]
    return out.reshape(U.shape[:-2] + (12, 12))


def su3_spin(T, V, seed, noise=0.3):
    """(S_u, S_d) = SU(3) colour matrix (x) (I_4 + noise * complex Gaussian)."""
    rng = np.random.default_rng(seed)
    shape = (T, V)
    out = []
    for _ in range(2):
        U = _haar_su3(rng, shape)
        N = _cgauss(rng, shape + (4, 4), 1.0)
        out.append(_colour_spin(U, np.eye(4) + noise * N))
    return out[0], out[1]


def random_su3(n, seed):
    """n Haar-random SU(3) matrices (for colour-rotation checks)."""
    return _haar_su3(np.random.default_rng(seed), (n,))

"""Determinant-form correlator, sum of |Wick terms|, and gradients (FP64).

Per site x and correlator c (eq. 1 with the determinant formulation the paper
cites in Sec. 1, Detmold-Orginos):

    C_c(x) = sum_{k in I_c} W_k det(S_u(x)[snk_u_k ; src_u_k]) det(S_d(x)[snk_d_k ; src_d_k]),

rows are sink indices and columns source indices, and the per-timeslice
correlator is the zero-momentum sink sum C_c[t] = sum_{x in t} C_c(x)
(Sec. 2, the sum over x with exp(-i p.x) at p = 0).

Determinants are LAPACK's (numpy.linalg.det, partial-pivot LU).  Propagators
are arrays S[t, v, 12, 12] (v = site within the timeslice).  Values of a
determinant that occurs in several entries are computed once and reused
(memoisation; no reordering of the sum over I).

Gradients follow PyTorch's convention for complex inputs:
grad_W[k]       = sum_t g[c_k, t] conj(dC_ck[t]/dW_k),
grad_S(x)[a, b] = sum_c g[c, t(x)] conj(dC_c[t(x)]/dS(x)[a, b]),
with dC/dW_k = sum_x det_u det_d (C is linear in W, eq. 1) and the derivative
of a determinant by Jacobi's formula, d det(A)/dA_ij = cofactor_ij, with the
cofactors formed explicitly from (n-1)x(n-1) minors (valid for singular A).
"""
from itertools import permutations

import numpy as np


def _unique_pairs(rows, cols):
    """Distinct (row tuple, col tuple) pairs and the inverse map per entry.

    Each pair is encoded as the base-12 integer of its 2n digits (n <= 6
    keeps it below 2^63) so that the search for duplicates is one 1-D sort.
    """
    digits = np.concatenate([rows, cols], axis=1).astype(np.int64)
    code = np.zeros(digits.shape[0], dtype=np.int64)
    for i in range(digits.shape[1]):
        code = code * 12 + digits[:, i]
    _, first, inv = np.unique(code, return_index=True, return_inverse=True)
    n = rows.shape[1]
    uniq = digits[first]
    return uniq[:, :n], uniq[:, n:], inv.reshape(-1)


def _submatrices(S, rows, cols):
    """S[..., rows[m, i], cols[m, j]] -> [..., m, n, n]."""
    return S[..., rows[:, :, None], cols[:, None, :]]


def _dets(S, rows, cols):
    return np.linalg.det(_submatrices(S, rows, cols))


def _permanents(A):
    """Permanent of the trailing n x n matrices of A by Leibniz's sum."""
    n = A.shape[-1]
    out = np.zeros(A.shape[:-2], dtype=A.dtype)
    for p in permutations(range(n)):
        term = np.ones(A.shape[:-2], dtype=A.dtype)
        for i in range(n):
            term = term * A[..., i, p[i]]
        out += term
    return out


class _Prepared:
    """Per index set: distinct u/d pairs, per-entry inverse maps, weights."""

    def __init__(self, iset):
        self.iset = iset
        self.ru, self.cu, self.inv_u = _unique_pairs(iset.snk_u, iset.src_u)
        self.rd, self.cd, self.inv_d = _unique_pairs(iset.snk_d, iset.src_d)
        self.W = iset.weights()
        self.corr = iset.corr_id


def _prep(iset):
    p = getattr(iset, "_oracle_prep", None)
    if p is None:
        p = _Prepared(iset)
        iset._oracle_prep = p
    return p


def _site_batches(n, batch):
    for s in range(0, n, batch):
        yield slice(s, min(n, s + batch))


def site_values(S_u, S_d, iset, batch=8):
    """C_c(x) for every site: returns [n_corr, n_sites] complex128.

    S_u, S_d: [n_sites, 12, 12] complex128.
    """
    p = _prep(iset)
    ns = S_u.shape[0]
    out = np.zeros((iset.n_corr, ns), dtype=np.complex128)
    for sl in _site_batches(ns, batch):
        Du = _dets(S_u[sl], p.ru, p.cu)[:, p.inv_u]
        Dd = _dets(S_d[sl], p.rd, p.cd)[:, p.inv_d]
        terms = p.W[None, :] * Du * Dd
        for c in range(iset.n_corr):
            out[c, sl] = terms[:, p.corr == c].sum(axis=1)
    return out


def correlator(S_u, S_d, iset, batch=8):
    """C[c, t] = sum over sites of timeslice t of C_c(x).

    S_u, S_d: [T, V, 12, 12] complex128.  Returns [n_corr, T] complex128.
    """
    T, V = S_u.shape[:2]
    vals = site_values(S_u.reshape(T * V, 12, 12), S_d.reshape(T * V, 12, 12), iset, batch)
    return vals.reshape(iset.n_corr, T, V).sum(axis=2)


def sum_abs_terms(S_u, S_d, iset, batch=8):
    """A[c, t] = sum_{x in t} sum_k |W_k| perm|S_u sub| perm|S_d sub|.

    The sum of the magnitudes of every quark-level Wick term (a permanent of
    the entrywise absolute values counts each of the n! terms of a determinant
    with its magnitude).  It is the scale against which reduced-precision
    results are bounded, since the signed sum cancels heavily.
    """
    p = _prep(iset)
    T, V = S_u.shape[:2]
    Su = np.abs(S_u.reshape(T * V, 12, 12))
    Sd = np.abs(S_d.reshape(T * V, 12, 12))
    aw = np.abs(p.W)
    out = np.zeros((iset.n_corr, T * V))
    for sl in _site_batches(T * V, batch):
        Pu = _permanents(_submatrices(Su[sl], p.ru, p.cu))[:, p.inv_u]
        Pd = _permanents(_submatrices(Sd[sl], p.rd, p.cd))[:, p.inv_d]
        terms = aw[None, :] * Pu * Pd
        for c in range(iset.n_corr):
            out[c, sl] = terms[:, p.corr == c].sum(axis=1)
    return out.reshape(iset.n_corr, T, V).sum(axis=2)


def _cofactors(S, rows, cols):
    """Cofactor matrices of every submatrix: [..., m, n, n].

    cof[..., i, j] = (-1)^(i+j) det(submatrix without row i and column j);
    for n = 1 the cofactor of the single entry is 1.
    """
    n = rows.shape[1]
    shape = S.shape[:-2] + (rows.shape[0], n, n)
    cof = np.empty(shape, dtype=np.complex128)
    if n == 1:
        cof[...] = 1.0
        return cof
    for i in range(n):
        ri = np.delete(rows, i, axis=1)
        for j in range(n):
            cj = np.delete(cols, j, axis=1)
            cof[..., i, j] = (-1) ** (i + j) * _dets(S, ri, cj)
    return cof


def gradients(S_u, S_d, iset, grad_C, want=("W", "S_u", "S_d"), batch=4):
    """Gradients of L with dL/dC* = grad_C (PyTorch's complex convention).

    grad_C: [n_corr, T] complex128.  Returns a dict with any of
    "W"   -> [nnz] complex128,
    "S_u" -> [T, V, 12, 12] complex128,
    "S_d" -> [T, V, 12, 12] complex128.
    """
    p = _prep(iset)
    T, V = S_u.shape[:2]
    ns = T * V
    Su = S_u.reshape(ns, 12, 12)
    Sd = S_d.reshape(ns, 12, 12)
    t_of = np.repeat(np.arange(T), V)
    nnz = iset.nnz
    out = {}
    if "W" in want:
        gW = np.zeros(nnz, dtype=np.complex128)
    if "S_u" in want:
        gSu = np.zeros((ns, 144), dtype=np.complex128)
    if "S_d" in want:
        gSd = np.zeros((ns, 144), dtype=np.complex128)
    nu, nd = iset.nu, iset.nd
    for sl in _site_batches(ns, batch):
        Du = _dets(Su[sl], p.ru, p.cu)[:, p.inv_u]          # [b, nnz]
        Dd = _dets(Sd[sl], p.rd, p.cd)[:, p.inv_d]
        g = grad_C[p.corr][:, t_of[sl]].T                   # [b, nnz]: g[c_k, t(x)]
        if "W" in want:
            gW += np.sum(g * np.conj(Du * Dd), axis=0)
        if "S_u" in want:
            cof = _cofactors(Su[sl], p.ru, p.cu)[:, p.inv_u]  # [b, nnz, nu, nu]
            coef = g * np.conj(p.W[None, :] * Dd)             # [b, nnz]
            for i in range(nu):
                for j in range(nu):
                    flat = iset.snk_u[:, i] * 12 + iset.src_u[:, j]
                    contrib = coef * np.conj(cof[:, :, i, j])
                    for bi, x in enumerate(range(sl.start, sl.stop)):
                        np.add.at(gSu[x], flat, contrib[bi])
        if "S_d" in want:
            cof = _cofactors(Sd[sl], p.rd, p.cd)[:, p.inv_d]
            coef = g * np.conj(p.W[None, :] * Du)
            for i in range(nd):
                for j in range(nd):
                    flat = iset.snk_d[:, i] * 12 + iset.src_d[:, j]
                    contrib = coef * np.conj(cof[:, :, i, j])
                    for bi, x in enumerate(range(sl.start, sl.stop)):
                        np.add.at(gSd[x], flat, contrib[bi])
    if "W" in want:
        out["W"] = gW
    if "S_u" in want:
        out["S_u"] = gSu.reshape(T, V, 12, 12)
    if "S_d" in want:
        out["S_d"] = gSd.reshape(T, V, 12, 12)
    return out


def _perm_cofactors(S, rows, cols):
    """Permanents of every (n-1)x(n-1) minor: [..., m, n, n] (no signs)."""
    n = rows.shape[1]
    shape = S.shape[:-2] + (rows.shape[0], n, n)
    cof = np.empty(shape, dtype=S.dtype)
    if n == 1:
        cof[...] = 1.0
        return cof
    for i in range(n):
        ri = np.delete(rows, i, axis=1)
        for j in range(n):
            cj = np.delete(cols, j, axis=1)
            cof[..., i, j] = _permanents(_submatrices(S, ri, cj))
    return cof


def gradient_abs_scales(S_u, S_d, iset, grad_C, batch=4):
    """Sum of |Wick terms| of every gradient entry (scales for tolerances).

    The same sums as ``gradients`` with |W|, |grad_C| and |S| and every sign
    +, i.e. determinants replaced by permanents: each entry is the sum of the
    magnitudes of the quark-level terms that make up that gradient entry.
    Returns a dict like ``gradients`` (real arrays).
    """
    p = _prep(iset)
    T, V = S_u.shape[:2]
    ns = T * V
    Su = np.abs(S_u.reshape(ns, 12, 12))
    Sd = np.abs(S_d.reshape(ns, 12, 12))
    t_of = np.repeat(np.arange(T), V)
    aW = np.abs(p.W)
    ag = np.abs(grad_C)
    gW = np.zeros(iset.nnz)
    gSu = np.zeros((ns, 144))
    gSd = np.zeros((ns, 144))
    for sl in _site_batches(ns, batch):
        Pu = _permanents(_submatrices(Su[sl], p.ru, p.cu))[:, p.inv_u]
        Pd = _permanents(_submatrices(Sd[sl], p.rd, p.cd))[:, p.inv_d]
        g = ag[p.corr][:, t_of[sl]].T
        gW += np.sum(g * Pu * Pd, axis=0)
        for name, S, rows, cols, inv, other, acc, n in (
                ("u", Su, p.ru, p.cu, p.inv_u, Pd, gSu, iset.nu), ("d", Sd, p.rd, p.cd, p.inv_d, Pu, gSd, iset.nd)):
            cof = _perm_cofactors(S[sl], rows, cols)[:, inv]
            coef = g * aW[None, :] * other
            snk = iset.snk_u if name == "u" else iset.snk_d
            src = iset.src_u if name == "u" else iset.src_d
            for i in range(n):
                for j in range(n):
                    flat = snk[:, i] * 12 + src[:, j]
                    contrib = coef * cof[:, :, i, j]
                    for bi, x in enumerate(range(sl.start, sl.stop)):
                        np.add.at(acc[x], flat, contrib[bi])
    return {"W": gW, "S_u": gSu.reshape(T, V, 12, 12), "S_d": gSd.reshape(T, V, 12, 12)}

"""Brute-force Grassmann Wick contraction, straight from eq. 1.

For one sink term q_1 ... q_n and one source term qbar_1 ... qbar_n (fields in
written order, each with a flavour and an index a = 4*colour + spin), the
expectation < q_1 ... q_n qbar_1 ... qbar_n > is the sum over all
flavour-preserving pairings pi (q_i with qbar_pi(i)) of

    sign(pi) * prod_i S^{f_i}[a_i, a'_pi(i)],

where sign(pi) is the parity of the field permutation that brings the sequence
(q_1 .. q_n qbar_1 .. qbar_n) to (q_1 qbar_pi(1) q_2 qbar_pi(2) ... ), after
which each adjacent (q qbar) pair is a propagator S = <q qbar> (Sec. 2, the
propagator definition before the proton block).  Nothing here uses
determinants, sorting, or the flavour-separation sign: it is the independent
check of those steps.  The cost is n_u! n_d! per term pair, so it is used on
tiny inputs only.
"""
from functools import lru_cache
from itertools import permutations

import numpy as np


def _parity(seq):
    inv = 0
    for i in range(len(seq)):
        for j in range(i + 1, len(seq)):
            if seq[i] > seq[j]:
                inv += 1
    return -1 if inv & 1 else 1


def pairings(snk_flav, src_flav):
    return _pairings(tuple(snk_flav), tuple(src_flav))


@lru_cache(maxsize=None)
def _pairings(snk_flav, src_flav):
    """All flavour-preserving pairings with their Grassmann signs.

    ``snk_flav`` / ``src_flav`` are the written flavour sequences of the sink
    and source terms.  Returns a list of (pi, sign): q_i pairs with qbar_pi[i].
    """
    n = len(snk_flav)
    out = []
    for pi in permutations(range(n)):
        if any(snk_flav[i] != src_flav[pi[i]] for i in range(n)):
            continue
        # target order: q_0, qbar_pi0, q_1, qbar_pi1, ... as original positions
        target = []
        for i in range(n):
            target += [i, n + pi[i]]
        out.append((pi, _parity(target)))
    return out


def wick_pairs(S_by_flavour, snk_flav, snk_idx, src_flav, src_idx):
    """< sink term r, source term c > for every (r, c) of two term lists.

    S_by_flavour: tuple of [12, 12] complex arrays indexed by flavour label.
    snk_flav:     written flavour sequence shared by the sink terms (length n).
    snk_idx:      [R, n] int, the sink terms' field indices in written order.
    src_flav, src_idx: the same for the source terms.
    Returns an [R, Cs] complex128 array of expectations.
    """
    snk_idx = np.asarray(snk_idx)
    src_idx = np.asarray(src_idx)
    out = np.zeros((snk_idx.shape[0], src_idx.shape[0]), dtype=np.complex128)
    for pi, sgn in pairings(snk_flav, src_flav):
        term = np.full(out.shape, float(sgn), dtype=np.complex128)
        for i, f in enumerate(snk_flav):
            S = S_by_flavour[f]
            term *= S[snk_idx[:, i][:, None], src_idx[:, pi[i]][None, :]]
        out += term
    return out


def correlator_bruteforce(S_u, S_d, terms, s2):
    """C at one site from raw (unseparated) operator terms, brute force.

    ``terms`` is the sink operator as (coef, fields) with coef a Gaussian
    integer (re, im) and fields ((flavour, index), ...) in written order; the
    source operator has the conjugated coefficients and the same fields.
    C = s2 * sum_{r, c} coef_r conj(coef_c) < r, c-bar >, evaluated per pair
    of written flavour sequences.
    """
    groups = {}
    for coef, fields in terms:
        key = tuple(f for f, _ in fields)
        g = groups.setdefault(key, ([], []))
        g[0].append([i for _, i in fields])
        g[1].append(complex(coef[0], coef[1]))
    tot = 0.0 + 0.0j
    for fr, (ir, cr) in groups.items():
        for fc, (ic, cc) in groups.items():
            E = wick_pairs((S_u, S_d), fr, np.array(ir), fc, np.array(ic))
            tot += np.array(cr) @ E @ np.conj(np.array(cc))
    return complex(s2) * tot

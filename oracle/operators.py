"""Operator algebra and index sets, in exact Gaussian-integer arithmetic.

Follows Sec. 1 of the paper: the single-baryon operators p, n, p+-, n+- (the
epsilon_abc (q^T Gamma q') q^alpha form with Gamma = C gamma5 or C gamma5 P+-),
the multi-baryon operators of eq. "ops" (D_I, D_II, 3He_I^j, 3He_II^j), and the
correlator of eq. 1,

    C = sum_{(a, a') in I} W^{a}_{a'} < q(a_1) ... q(a_nq) qbar(a'_1) ... qbar(a'_nq) >,

with I the set of index pairs with non-zero weight (the "index set").

Conventions (readings where the paper is silent):
* a quark index is a = 4*colour + spin, 0 <= a < 12;
* a sink operator is a list of terms (coefficient, fields), the fields an
  ordered product of Grassmann quark fields kept in written order;
* the source operator carries the conjugated coefficients and the same written
  field order, so a single correlator's weight is W_{r,c} = sigma s^2 w_r conj(w_c);
* sigma = (-1)^(n_u n_d + n_u(n_u-1)/2 + n_d(n_d-1)/2) is the Grassmann sign of
  bringing <u..u d..d ubar..ubar dbar..dbar> to a product of two determinants
  (moving the ubar block past the d block, then <q_1..q_n qbar_1..qbar_n> =
  (-1)^(n(n-1)/2) det);
* sign_mode "exact" keeps every written relative sign of eq. "ops"; sign_mode
  "r2" replaces each written relative sign by +1 (equivalently: the baryons
  treated as commuting labels).  Under exact Grassmann algebra D_II and 3He_II
  vanish at a local sink (X^T Gamma Y = Y^T Gamma X for Grassmann-odd X, Y and
  antisymmetric Gamma), so "r2" is the non-physical stand-in that gives those
  operators a non-empty index set.

Coefficients are Gaussian integers held as (re, im) pairs of Python ints.
"""
from fractions import Fraction
from itertools import permutations

import numpy as np

from .gamma import cg5

U, D = 0, 1  # flavour labels

OPS = ("proton", "neutron", "DI", "DII", "HE3_I", "HE3_II")


# ----------------------------------------------------------------------------
# Gaussian integers
# ----------------------------------------------------------------------------
def gmul(x, y):
    return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])


def gconj(x):
    return (x[0], -x[1])


def gadd(x, y):
    return (x[0] + y[0], x[1] + y[1])


def gscale(x, s):
    return (x[0] * s, x[1] * s)


def _perm_parity(seq):
    """(-1)^(number of inversions) of a sequence of distinct integers."""
    inv = 0
    for i in range(len(seq)):
        for j in range(i + 1, len(seq)):
            if seq[i] > seq[j]:
                inv += 1
    return -1 if inv & 1 else 1


def _levi_civita3():
    """[(a, b, c), eps_abc] over the six permutations of (0, 1, 2)."""
    return [(p, _perm_parity(p)) for p in permutations(range(3))]


# ----------------------------------------------------------------------------
# Single-baryon operators (Sec. 1)
# ----------------------------------------------------------------------------
def baryon_terms(kind, spin, projector=0):
    """Terms of a single-baryon operator at one open spin index.

    kind "p": p^alpha = eps_abc (u_a^T Gamma d_b) u_c^alpha
    kind "n": n^alpha = eps_abc (d_a^T Gamma u_b) d_c^alpha
    with Gamma = C gamma5 (projector 0) or C gamma5 P+- (projector +-1).
    Expanded: sum over a, b, c, beta, gamma of eps_abc Gamma_{beta gamma}
    q1(4a+beta) q2(4b+gamma) q1(4c+alpha), fields kept in that written order.
    Returns a list of (coef, fields) with fields a tuple of (flavour, index).
    """
    gre, gim = cg5(projector)
    f1, f2 = (U, D) if kind == "p" else (D, U)
    out = []
    for (a, b, c), eps in _levi_civita3():
        for beta in range(4):
            for gam in range(4):
                g = (int(gre[beta, gam]), int(gim[beta, gam]))
                if g == (0, 0):
                    continue
                out.append((gscale(g, eps),
                            ((f1, 4 * a + beta), (f2, 4 * b + gam), (f1, 4 * c + spin))))
    return out


# (kind, projector) of the baryons used by eq. "ops"
_B = {"p": ("p", 0), "n": ("n", 0), "p+": ("p", 1), "p-": ("p", -1),
      "n+": ("n", 1), "n-": ("n", -1)}

def _baryon(name, spin):
    kind, proj = _B[name]
    return baryon_terms(kind, spin, proj)


# eq. "ops": each operator is a signed sum of products X^T (C gamma5) Y [Z^j],
# with the overall scale s (s^2 kept exactly).
_MULTI = {
    "DI": (Fraction(1), [(+1, "n", "p")]),
    "DII": (Fraction(1, 2), [(+1, "n", "p"), (-1, "p", "n")]),
    "HE3_I": (Fraction(1), [(+1, "p-", "n+", "p+")]),
    "HE3_II": (Fraction(1, 6), [(+1, "p-", "n+", "p+"), (-1, "p+", "n+", "p-"),
                                (+1, "n+", "p+", "p-"), (-1, "n+", "p-", "p+"),
                                (+1, "p+", "p-", "n+"), (-1, "p-", "p+", "n+")]),
}


def operator_terms(op, spin=0, sign_mode="exact"):
    """Sink operator of eq. "ops" (or a single baryon) as raw Grassmann terms.

    Returns (terms, s2): terms a list of (coef, fields) in written field order,
    s2 the exact square of the operator's overall scale (1, 1/2 or 1/6).
    ``spin`` is alpha for the proton/neutron and j for 3He; it is ignored for
    the dinucleons.  X^T (C gamma5) Y = sum_{alpha beta} (C gamma5)_{alpha beta}
    X^alpha Y^beta, fields of X written before those of Y (and of Z^j last).
    """
    if sign_mode not in ("exact", "r2"):
        raise ValueError(sign_mode)
    if op in ("proton", "neutron"):
        return baryon_terms("p" if op == "proton" else "n", spin, 0), Fraction(1)
    if op not in _MULTI:
        raise ValueError(op)
    s2, products = _MULTI[op]
    gre, gim = cg5(0)
    terms = []
    for relsign, *names in products:
        if sign_mode == "r2":
            relsign = 1
        third = [_baryon(names[2], spin)] if len(names) == 3 else [[((1, 0), ())]]
        for al in range(4):
            for be in range(4):
                g = (int(gre[al, be]), int(gim[al, be]))
                if g == (0, 0):
                    continue
                g = gscale(g, relsign)
                for cx, fx in _baryon(names[0], al):
                    for cy, fy in _baryon(names[1], be):
                        cxy = gmul(g, gmul(cx, cy))
                        for cz, fz in third[0]:
                            terms.append((gmul(cxy, cz), fx + fy + fz))
    return terms, s2


def baryon_products(op, spin=0, sign_mode="exact"):
    """Sink operator of eq. "ops" as a sum of products of single baryons.

    Returns (products, s2): products a list of (coef, slots) with slots a
    tuple of (baryon name, open spin) in written order, so that the operator
    is sum coef * prod_i B_i^{spin_i}; coef carries the written relative sign
    (or +1 under "r2") times (C gamma5)_{alpha beta} of the first two baryons.
    The third baryon of 3He carries the open index j = ``spin``.  A single
    baryon is one product with coefficient 1.  Used by the block-level
    correlator, where baryon i of a product sits at its own sink point.
    """
    if sign_mode not in ("exact", "r2"):
        raise ValueError(sign_mode)
    if op in ("proton", "neutron"):
        return [((1, 0), (("p" if op == "proton" else "n", spin),))], Fraction(1)
    if op not in _MULTI:
        raise ValueError(op)
    s2, prods = _MULTI[op]
    gre, gim = cg5(0)
    out = []
    for relsign, *names in prods:
        if sign_mode == "r2":
            relsign = 1
        for al in range(4):
            for be in range(4):
                g = (int(gre[al, be]), int(gim[al, be]))
                if g == (0, 0):
                    continue
                slots = ((names[0], al), (names[1], be)) + (((names[2], spin),) if len(names) == 3 else ())
                out.append((gscale(g, relsign), slots))
    return out, s2


def quark_counts(op):
    """(n_u, n_d) of an operator."""
    terms, _ = operator_terms(op)
    fields = terms[0][1]
    nu = sum(1 for f, _ in fields if f == U)
    return nu, len(fields) - nu


# ----------------------------------------------------------------------------
# Flavour separation and canonical ordering (Sec. 3: canonical order + multiplicity)
# ----------------------------------------------------------------------------
def flavour_separate(terms):
    """Stable-partition each term's fields into u...u d...d.

    Grassmann sign: (-1)^(number of (d, u) pairs with the d written first).
    Returns the raw sink tensor: list of (coef, u_tuple, d_tuple), tuples in
    written order (no sorting, no merging).
    """
    out = []
    for coef, fields in terms:
        nswap = 0
        seen_d = 0
        for f, _ in fields:
            if f == D:
                seen_d += 1
            else:
                nswap += seen_d
        u = tuple(i for f, i in fields if f == U)
        d = tuple(i for f, i in fields if f == D)
        out.append((gscale(coef, -1 if nswap & 1 else 1), u, d))
    return out


def canonical_tensor(raw):
    """Symmetrise a raw sink tensor into canonical keys.

    For each raw term: drop it if a flavour tuple repeats an index (the
    Grassmann product vanishes); otherwise sort each tuple ascending, multiply
    by both permutation parities, and accumulate exactly per key
    (sorted u, sorted d).  Zero sums are dropped.  Returns a dict
    {(u_sorted, d_sorted): coef}.  This is the determinant-form analogue of
    the paper's canonical lexicographic ordering with multiplicities (Sec. 3).
    """
    acc = {}
    for coef, u, d in raw:
        if len(set(u)) != len(u) or len(set(d)) != len(d):
            continue
        su = tuple(sorted(u))
        sd = tuple(sorted(d))
        par = _perm_parity(u) * _perm_parity(d)
        key = (su, sd)
        acc[key] = gadd(acc.get(key, (0, 0)), gscale(coef, par))
    return {k: v for k, v in acc.items() if v != (0, 0)}


def grassmann_sigma(nu, nd):
    """sigma = (-1)^(n_u n_d + n_u(n_u-1)/2 + n_d(n_d-1)/2)."""
    e = nu * nd + nu * (nu - 1) // 2 + nd * (nd - 1) // 2
    return -1 if e & 1 else 1


# ----------------------------------------------------------------------------
# Index sets (eq. 1)
# ----------------------------------------------------------------------------
class IndexSet:
    """Flat index set of one or more correlators over the same (n_u, n_d).

    Entry k carries sink/source index tuples snk_u[k], src_u[k] (length n_u)
    and snk_d[k], src_d[k] (length n_d), its correlator corr_id[k], and the
    exact weight W_k = (w_num_re[k] + i w_num_im[k]) / w_den[corr_id[k]].
    Canonical entries are ordered by correlator, then lexicographically by
    (snk_u, src_u, snk_d, src_d).
    """

    def __init__(self, nu, nd, snk_u, src_u, snk_d, src_d, corr_id, w_re, w_im, w_den):
        self.nu, self.nd = nu, nd
        self.snk_u = np.asarray(snk_u, dtype=np.int32).reshape(-1, nu)
        self.src_u = np.asarray(src_u, dtype=np.int32).reshape(-1, nu)
        self.snk_d = np.asarray(snk_d, dtype=np.int32).reshape(-1, nd)
        self.src_d = np.asarray(src_d, dtype=np.int32).reshape(-1, nd)
        self.corr_id = np.asarray(corr_id, dtype=np.int32)
        self.w_re = np.asarray(w_re, dtype=np.int64)
        self.w_im = np.asarray(w_im, dtype=np.int64)
        self.w_den = np.asarray(w_den, dtype=np.int64)

    @property
    def nnz(self):
        return int(self.corr_id.shape[0])

    @property
    def n_corr(self):
        return int(self.w_den.shape[0])

    def weights(self):
        """Complex128 weights W_k (rounded from the exact rationals)."""
        den = self.w_den[self.corr_id].astype(float)
        return (self.w_re.astype(float) + 1j * self.w_im.astype(float)) / den


def _tensor_for(op, spin, sign_mode, symmetrise):
    terms, s2 = operator_terms(op, spin, sign_mode)
    raw = flavour_separate(terms)
    if symmetrise:
        return {k: v for k, v in canonical_tensor(raw).items()}, s2, True
    # raw: merge nothing, keep written-order tuples (repeats included)
    return raw, s2, False


def _key_arrays(items, nu, nd):
    """(coef, u_tuple, d_tuple) list -> int arrays [n, nu], [n, nd], [n, 2]."""
    u = np.array([it[1] for it in items], dtype=np.int32).reshape(-1, nu)
    d = np.array([it[2] for it in items], dtype=np.int32).reshape(-1, nd)
    w = np.array([it[0] for it in items], dtype=np.int64).reshape(-1, 2)
    return u, d, w


def _ranks(tuples):
    """Rank of each row among the distinct rows, in lexicographic order."""
    _, inv = np.unique(tuples, axis=0, return_inverse=True)
    return inv.reshape(-1)


def build_index_set(ops):
    """Index set of a batch of correlators sharing (n_u, n_d).

    ``ops`` is a list of dicts with keys op, snk_spin, src_spin, sign_mode
    ("exact"/"r2"), symmetrise (True: canonical keys; False: raw terms).
    Correlator i has W_{r,c} = sigma s^2 w^{snk}_r conj(w^{src}_c) on the
    Cartesian product of its sink and source keys; zero weights never occur
    (products of non-zero Gaussian integers).
    """
    nu = nd = None
    cols = {k: [] for k in ("snk_u", "src_u", "snk_d", "src_d", "corr", "re", "im")}
    dens = []
    for ci, od in enumerate(ops):
        op = od["op"]
        mode = od.get("sign_mode", "exact")
        sym = od.get("symmetrise", True)
        cnu, cnd = quark_counts(op)
        if nu is None:
            nu, nd = cnu, cnd
        elif (nu, nd) != (cnu, cnd):
            raise ValueError("correlators in one index set must share (n_u, n_d)")
        sig = grassmann_sigma(nu, nd)
        snk, s2, _ = _tensor_for(op, od.get("snk_spin", 0), mode, sym)
        src, _, _ = _tensor_for(op, od.get("src_spin", 0), mode, sym)
        if sym:
            snk_items = sorted(snk.items())
            src_items = sorted(src.items())
            snk_list = [(c, k[0], k[1]) for k, c in snk_items]
            src_list = [(c, k[0], k[1]) for k, c in src_items]
        else:
            snk_list, src_list = snk, src
        if s2.numerator != 1:
            raise ValueError("scale numerator must be 1")
        dens.append(s2.denominator)
        ru, rd, rw = _key_arrays(snk_list, nu, nd)
        cu, cd, cw = _key_arrays(src_list, nu, nd)
        nr, nc = len(snk_list), len(src_list)
        ii = np.repeat(np.arange(nr), nc)
        jj = np.tile(np.arange(nc), nr)
        if sym and nr and nc:
            # lexicographic order of (snk_u, src_u, snk_d, src_d): equal-length
            # tuples compare like their ranks among the distinct tuples
            order = np.lexsort((_ranks(cd)[jj], _ranks(rd)[ii], _ranks(cu)[jj], _ranks(ru)[ii]))
            ii, jj = ii[order], jj[order]
        # W numerator = sigma * w_r * conj(w_c)
        a, b = rw[ii, 0], rw[ii, 1]
        c, d = cw[jj, 0], cw[jj, 1]
        cols["snk_u"].append(ru[ii])
        cols["src_u"].append(cu[jj])
        cols["snk_d"].append(rd[ii])
        cols["src_d"].append(cd[jj])
        cols["corr"].append(np.full(ii.shape[0], ci, dtype=np.int32))
        cols["re"].append(sig * (a * c + b * d))
        cols["im"].append(sig * (b * c - a * d))
    cat = {k: (np.concatenate(v) if v else np.zeros(0, dtype=np.int64)) for k, v in cols.items()}
    return IndexSet(nu, nd, cat["snk_u"], cat["src_u"], cat["snk_d"], cat["src_d"],
                    cat["corr"], cat["re"], cat["im"], dens)


def sink_tensor(op, spin=0, sign_mode="exact"):
    """Canonical sink tensor {(u_sorted, d_sorted): coef} of one operator."""
    terms, _ = operator_terms(op, spin, sign_mode)
    return canonical_tensor(flavour_separate(terms))

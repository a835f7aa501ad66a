"""Hadron blocks and block-level correlators (Sec. 2 and Sec. 3), FP64.

TEST INFRASTRUCTURE ONLY: like the rest of ``oracle``, nothing in the library
imports or calls this module.

A baryon block (Sec. 2) is the three-quark expectation of one sink baryon,
momentum projected over the sink points of a timeslice, with the three
source antiquark indices left open:

    f^h_p[t, alpha, A, Y, C] = sum_{x in t} e^{-i p.x} < h_alpha(x) q1bar(A) q2bar(Y) q1bar(C) >,

with (q1, q2) = (u, d) for the proton family and (d, u) for the neutron
family, h_alpha the baryon operator of Sec. 1 with open spin alpha, and the
antiquarks in the order of the paper's proton block (u, d, u).  Here the
expectation is taken by the brute-force Grassmann pairing sum of ``wick``.

The block-level correlator (Sec. 3, the expanded form of the general block
expression) places baryon i of every written product of the sink operator at
its own sink point x_i, projected to its own momentum p_i:

    C[t] = sum_{x_1..x_A in t} e^{-i sum_i p_i.x_i} < O_snk(x_1, .., x_A) Obar_src >,

with the source operator local at the (implicit) source point, written with
conjugated coefficients in the same field order as the sink (the reading used
throughout the oracle).  Wick's theorem splits every contraction by the set
partition of the source antiquarks among the baryons:

    < h_1 .. h_A qbar_1 .. qbar_n > = sum_P sign(P) (-1)^{A(A-1)/2} prod_i < h_i Qbar_i >,

Qbar_i the antiquarks of group i in block order, sign(P) the parity of
bringing qbar_1 .. qbar_n to Qbar_1 .. Qbar_A, and (-1)^{A(A-1)/2} that of
moving each (odd) group next to its (odd) baryon.  For D_I there are 3 x 3 = 9
partitions (the N_w = 9 terms of Sec. 3).

Readings where the paper is silent: baryon i of a written product sits at
sink point i (so the two products of D_II place p and n at opposite points);
site v of a timeslice has coordinates x1 + L1 (x2 + L2 x3) = v; a momentum is
an integer triple n with p.x = 2 pi sum_d n_d x_d / L_d.

``multiplicity_histogram`` is the Sec. 3 procedure behind Fig. 2: expand the
correlator into strings of block factors, order each string's factors
lexicographically by (hadron, momentum, source point, index bundle), and
count how often each distinct string occurs.
"""
from collections import Counter
from itertools import combinations, product as iproduct

import numpy as np

from . import operators as O
from . import wick
from .correlator import _dets

U, D = O.U, O.D

# block-order flavours of each baryon family: (q1, q2, q1)
_FLAV = {"p": (U, D, U), "n": (D, U, D)}


def kind_of(name):
    """(family "p"/"n", projector 0/+1/-1) of a baryon name of eq. "ops"."""
    return O._B[name]


def site_coords(dims):
    """[V, 3] integer coordinates of the sites of one timeslice (x1 fastest)."""
    L1, L2, L3 = dims
    v = np.arange(L1 * L2 * L3)
    return np.stack([v % L1, (v // L1) % L2, v // (L1 * L2)], axis=1)


def phases(mom, dims):
    """e^{-i p.x} per site of a timeslice, p = 2 pi n / L componentwise."""
    x = site_coords(dims)
    frac = sum(x[:, d] * mom[d] / dims[d] for d in range(3))
    return np.exp(-2j * np.pi * frac)


def _all_source_triples():
    a = np.arange(12)
    A, Y, C = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([A.ravel(), Y.ravel(), C.ravel()], axis=1)  # xi = (A*12 + Y)*12 + C


def _points(S):
    """Propagators as [P, T, V, 12, 12]: one set per source point (P = 1 for [T, V, 12, 12])."""
    return S[None] if S.ndim == 4 else S


def _projected(S_u, S_d, name, mom, dims, alpha, src, batch, sites=None, srcs=(0, 0, 0)):
    """[T, len(src)]: sum_x e^{-i p.x} < h_alpha(x) q1bar(A) q2bar(Y) q1bar(C) > for src rows (A, Y, C).

    ``sites``: optional flat site indices t*V + v to sum over (the others are
    taken to be zero); default every site.  ``srcs``: the source points of
    the three antiquarks (A, Y, C): a quark paired with antiquark k propagates
    from source point srcs[k].
    """
    S_u, S_d = _points(S_u), _points(S_d)
    T, V = S_u.shape[1:3]
    if V != dims[0] * dims[1] * dims[2]:
        raise ValueError("sites per timeslice do not match dims")
    kind, proj = kind_of(name)
    flav = _FLAV[kind]
    pairs = wick.pairings(flav, flav)
    ph = phases(mom, dims)
    S_of = {U: S_u.reshape(S_u.shape[0], T * V, 12, 12), D: S_d.reshape(S_d.shape[0], T * V, 12, 12)}
    terms = O.baryon_terms(kind, alpha, proj)
    coef = np.array([complex(c[0], c[1]) for c, _ in terms])
    snk = np.array([[i for _, i in f] for _, f in terms])
    out = np.zeros((T, src.shape[0]), dtype=np.complex128)
    every = np.arange(T * V) if sites is None else np.asarray(sites, dtype=np.int64)
    for s0 in range(0, every.shape[0], batch):
        sl = every[s0:s0 + batch]
        E = np.zeros((sl.shape[0], snk.shape[0], src.shape[0]), dtype=np.complex128)
        for pi, sgn in pairs:
            term = np.full(E.shape, float(sgn), dtype=np.complex128)
            for i, f in enumerate(flav):
                term *= S_of[f][srcs[pi[i]]][sl][:, snk[:, i][:, None], src[:, pi[i]][None, :]]
            E += term
        vals = np.einsum("r,brx->bx", coef, E)
        w = ph[sl % V]
        for t in np.unique(sl // V):
            m = (sl // V) == t
            out[t] += (w[m, None] * vals[m]).sum(axis=0)
    return out


def block(S_u, S_d, name, mom, dims, batch=16, sites=None, srcs=(0, 0, 0)):
    """f^h_p[t, alpha, xi] for baryon ``name``, xi = (A*12 + Y)*12 + C.

    S_u, S_d: [T, V, 12, 12] complex128 with V = L1 L2 L3, or [P, T, V, 12,
    12] for P source points, with ``srcs`` the source points of the
    antiquarks (A, Y, C).  Returns [T, 4, 1728] complex128.  Every entry is
    the pairing sum of ``wick`` over the baryon's written terms (Sec. 1),
    summed over sites with e^{-i p.x} (over the flat sites t*V + v listed in
    ``sites`` only, if given).
    """
    src = _all_source_triples()
    return np.stack([_projected(S_u, S_d, name, mom, dims, alpha, src, batch, sites, srcs) for alpha in range(4)],
                    axis=1)


def block_entries(S_u, S_d, name, mom, dims, entries, batch=512, srcs=(0, 0, 0)):
    """Selected block entries [T, len(entries)] for entries (alpha, A, Y, C).

    The same definition as ``block``, evaluated for a few entries only, so
    that large lattices stay cheap.
    """
    entries = [tuple(int(v) for v in e) for e in entries]
    out = np.zeros((_points(S_u).shape[1], len(entries)), dtype=np.complex128)
    for alpha in sorted({e[0] for e in entries}):
        cols = [k for k, e in enumerate(entries) if e[0] == alpha]
        src = np.array([entries[k][1:] for k in cols])
        out[:, cols] = _projected(S_u, S_d, name, mom, dims, alpha, src, batch, srcs=srcs)
    return out


def _labelled(terms, pts):
    """Written terms with field i of baryon slot i // 3 at source point pts[i // 3],
    encoded as index 12 * point + a (a field's point and index sort together)."""
    return [(c, tuple((f, 12 * pts[i // 3] + a) for i, (f, a) in enumerate(fl))) for c, fl in terms]


def _source_terms(op, spin, sign_mode, form, src_pts=None):
    """Source operator terms as (coef, flavours, indices, points), coefficients not yet conjugated.

    Baryon slot i of the source (written order) sits at source point
    src_pts[i] (default: every slot at point 0, a local source).
    form "raw": the written terms of eq. "ops" (fields in written order);
    form "canonical": the canonical keys (ubar..ubar dbar..dbar, each sorted
    by (point, index)), with the flavour-separation and sorting signs in the
    coefficient.  Both are the same Grassmann polynomial.
    """
    terms, _ = O.operator_terms(op, spin, sign_mode)
    A = len(terms[0][1]) // 3 if terms else 0
    pts = tuple(src_pts) if src_pts is not None else (0,) * A
    lab = _labelled(terms, pts)
    if form == "raw":
        return [(c, tuple(f for f, _ in fl), tuple(v % 12 for _, v in fl), tuple(v // 12 for _, v in fl))
                for c, fl in lab]
    if form != "canonical":
        raise ValueError(form)
    out = []
    for (u, d), c in sorted(O.canonical_tensor(O.flavour_separate(lab)).items()):
        v = tuple(u) + tuple(d)
        out.append((c, (U,) * len(u) + (D,) * len(d), tuple(x % 12 for x in v), tuple(x // 12 for x in v)))
    return out


def partitions(slot_kinds, src_flav):
    """Set partitions of the source antiquarks among the baryon slots.

    slot_kinds: families ("p"/"n") of the slots in written order; src_flav:
    flavours of the source antiquarks in their order.  Each partition is
    (groups, sign): groups[i] = positions (first q1, q2, second q1) of slot i's
    antiquarks in block order, sign = sign(P) (-1)^{A(A-1)/2}.
    """
    n = len(src_flav)
    A = len(slot_kinds)
    out = []

    def rec(i, free, groups):
        if i == A:
            seq = [p for g in groups for p in g]
            out.append((tuple(groups), O._perm_parity(seq) * (-1 if (A * (A - 1) // 2) & 1 else 1)))
            return
        q1, q2, _ = _FLAV[slot_kinds[i]]
        ones = [p for p in free if src_flav[p] == q1]
        twos = [p for p in free if src_flav[p] == q2]
        for a, c in combinations(ones, 2):
            for y in twos:
                rest = [p for p in free if p not in (a, y, c)]
                rec(i + 1, rest, groups + [(a, y, c)])

    if sum(3 for _ in slot_kinds) == n:
        rec(0, list(range(n)), [])
    return out


def block_correlator(S_u, S_d, op, snk_spin, src_spin, sign_mode, moms, dims, source="canonical",
                     blocks=None, src_pts=None, compute_missing=True):
    """C[t] of one block-level correlator, from blocks and the partition sum.

    moms: one integer momentum triple per sink baryon slot; src_pts: the
    source point of each source baryon slot (default all 0, a local source),
    with S_u, S_d [P, T, V, 12, 12] for P points.  ``blocks`` may hold
    precomputed {(name, mom, srcs): block(...)} arrays; a missing one is
    computed over every site, or raises KeyError if not compute_missing.
    Returns [T] complex128.
    """
    products, s2 = O.baryon_products(op, snk_spin, sign_mode)
    src = _source_terms(op, src_spin, sign_mode, source, src_pts)
    T = _points(S_u).shape[1]
    blocks = {} if blocks is None else blocks
    C = np.zeros(T, dtype=np.complex128)
    groups_of = {}
    for c, fl, idx, pts in src:
        groups_of.setdefault((fl, pts), []).append((c, idx))
    for coef_s, slots in products:
        if len(slots) != len(moms):
            raise ValueError("one momentum per baryon slot")
        names = [nm for nm, _ in slots]
        for (fl, pts), items in groups_of.items():
            cw = np.conj(np.array([complex(c[0], c[1]) for c, _ in items]))
            idx = np.array([i for _, i in items])
            for groups, sgn in partitions([kind_of(nm)[0] for nm in names], fl):
                prod = np.ones((T, len(items)), dtype=np.complex128)
                for i, (a, y, c) in enumerate(groups):
                    key = (names[i], tuple(moms[i]), (pts[a], pts[y], pts[c]))
                    if key not in blocks:
                        if not compute_missing:
                            raise KeyError(key)
                        blocks[key] = block(S_u, S_d, names[i], moms[i], dims, srcs=key[2])
                    xi = (idx[:, a] * 12 + idx[:, y]) * 12 + idx[:, c]
                    prod *= blocks[key][:, slots[i][1], xi]
                C += complex(coef_s[0], coef_s[1]) * sgn * (prod @ cw)
    return complex(s2) * C


def block_correlator_bruteforce(S_u, S_d, op, snk_spin, src_spin, sign_mode, moms, dims, src_pts=None):
    """The same correlator without blocks: sum over every tuple of sink points.

    For each (x_1, .., x_A) the sink fields of baryon slot i are labelled with
    x_i and the source fields of slot i with source point src_pts[i]; the
    expectation is taken in the determinant form, rows 12 i + a and columns
    12 p + a' of the stacked propagators S^(p)(x_i), summed with
    e^{-i sum_i p_i.x_i}.  Cost V^A determinant sums: tiny lattices only.
    """
    S_u, S_d = _points(S_u), _points(S_d)
    P = S_u.shape[0]
    terms, s2 = O.operator_terms(op, snk_spin, sign_mode)
    A = len(terms[0][1]) // 3
    if len(moms) != A:
        raise ValueError("one momentum per baryon slot")
    pts = tuple(src_pts) if src_pts is not None else (0,) * A
    snk = sorted(O.canonical_tensor(O.flavour_separate(_labelled(terms, tuple(range(A))))).items())
    src_terms, _ = O.operator_terms(op, src_spin, sign_mode)
    src = sorted(O.canonical_tensor(O.flavour_separate(_labelled(src_terms, pts))).items())
    T, V = S_u.shape[1:3]
    C = np.zeros(T, dtype=np.complex128)
    if not snk or not src:
        return C
    nu = len(snk[0][0][0])
    nd = len(snk[0][0][1])
    sig = O.grassmann_sigma(nu, nd)

    def uniq(keys):
        arr = np.array(keys, dtype=np.int64).reshape(len(keys), -1)
        u, inv = np.unique(arr, axis=0, return_inverse=True)
        return u, inv.reshape(-1)

    ru, iru = uniq([k[0] for k, _ in snk])
    rd, ird = uniq([k[1] for k, _ in snk])
    cu, icu = uniq([k[0] for k, _ in src])
    cd, icd = uniq([k[1] for k, _ in src])
    wr = np.array([complex(c[0], c[1]) for _, c in snk])
    wc = np.conj(np.array([complex(c[0], c[1]) for _, c in src]))
    ph = [phases(m, dims) for m in moms]

    def grid_dets(S, rows, cols):
        R = np.repeat(rows, cols.shape[0], axis=0)
        Cc = np.tile(cols, (rows.shape[0], 1))
        return _dets(S, R, Cc).reshape(rows.shape[0], cols.shape[0])

    def stacked(S, t, xs):
        # [12 A, 12 P]: block (i, p) = S^(p)(x_i)
        return np.concatenate([np.concatenate([S[p, t, x] for p in range(P)], axis=1) for x in xs], axis=0)

    for t in range(T):
        for xs in iproduct(range(V), repeat=A):
            Du = grid_dets(stacked(S_u, t, xs), ru, cu)[iru][:, icu]
            Dd = grid_dets(stacked(S_d, t, xs), rd, cd)[ird][:, icd]
            val = wr @ (Du * Dd) @ wc
            w = np.prod([ph[i][x] for i, x in enumerate(xs)])
            C[t] += w * val
    return complex(sig) * complex(s2) * C


def multiplicity_histogram(op, snk_spin, src_spin, sign_mode, moms=None, src_pts=None):
    """Sec. 3's multiplicity count of the expanded block-level correlator.

    Every term of the expansion (written source term x sink product x
    partition) is a string of block factors (hadron, momentum, source points,
    index bundle (A, Y, C, alpha)); the string's factors are put in
    lexicographic order and identical strings are counted.  Returns
    (n_terms, Counter{multiplicity: number of distinct strings}).
    """
    products, _ = O.baryon_products(op, snk_spin, sign_mode)
    src = _source_terms(op, src_spin, sign_mode, "raw", src_pts)
    A = len(products[0][1])
    moms = [(0, 0, 0)] * A if moms is None else [tuple(m) for m in moms]
    names = sorted(O._B)
    strings = Counter()
    n_terms = 0
    part_cache = {}
    for _, slots in products:
        kinds = tuple(kind_of(nm)[0] for nm, _ in slots)
        for _, fl, idx, pts in src:
            key = (kinds, fl)
            if key not in part_cache:
                part_cache[key] = partitions(list(kinds), fl)
            for groups, _ in part_cache[key]:
                fac = []
                for i, (a, y, c) in enumerate(groups):
                    nm, al = slots[i]
                    fac.append((names.index(nm), moms[i], (pts[a], pts[y], pts[c]), (idx[a], idx[y], idx[c], al)))
                strings[tuple(sorted(fac))] += 1
                n_terms += 1
    return n_terms, Counter(strings.values())

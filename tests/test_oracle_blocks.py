"""Pins of the oracle's hadron blocks and block-level correlators.

Each check takes a route that shares no step with the block construction:
the paper's explicit proton block formula (Sec. 2), the determinant-form
oracle at a single site (already pinned against brute-force Wick sums), a
site-labelled determinant brute force over every tuple of sink points, the
partition count N_w = 9 of D_I (Sec. 3), lattice translations, and exact
counting identities of the expansion.
"""
import numpy as np
import pytest

from oracle import blocks as B
from oracle import correlator as CO
from oracle import gamma as G
from oracle import operators as O
from paper_2201_04269_amd import synth


def _iset(op, s, sp, mode):
    return O.build_index_set([dict(op=op, snk_spin=s, src_spin=sp, sign_mode=mode)])


def test_proton_block_entries_equal_the_papers_formula():
    # f^P(a', beta', b', gamma', c', alpha')_alpha of Sec. 2, written out with
    # plain loops, against the oracle's pairing-sum block at one site.
    Su, Sd = synth.iid(1, 1, seed=21)
    f = B.block(Su, Sd, "p", (0, 0, 0), (1, 1, 1))[0]
    Gm = G.complex_of(G.cg5(0))
    eps = dict(O._levi_civita3())
    su, sd = Su[0, 0], Sd[0, 0]
    rng = np.random.default_rng(0)
    for _ in range(40):
        al, A, Y, C = (int(v) for v in rng.integers(0, [4, 12, 12, 12]))
        ref = 0j
        for (a, b, c), e in eps.items():
            for be in range(4):
                for ga in range(4):
                    if Gm[be, ga] == 0:
                        continue
                    ref += e * Gm[be, ga] * (su[4 * a + be, C] * su[4 * c + al, A]
                                             - su[4 * a + be, A] * su[4 * c + al, C]) * sd[4 * b + ga, Y]
        assert abs(f[al, (A * 12 + Y) * 12 + C] - ref) <= 1e-14 * max(1.0, abs(ref))


def test_blocks_are_antisymmetric_in_the_two_like_antiquarks():
    Su, Sd = synth.iid(1, 2, seed=22)
    for name in ("p", "n+", "p-"):
        f = B.block(Su, Sd, name, (1, 0, 0), (2, 1, 1)).reshape(1, 4, 12, 12, 12)
        assert np.allclose(f, -f.transpose(0, 1, 4, 3, 2), rtol=0, atol=1e-15)
        assert np.abs(np.einsum("taiyi->tay", f)).max() == 0.0


def test_block_momentum_phase_under_a_lattice_translation():
    # S'(x) = S(x + e_d) gives f'_p = e^{+2 pi i n_d / L_d} f_p: pins the site
    # order (x1 fastest) and the sign of the exponent together.
    dims = (3, 2, 2)
    Su, Sd = synth.iid(1, 12, seed=23)
    mom = (1, 1, 0)
    f = B.block(Su, Sd, "n", mom, dims)
    for axis, d in ((3, 0), (2, 1)):
        sh = [np.roll(S.reshape(1, 2, 2, 3, 12, 12), -1, axis=axis).reshape(1, 12, 12, 12) for S in (Su, Sd)]
        f2 = B.block(sh[0], sh[1], "n", mom, dims)
        assert np.allclose(f2, np.exp(2j * np.pi * mom[d] / dims[d]) * f, rtol=0, atol=1e-13)


@pytest.mark.parametrize("op,s,sp,mode", [("proton", 1, 2, "exact"), ("neutron", 3, 0, "exact"),
                                          ("DI", 0, 0, "exact"), ("DII", 0, 0, "r2"),
                                          ("HE3_I", 1, 1, "exact")])
def test_one_site_equals_the_local_determinant_form(op, s, sp, mode):
    # With one site per timeslice every baryon sits at the same point, so the
    # block-level correlator is eq. 1's local correlator.
    Su, Sd = synth.iid(2, 1, seed=24)
    A = 1 if op in ("proton", "neutron") else (2 if op.startswith("D") else 3)
    C = B.block_correlator(Su, Sd, op, s, sp, mode, [(0, 0, 0)] * A, (1, 1, 1))
    ref = CO.correlator(Su, Sd, _iset(op, s, sp, mode))[0]
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("op,moms,dims,T", [
    ("proton", [(1, 1, 0)], (2, 2, 1), 2),
    ("neutron", [(0, 1, 0)], (2, 2, 1), 2),
    ("DI", [(1, 0, 0), (0, 1, 0)], (2, 2, 1), 1),
    ("DI", [(1, 0, 0), (-1, 0, 0)], (2, 1, 1), 2),
])
def test_separate_sinks_equal_the_labelled_determinant_bruteforce(op, moms, dims, T):
    V = dims[0] * dims[1] * dims[2]
    Su, Sd = synth.iid(T, V, seed=25)
    C = B.block_correlator(Su, Sd, op, 2, 1, "exact", moms, dims)
    bf = B.block_correlator_bruteforce(Su, Sd, op, 2, 1, "exact", moms, dims)
    assert np.abs(C - bf).max() <= 1e-13 * np.abs(bf).max()


def test_three_baryons_at_two_points_equal_the_bruteforce():
    Su, Sd = synth.iid(1, 2, seed=26)
    moms = [(1, 0, 0), (0, 0, 0), (-1, 0, 0)]
    C = B.block_correlator(Su, Sd, "HE3_I", 1, 3, "exact", moms, (2, 1, 1))
    bf = B.block_correlator_bruteforce(Su, Sd, "HE3_I", 1, 3, "exact", moms, (2, 1, 1))
    assert abs(C[0] - bf[0]) <= 1e-13 * abs(bf[0])


def test_raw_and_canonical_source_forms_agree():
    Su, Sd = synth.iid(1, 2, seed=27)
    moms = [(1, 0, 0), (-1, 0, 0)]
    a = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (2, 1, 1), source="raw")
    b = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (2, 1, 1))
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0])


def test_dinucleon_has_nine_partitions_and_three_helium_three_sixty():
    # N_w = 9 for D_I (Sec. 3): 3 ways to give the proton two of the three
    # ubar, times 3 ways to give it one of the three dbar.
    for fl in [(O.U,) * 3 + (O.D,) * 3, (O.D, O.U, O.D, O.U, O.U, O.D)]:
        parts = B.partitions(["n", "p"], fl)
        assert len(parts) == 9
        assert len({g for g, _ in parts}) == 9
    # 3He (p-, n+, p+): 5!/(2! 1! 2!) u assignments x 4!/(1! 2! 1!) d assignments
    assert len(B.partitions(["p", "n", "p"], (O.U,) * 5 + (O.D,) * 4)) == 30 * 12


def test_exact_sign_dii_vanishes_and_r2_is_twice_di():
    Su, Sd = synth.iid(1, 2, seed=28)
    moms = [(1, 0, 0), (-1, 0, 0)]
    blocks = {}
    di = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (2, 1, 1), blocks=blocks)
    ex = B.block_correlator(Su, Sd, "DII", 0, 0, "exact", moms, (2, 1, 1), blocks=blocks)
    r2 = B.block_correlator(Su, Sd, "DII", 0, 0, "r2", moms, (2, 1, 1), blocks=blocks)
    assert ex[0] == 0
    assert abs(r2[0] - 2 * di[0]) <= 1e-13 * abs(di[0])


@pytest.mark.parametrize("op,mode,n_src,n_prod,n_part", [("DI", "exact", 2304, 4, 9),
                                                         ("DII", "r2", 4608, 8, 9)])
def test_multiplicity_histogram_counts(op, mode, n_src, n_prod, n_part):
    n, hist = B.multiplicity_histogram(op, 0, 0, mode)
    assert n == n_src * n_prod * n_part
    assert sum(m * k for m, k in hist.items()) == n
    assert min(hist) >= 1


def _two_points(T, V, seed):
    S = [synth.iid(T, V, seed=seed + p) for p in range(2)]
    return np.stack([s[0] for s in S]), np.stack([s[1] for s in S])


def test_displaced_sources_equal_the_labelled_bruteforce_and_revive_dii():
    # each source baryon at its own point (its own propagator set): the
    # partition sum with mixed-source blocks against the determinant brute
    # force with stacked (sink point, source point) propagators; exact-sign
    # D_II no longer vanishes, and swapping the two source points flips its sign
    Su, Sd = _two_points(1, 3, 70)
    moms = [(1, 0, 0), (-1, 0, 0)]
    dii = B.block_correlator(Su, Sd, "DII", 0, 0, "exact", moms, (3, 1, 1), src_pts=(0, 1))
    bf = B.block_correlator_bruteforce(Su, Sd, "DII", 0, 0, "exact", moms, (3, 1, 1), src_pts=(0, 1))
    assert abs(dii[0] - bf[0]) <= 1e-13 * abs(bf[0])
    assert abs(bf[0]) > 1.0
    swapped = B.block_correlator(Su, Sd, "DII", 0, 0, "exact", moms, (3, 1, 1), src_pts=(1, 0))
    assert abs(swapped[0] + dii[0]) <= 1e-13 * abs(dii[0])
    di = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (3, 1, 1), src_pts=(0, 1))
    di_bf = B.block_correlator_bruteforce(Su, Sd, "DI", 0, 0, "exact", moms, (3, 1, 1), src_pts=(0, 1))
    assert abs(di[0] - di_bf[0]) <= 1e-13 * abs(di_bf[0])
    raw = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (3, 1, 1), src_pts=(0, 1), source="raw")
    assert abs(raw[0] - di_bf[0]) <= 1e-13 * abs(di_bf[0])


def test_one_source_point_set_reproduces_the_local_source():
    Su, Sd = _two_points(2, 2, 72)
    moms = [(1, 0, 0), (-1, 0, 0)]
    a = B.block_correlator(Su[0], Sd[0], "DI", 0, 0, "exact", moms, (2, 1, 1))
    b = B.block_correlator(Su, Sd, "DI", 0, 0, "exact", moms, (2, 1, 1), src_pts=(0, 0))
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    # a mixed-source block is the plain block when every antiquark uses one set
    f = B.block(Su, Sd, "p", (1, 0, 0), (2, 1, 1), srcs=(1, 1, 1))
    g = B.block(Su[1], Sd[1], "p", (1, 0, 0), (2, 1, 1))
    assert np.array_equal(f, g)


# ---------------------------------------------------------------------------
# Multiplicity histogram (Sec. 3, Fig. 2): pins of the counting rule
# ---------------------------------------------------------------------------
# Non-zero entries (row, column) of C gamma5 in the Dirac basis (reading of
# Sec. 1's C gamma5: real, antisymmetric, one entry per row and column).
_CG5_PAIRS = {(0, 1), (1, 0), (2, 3), (3, 2)}


def test_multiplicity_histogram_of_the_proton_by_hand():
    # p^alpha's source expands into 6 colour permutations x 4 (beta', gamma')
    # entries of C gamma5 = 24 written terms, each with the one partition
    # (A, Y, C) = (ubar, dbar, ubar) in written order; the bundles
    # (4a'+beta', 4b'+gamma', 4c'+alpha') recover (a', b', c', beta', gamma'),
    # so all 24 strings are distinct
    for op in ("proton", "neutron"):
        n, hist = B.multiplicity_histogram(op, 0, 0, "exact")
        assert n == 24 and dict(hist) == {1: 24}


def test_multiplicity_histogram_of_di_by_inverting_the_expansion():
    """D_I's histogram counted the other way round: for every candidate string,
    the number of (source term, partition) pairs that produce it.

    A D_I term is a written source term nbar^{a'} pbar^{b'} (fields
    dbar ubar dbar | ubar dbar ubar at positions 0..5), a sink product (the
    n and p spins (alpha, beta), a C gamma5 entry) and a partition: the n
    block takes two of the three dbar (in position order, A and C) and one
    ubar (Y), the p block the other two ubar (A', C') and the last dbar (Y').
    Given a string (A, Y, C, A', Y', C'; alpha, beta) and a partition (which
    dbar k went to p, which ubar m went to n), the source term is fixed: it
    exists iff each source baryon's three colours are a permutation (eps),
    its first two spins are a C gamma5 pair, and the two source baryons'
    open spins are a C gamma5 pair.  A string's multiplicity is the number
    of the 9 partitions for which that holds.  The sink spins only label the
    string, so every sink product contributes the same counts.
    """
    from collections import Counter
    lab = np.indices((12,) * 6).reshape(6, -1)
    A, Y, Cc, A2, Y2, C2 = lab
    col, spin = lab // 4, lab % 4

    def pair_ok(s1, s2):
        ok = np.zeros(s1.shape, bool)
        for a, b in _CG5_PAIRS:
            ok |= (s1 == a) & (s2 == b)
        return ok

    def colours_ok(c1, c2, c3):
        return (c1 != c2) & (c1 != c3) & (c2 != c3)

    mult = np.zeros(A.shape, np.int64)
    for k in range(3):          # the dbar that went to the p block (as Y')
        for m in range(3):      # the ubar that went to the n block (as Y)
            d = [None] * 3
            d[k] = Y2
            rest = iter((A, Cc))
            for q in range(3):
                if q != k:
                    d[q] = next(rest)
            u = [None] * 3
            u[m] = Y
            rest = iter((A2, C2))
            for q in range(3):
                if q != m:
                    u[q] = next(rest)
            # written source: nbar = dbar(d0) ubar(u0) dbar(d1), pbar = ubar(u1) dbar(d2) ubar(u2)
            ok = colours_ok(d[0] // 4, u[0] // 4, d[1] // 4) & pair_ok(d[0] % 4, u[0] % 4)
            ok &= colours_ok(u[1] // 4, d[2] // 4, u[2] // 4) & pair_ok(u[1] % 4, d[2] % 4)
            ok &= pair_ok(d[1] % 4, u[2] % 4)
            mult += ok
    per_product = Counter(mult[mult > 0].tolist())
    expect = Counter({m: len(_CG5_PAIRS) * c for m, c in per_product.items()})
    n, hist = B.multiplicity_histogram("DI", 0, 0, "exact")
    assert n == sum(m * c for m, c in expect.items()) == 82944
    assert dict(hist) == dict(expect)
    assert max(hist) == 9  # every partition of one string


@pytest.mark.slow
def test_multiplicity_histogram_of_dii_is_sign_free_and_symmetric():
    # the counting key carries no sign: exact and R2 signs give one histogram;
    # the key is sorted: product (p, n) of every term has a twin from
    # product (n, p) with the same factors (the slots' blocks swapped), so
    # every multiplicity is even
    n1, h1 = B.multiplicity_histogram("DII", 0, 0, "exact")
    n2, h2 = B.multiplicity_histogram("DII", 0, 0, "r2")
    assert n1 == n2 and h1 == h2
    assert all(m % 2 == 0 for m in h1)

"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses an independent
route (the paper's explicit proton block formula, a brute-force Grassmann
Wick sum that never sorts or separates flavours, group invariances, exact
homogeneity, closed forms at S = I derived by hand, finite differences).
"""
import numpy as np
import pytest

from oracle import correlator as CO
from oracle import gamma as G
from oracle import operators as O
from oracle import wick
from paper_2201_04269_amd import synth


def cplx(p):
    return G.complex_of(p)


def one_site(S):
    return S.reshape(1, 1, 12, 12)


def iset_of(op, spin=0, src_spin=None, mode="exact", sym=True):
    return O.build_index_set([dict(op=op, snk_spin=spin,
                                   src_spin=spin if src_spin is None else src_spin,
                                   sign_mode=mode, symmetrise=sym)])


# ---------------------------------------------------------------------------
# Dirac basis (reading of Sec. 1's C gamma5, P+-)
# ---------------------------------------------------------------------------
def test_dirac_basis_clifford_and_charge_conjugation():
    g = {k: cplx(v) for k, v in G.gamma_matrices().items()}
    C = cplx(G.charge_conjugation())
    Ci = np.linalg.inv(C)
    I4 = np.eye(4)
    for mu in (1, 2, 3, 4):
        assert np.allclose(C @ g[mu] @ Ci, -g[mu].T)
        assert np.allclose(g[mu] @ g[5] + g[5] @ g[mu], 0)
        for nu in (1, 2, 3, 4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * I4 * (mu == nu))
    assert np.allclose(g[5] @ g[5], I4)
    cg5 = cplx(G.cg5(0))
    # antisymmetry of C gamma5 is what makes D_II and 3He_II vanish locally
    assert np.array_equal(cg5, -cg5.T)
    expected = np.array([[0, -1, 0, 0], [1, 0, 0, 0], [0, 0, 0, -1], [0, 0, 1, 0]])
    assert np.array_equal(cg5, expected)
    for s in (+1, -1):
        P = (I4 + s * g[4]) / 2
        assert np.array_equal(cplx(G.cg5(s)), cg5 @ P)
        assert np.allclose(cg5 @ P, P @ cg5 @ P)


# ---------------------------------------------------------------------------
# Proton: the explicit two-term block formula of Sec. 2
# ---------------------------------------------------------------------------
def proton_block_formula(Su, Sd, alpha, alpha_p):
    """<p_alpha pbar_alpha'> from the proton block formula of Sec. 2.

    f^P(a', beta', b', gamma', c', alpha')_alpha =
      eps^{abc} Gamma_{beta gamma} [S^u_{(a beta)(c' alpha')} S^u_{(c alpha)(a' beta')}
                                   - S^u_{(a beta)(a' beta')} S^u_{(c alpha)(c' alpha')}]
                                   S^d_{(b gamma)(b' gamma')}
    contracted with the source's eps_{a'b'c'} conj(Gamma_{beta' gamma'}).
    Written with plain loops; shares nothing with the determinant form.
    """
    Gm = cplx(G.cg5(0))
    eps = {p: s for p, s in O._levi_civita3()}
    tot = 0.0 + 0.0j
    for (a, b, c), e in eps.items():
        for beta in range(4):
            for gam in range(4):
                if Gm[beta, gam] == 0:
                    continue
                for (ap, bp, cp), ep in eps.items():
                    for betap in range(4):
                        for gamp in range(4):
                            if Gm[betap, gamp] == 0:
                                continue
                            u1 = (Su[4 * a + beta, 4 * cp + alpha_p] * Su[4 * c + alpha, 4 * ap + betap]
                                  - Su[4 * a + beta, 4 * ap + betap] * Su[4 * c + alpha, 4 * cp + alpha_p])
                            f = e * Gm[beta, gam] * u1 * Sd[4 * b + gam, 4 * bp + gamp]
                            tot += ep * np.conj(Gm[betap, gamp]) * f
    return tot


def test_proton_identity_closed_form_is_minus_30():
    # By hand from the block formula at S = 1 (alpha = alpha' = 0): the
    # second term gives -(6 colour perms)(4 non-zero Gamma entries) = -24 and
    # the first gives eps_abc eps_cba (sum_gamma Gamma_0gamma^2) = -6.
    I = np.eye(12, dtype=complex)
    assert proton_block_formula(I, I, 0, 0) == pytest.approx(-30)
    C = CO.correlator(one_site(I), one_site(I), iset_of("proton"))
    assert C[0, 0] == pytest.approx(-30, abs=1e-12)
    terms, s2 = O.operator_terms("proton", 0)
    assert wick.correlator_bruteforce(I, I, terms, s2) == pytest.approx(-30)


@pytest.mark.parametrize("alpha,alpha_p", [(0, 0), (1, 3), (2, 2)])
def test_proton_det_form_equals_block_formula(alpha, alpha_p):
    Su, Sd = synth.iid(1, 1, seed=11 + alpha)
    C = CO.correlator(Su, Sd, iset_of("proton", alpha, alpha_p))[0, 0]
    ref = proton_block_formula(Su[0, 0], Sd[0, 0], alpha, alpha_p)
    assert abs(C - ref) <= 1e-13 * max(1.0, abs(ref))


# ---------------------------------------------------------------------------
# Determinant form vs brute-force Grassmann Wick sum (no sorting, no sigma)
# ---------------------------------------------------------------------------
def test_bruteforce_wick_proton_random_and_neutron():
    Su, Sd = synth.iid(1, 1, seed=3)
    for op in ("proton", "neutron"):
        terms, s2 = O.operator_terms(op, 1)
        bf = wick.correlator_bruteforce(Su[0, 0], Sd[0, 0], terms, s2)
        C = CO.correlator(Su, Sd, iset_of(op, 1))[0, 0]
        assert abs(C - bf) <= 1e-13 * abs(bf)


@pytest.mark.slow
def test_bruteforce_wick_dinucleon_full_sum():
    # 2304 x 2304 raw term pairs x 3!3! pairings at one site
    Su, Sd = synth.su3_spin(1, 1, seed=5)
    terms, s2 = O.operator_terms("DI")
    bf = wick.correlator_bruteforce(Su[0, 0], Sd[0, 0], terms, s2)
    C = CO.correlator(Su, Sd, iset_of("DI"))[0, 0]
    assert abs(C - bf) <= 1e-12 * abs(bf)
    # at S = 1 the brute force gives the closed form sigma * sum |w|^2
    I = np.eye(12, dtype=complex)
    assert wick.correlator_bruteforce(I, I, terms, s2).real == pytest.approx(-4320)


@pytest.mark.parametrize("op,spin,mode", [("HE3_I", 0, "exact"), ("HE3_I", 3, "exact"),
                                          ("HE3_II", 2, "r2"), ("DII", 0, "r2")])
def test_bruteforce_wick_termwise_sign(op, spin, mode):
    """Per raw term pair: Wick sum == sigma * flavour signs * det_u * det_d."""
    rng = np.random.default_rng(7)
    Su, Sd = synth.iid(1, 1, seed=8)
    Su, Sd = Su[0, 0], Sd[0, 0]
    terms, _ = O.operator_terms(op, spin, mode)
    pick = rng.choice(len(terms), size=6, replace=False)
    sep = O.flavour_separate([terms[p] for p in pick])
    nu, nd = O.quark_counts(op)
    sig = O.grassmann_sigma(nu, nd)
    for r in range(len(pick)):
        for c in range(len(pick)):
            sr = sep[r][0][0] * terms[pick[r]][0][0] + sep[r][0][1] * terms[pick[r]][0][1]
            sc = sep[c][0][0] * terms[pick[c]][0][0] + sep[c][0][1] * terms[pick[c]][0][1]
            # flavour-separation sign of each term = sep coef / original coef
            nr = terms[pick[r]][0][0] ** 2 + terms[pick[r]][0][1] ** 2
            ncc = terms[pick[c]][0][0] ** 2 + terms[pick[c]][0][1] ** 2
            fr, fc = sr // nr, sc // ncc
            E = wick.wick_pairs((Su, Sd), [f for f, _ in terms[pick[r]][1]],
                                [[i for _, i in terms[pick[r]][1]]],
                                [f for f, _ in terms[pick[c]][1]],
                                [[i for _, i in terms[pick[c]][1]]])[0, 0]
            du = np.linalg.det(Su[np.ix_(sep[r][1], sep[c][1])])
            dd = np.linalg.det(Sd[np.ix_(sep[r][2], sep[c][2])])
            assert abs(E - sig * fr * fc * du * dd) <= 1e-14 * max(1e-3, abs(E))


def test_identity_closed_forms_bruteforce():
    """C(S = 1) = sigma s^2 sum|w|^2; brute force on the written operator."""
    I = np.eye(12, dtype=complex)
    expected = {("proton", 0, "exact"): -30, ("DI", 0, "exact"): -4320,
                ("HE3_I", 0, "exact"): 8064, ("HE3_I", 2, "exact"): 4608,
                ("DII", 0, "r2"): -8640, ("HE3_II", 0, "r2"): 15168, ("HE3_II", 2, "r2"): 20160,
                ("DII", 0, "exact"): 0, ("HE3_II", 1, "exact"): 0}
    for (op, spin, mode), val in expected.items():
        C = CO.correlator(one_site(I), one_site(I), iset_of(op, spin, mode=mode))
        if val == 0:
            assert C.shape[1] == 1 and np.all(C == 0)
        else:
            assert C[0, 0] == pytest.approx(val, abs=1e-9)
        # homogeneity at S = lambda * 1
        nu, nd = O.quark_counts(op)
        if val:
            C2 = CO.correlator(one_site(2 * I), one_site(3 * I), iset_of(op, spin, mode=mode))
            assert C2[0, 0] == pytest.approx(val * 2 ** nu * 3 ** nd, rel=1e-12)


# ---------------------------------------------------------------------------
# Appendix-C statement: D_II and 3He_II vanish at a local sink
# ---------------------------------------------------------------------------
def test_two_exact_sign_operators_have_empty_canonical_sets():
    assert O.sink_tensor("DII") == {}
    for j in range(4):
        assert O.sink_tensor("HE3_II", j) == {}
    # the raw (unsymmetrised) written expansions are not empty: the cancellation
    # happens between terms, exactly as the Grassmann argument says
    for op, n in (("DII", 4608), ("HE3_II", 41472)):
        assert len(O.flavour_separate(O.operator_terms(op, 0)[0])) == n


# ---------------------------------------------------------------------------
# Symmetries of the colour-singlet operators, homogeneity, raw == canonical
# ---------------------------------------------------------------------------
def _colour_rotate(S, g, h):
    G12 = np.kron(g, np.eye(4))
    H12 = np.kron(h, np.eye(4))
    return G12 @ S @ H12.conj().T


@pytest.mark.parametrize("op,spin,mode", [("proton", 0, "exact"), ("DI", 0, "exact"),
                                          ("HE3_I", 1, "exact"), ("HE3_II", 3, "r2")])
def test_colour_rotation_invariance(op, spin, mode):
    Su, Sd = synth.iid(1, 2, seed=4)
    iset = iset_of(op, spin, mode=mode)
    C0 = CO.site_values(Su[0], Sd[0], iset)
    g = synth.random_su3(2, seed=9)
    Su2 = np.stack([_colour_rotate(Su[0, v], g[0], g[1]) for v in range(2)])
    Sd2 = np.stack([_colour_rotate(Sd[0, v], g[0], g[1]) for v in range(2)])
    C1 = CO.site_values(Su2, Sd2, iset)
    A = CO.sum_abs_terms(Su, Sd, iset).sum()
    assert np.max(np.abs(C1 - C0)) <= 1e-13 * A
    assert np.max(np.abs(C0)) > 1e-6 * A  # not trivially zero


def test_homogeneity_random():
    Su, Sd = synth.iid(1, 1, seed=6)
    for op, spin in (("proton", 0), ("DI", 0)):
        iset = iset_of(op, spin)
        nu, nd = iset.nu, iset.nd
        C0 = CO.correlator(Su, Sd, iset)
        lam, mu = 1.7 - 0.4j, -0.8 + 0.3j
        C1 = CO.correlator(lam * Su, mu * Sd, iset)
        assert np.allclose(C1, lam ** nu * mu ** nd * C0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("op", ["proton", "DI"])
def test_raw_equals_canonical(op):
    Su, Sd = synth.iid(1, 1, seed=12)
    Cc = CO.correlator(Su, Sd, iset_of(op))
    Cr = CO.correlator(Su, Sd, iset_of(op, sym=False))
    A = CO.sum_abs_terms(Su, Sd, iset_of(op))
    assert np.max(np.abs(Cc - Cr)) <= 1e-13 * A.max()


# ---------------------------------------------------------------------------
# Sum of |Wick terms| (permanents)
# ---------------------------------------------------------------------------
def test_permanent_pins():
    A = np.ones((1, 4, 4))
    assert CO._permanents(A)[0] == 24
    M = np.array([[[1.0, 2.0], [3.0, 4.0]]])
    assert CO._permanents(M)[0] == 1 * 4 + 2 * 3
    # a permutation matrix has permanent 1
    P = np.eye(5)[[2, 0, 4, 1, 3]][None]
    assert CO._permanents(P)[0] == 1


def test_sum_abs_terms_bounds_and_scaling():
    Su, Sd = synth.iid(1, 2, seed=13)
    iset = iset_of("DI")
    A = CO.sum_abs_terms(Su, Sd, iset)
    C = CO.correlator(Su, Sd, iset)
    assert np.all(A >= np.abs(C))
    A2 = CO.sum_abs_terms(2 * Su, 3 * Sd, iset)
    assert np.allclose(A2, 2 ** 3 * 3 ** 3 * A, rtol=1e-12)
    I = np.eye(12, dtype=complex)
    AI = CO.sum_abs_terms(one_site(I), one_site(I), iset)
    assert AI[0, 0] == pytest.approx(4320)  # every surviving term is a diagonal


# ---------------------------------------------------------------------------
# Gradients: finite differences, linearity in W, Euler's identity
# ---------------------------------------------------------------------------
def _loss(Su, Sd, iset, v, W=None):
    if W is not None:
        iset = _with_weights(iset, W)
    return np.real(np.sum(np.conj(v) * CO.correlator(Su, Sd, iset)))


def _with_weights(iset, W):
    """Copy of an index set whose weights are the given complex values."""
    cp = O.IndexSet(iset.nu, iset.nd, iset.snk_u, iset.src_u, iset.snk_d, iset.src_d,
                    iset.corr_id, np.zeros(iset.nnz), np.zeros(iset.nnz), iset.w_den)
    cp.weights = lambda: W
    return cp


@pytest.mark.parametrize("op", ["proton", "DI"])
def test_gradients_central_differences(op):
    T, V = 2, 1
    Su, Sd = synth.iid(T, V, seed=21)
    iset = iset_of(op)
    rng = np.random.default_rng(22)
    v = rng.standard_normal((1, T)) + 1j * rng.standard_normal((1, T))
    g = CO.gradients(Su, Sd, iset, v)
    h = 1e-4
    for name in ("S_u", "S_d"):
        E = rng.standard_normal(Su.shape) + 1j * rng.standard_normal(Su.shape)
        if name == "S_u":
            lp, lm = _loss(Su + h * E, Sd, iset, v), _loss(Su - h * E, Sd, iset, v)
        else:
            lp, lm = _loss(Su, Sd + h * E, iset, v), _loss(Su, Sd - h * E, iset, v)
        fd = (lp - lm) / (2 * h)
        an = np.real(np.sum(np.conj(g[name]) * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), name
    # W: C is linear in W, so the difference quotient is exact up to rounding
    W = iset.weights()
    dW = rng.standard_normal(W.shape) + 1j * rng.standard_normal(W.shape)
    fd = (_loss(Su, Sd, iset, v, W + h * dW) - _loss(Su, Sd, iset, v, W - h * dW)) / (2 * h)
    an = np.real(np.sum(np.conj(g["W"]) * dW))
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_gradient_euler_identity():
    """sum S dC/dS = n_f C for each flavour (C homogeneous of degree n_f)."""
    T, V = 2, 2
    Su, Sd = synth.su3_spin(T, V, seed=31)
    iset = iset_of("DI")
    C = CO.correlator(Su, Sd, iset)
    for t in range(T):
        e = np.zeros((1, T), dtype=complex)
        e[0, t] = 1.0
        g = CO.gradients(Su, Sd, iset, e, want=("S_u", "S_d"))
        for name, S, n in (("S_u", Su, iset.nu), ("S_d", Sd, iset.nd)):
            # with grad_C = e_t the returned gradient is conj(dC[t]/dS)
            val = np.sum(S[t] * np.conj(g[name][t]))
            assert abs(val - n * C[0, t]) <= 1e-11 * abs(C[0, t])
            others = [u for u in range(T) if u != t]
            assert np.all(g[name][others] == 0)


def test_gradient_w_equals_site_products():
    Su, Sd = synth.iid(2, 2, seed=41)
    iset = iset_of("proton")
    gC = np.array([[1.0 + 2.0j, -0.5j]])
    gW = CO.gradients(Su, Sd, iset, gC, want=("W",))["W"]
    # brute per entry, per site
    ref = np.zeros(iset.nnz, dtype=complex)
    for t in range(2):
        for v in range(2):
            for k in range(iset.nnz):
                du = np.linalg.det(Su[t, v][np.ix_(iset.snk_u[k], iset.src_u[k])])
                dd = np.linalg.det(Sd[t, v][np.ix_(iset.snk_d[k], iset.src_d[k])])
                ref[k] += gC[0, t] * np.conj(du * dd)
    assert np.allclose(gW, ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# Gradient scales (the tolerance of every gradient parity test)
# ---------------------------------------------------------------------------
def _monomial_gradient_scales(Su, Sd, iset, gC):
    """Sum of |monomial| derivatives at one site, by explicit enumeration.

    Every canonical entry k expands (eq. 1 with Leibniz's formula for both
    determinants) into the monomials W_k sgn(pu) sgn(pd) prod_i S_u[ru_i, cu_pu(i)]
    prod_i S_d[rd_i, cd_pd(i)], one per pair of permutations (pu, pd).  With
    every sign dropped, the scale of a gradient entry is the sum over the
    monomials that contain that propagator entry of |g| |W_k| times the
    magnitudes of the monomial's other factors; the scale of grad_W[k] is the
    sum of |g| times the magnitudes of all factors of entry k's monomials.
    No permanent and no cofactor is formed here.
    """
    from itertools import permutations
    aSu, aSd = np.abs(Su), np.abs(Sd)
    ag = np.abs(gC[iset.corr_id, 0])
    aW = np.abs(iset.weights())
    nu, nd = iset.nu, iset.nd
    out_W = np.zeros(iset.nnz)
    out_u = np.zeros(144)
    out_d = np.zeros(144)
    for pu in permutations(range(nu)):
        fu = [aSu[iset.snk_u[:, i], iset.src_u[:, pu[i]]] for i in range(nu)]
        for pd in permutations(range(nd)):
            fd = [aSd[iset.snk_d[:, i], iset.src_d[:, pd[i]]] for i in range(nd)]
            allf = fu + fd
            out_W += ag * np.prod(allf, axis=0)
            for slot in range(nu + nd):
                rest = ag * aW * np.prod([f for q, f in enumerate(allf) if q != slot], axis=0)
                if slot < nu:
                    flat = iset.snk_u[:, slot] * 12 + iset.src_u[:, pu[slot]]
                    out_u += np.bincount(flat, weights=rest, minlength=144)
                else:
                    i = slot - nu
                    flat = iset.snk_d[:, i] * 12 + iset.src_d[:, pd[i]]
                    out_d += np.bincount(flat, weights=rest, minlength=144)
    return out_W, out_u.reshape(12, 12), out_d.reshape(12, 12)


@pytest.mark.parametrize("op", ["proton", "neutron", "DI"])
def test_gradient_abs_scales_equal_the_monomial_enumeration(op):
    # catches, in gradient_abs_scales: a dropped |W| or |g|, the other
    # flavour's permanent taken from the wrong flavour, a transposed
    # (source, sink) flat index, or a cofactor permanent of the wrong minor
    Su, Sd = synth.iid(1, 1, seed=91)
    iset = iset_of(op)
    gC = np.array([[0.7 - 1.3j]])
    got = CO.gradient_abs_scales(Su, Sd, iset, gC)
    ref_W, ref_u, ref_d = _monomial_gradient_scales(Su[0, 0], Sd[0, 0], iset, gC)
    assert np.allclose(got["W"], ref_W, rtol=1e-12, atol=0)
    assert np.allclose(got["S_u"][0, 0], ref_u, rtol=1e-12, atol=0)
    assert np.allclose(got["S_d"][0, 0], ref_d, rtol=1e-12, atol=0)
    # and each scale bounds its gradient entry (every term counted by magnitude)
    g = CO.gradients(Su, Sd, iset, gC)
    for name in ("W", "S_u", "S_d"):
        assert np.all(np.abs(g[name]) <= got[name] * (1 + 1e-12) + 1e-300)

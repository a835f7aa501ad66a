"""GPU parity on populated lattices and on the 3He batch's backward at its
full shape.

Expected values come from tests/golden/populated.json, written by
tests/golden/make_populated.py from the FP64 oracle over every populated site
(the neutron case runs the oracle here: its index set is small).  Unlike the
sampled-site tests, thousands of live sites feed the compensated per-chunk
sums and the fixed-order cross-chunk reductions:
  * D_I on all 8192 sites of 8^3 x 16 (SU(3) x spin propagators);
  * a fully populated 4^3 x 4 block inside the 16^3 x 32 launch, forward for
    D_II (exact and R2) and D_I, and forward and gradients for the mixed
    weights W_DI + 0.5 W_DII(R2);
  * the 8 3He correlators: a populated 4^3 block at t = 0 of 32^3 x 8 (forward),
    and every site of 32^3 x 8 populated for the gradients (sampled sites of
    grad_S; sampled entries of grad_W, each summed over all 262144 sites);
  * the neutron (n_u, n_d) = (1, 2) family, forward and backward.
Tolerances as in tests/parity.py; each FP64 check prints which term of its
bound applied.
"""
import json
import os

import numpy as np
import pytest

from oracle import correlator as CO
from oracle import operators as O
from paper_2201_04269_amd import synth
from tests.parity import f64_branch, kappa, tol_f32c, tol_f64

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "populated.json")
HE3 = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
      [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _c(a):
    a = np.asarray(a)
    return a[..., 0] + 1j * a[..., 1]


def _api():
    from paper_2201_04269_amd import api
    return api


def block_sites(L, n):
    return [x + L * (y + L * z) for z in range(n) for y in range(n) for x in range(n)]


def keep_block(Su, Sd, ts, sites):
    mask = np.zeros(Su.shape[:2], dtype=bool)
    for t in ts:
        mask[t, sites] = True
    Su, Sd = Su.copy(), Sd.copy()
    Su[~mask] = 0
    Sd[~mask] = 0
    return Su, Sd


def check(C, ref, A, nu, nd, prec, label):
    C, ref, A = np.asarray(C), np.asarray(ref), np.asarray(A)
    err = np.abs(C - ref)
    tol = tol_f64(ref, A, nu, nd) if prec == "f64" else tol_f32c(A, nu, nd)
    msg = f"{label} {prec}: max |err|/A = {float(np.max(err / np.maximum(A, 1e-300))):.3e}"
    if prec == "f64":
        msg += "; " + f64_branch(ref, A, nu, nd)
    print(msg, flush=True)
    assert np.all(err <= tol + 1e-300), label


def grad_tol(ref, scale, nu, nd, prec):
    u = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    tol = kappa(nu, nd) * u * np.asarray(scale)
    if prec == "f64":
        tol = np.maximum(tol, 1e-12 * np.abs(ref))
    return tol


def forward(ods, Su, Sd, prec, W=None):
    api = _api()
    plan = api.Plan(api.IndexSet(ods), prec)
    su, sd = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda()
    C = api.contract(plan, su, sd, None if W is None else torch.from_numpy(W).cuda())
    return C.cpu().numpy()


def mixed_weights():
    api = _api()
    both = api.IndexSet([dict(op="DI"), dict(op="DII", sign_mode="r2")])
    w = both.weights()
    n = both.nnz // 2
    return w[:n] + 0.5 * w[n:]


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_dinucleon_8x8x8x16_every_site(prec):
    g = _gold()["di8"]
    Su, Sd = synth.su3_spin(g["T"], g["V"], seed=g["seed"])
    C = forward([dict(op="DI")], Su, Sd, prec)
    check(C[0], _c(g["C"]), g["A"], 3, 3, prec, "D_I 8^3x16, 8192 sites")


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_dinucleon_populated_block_in_16x16x16x32(prec):
    g = _gold()["di_block"]
    L, T = g["L"], g["T"]
    Su, Sd = synth.iid(T, L ** 3, seed=g["seed"])
    Su, Sd = keep_block(Su, Sd, range(4), block_sites(L, g["block"]))
    ods = [dict(op="DII"), dict(op="DII", sign_mode="r2"), dict(op="DI")]
    C = forward(ods, Su, Sd, prec)
    assert np.all(C[0] == 0)            # exact-sign D_II vanishes identically
    assert np.all(C[:, 4:] == 0)        # empty timeslices
    ref = _c(g["di_block"]["C"]).T      # [corr, t]
    A = np.asarray(g["di_block"]["A"]).T
    check(C[1:, :4], ref[1:], A[1:], 3, 3, prec, "D_II(R2)/D_I, 256-site block")
    # config 4's mixed weights on D_I's index set
    C = forward([dict(op="DI")], Su, Sd, prec, W=mixed_weights())
    check(C[0, :4], _c(g["di_mixed"]["C"])[:, 0], np.asarray(g["di_mixed"]["A"])[:, 0], 3, 3, prec,
          "W_DI + 0.5 W_DII(R2), 256-site block")


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_dinucleon_populated_block_gradients(prec):
    api = _api()
    g = _gold()["di_block"]
    gg = g["grad"]
    L, T = g["L"], g["T"]
    sites = block_sites(L, g["block"])
    Su, Sd = synth.iid(T, L ** 3, seed=g["seed"])
    Su, Sd = keep_block(Su, Sd, range(4), sites)
    W = mixed_weights()
    gC = _c(gg["gC"])
    plan = api.Plan(api.IndexSet([dict(op="DI")]), prec)
    gW, gSu, gSd = api.contract_backward(plan, torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(),
                                         torch.from_numpy(W).cuda(), torch.from_numpy(gC).cuda())
    gW, gSu, gSd = gW.cpu().numpy(), gSu.cpu().numpy(), gSd.cpu().numpy()
    ent = np.asarray(gg["entries"])
    ref, scl = _c(gg["gW"]), np.asarray(gg["sW"])
    err = np.abs(gW[ent] - ref)
    print(f"block grad_W {prec}: max |err|/scale = {float(np.max(err / scl)):.3e}", flush=True)
    assert np.all(err <= grad_tol(ref, scl, 3, 3, prec) + 1e-300)
    # every entry at once: sum_k W_k conj(grad_W_k)
    dot, dscl = _c(gg["grad_W_dot"]), gg["grad_W_dot_scale"]
    assert abs(np.sum(W * np.conj(gW)) - dot) <= grad_tol(dot, dscl, 3, 3, prec)
    for (t, v), rSu, rSd, sSu, sSd in zip(gg["sites"], gg["gSu"], gg["gSd"], gg["sSu"], gg["sSd"]):
        for got, r, s in ((gSu[t, v], _c(rSu), np.asarray(sSu)), (gSd[t, v], _c(rSd), np.asarray(sSd))):
            assert np.all(np.abs(got - r) <= grad_tol(r, s, 3, 3, prec) + 1e-300), (prec, t, v)
    outside = np.ones(Su.shape[:2], dtype=bool)
    outside[:4][:, sites] = False
    assert np.all(gSu[outside] == 0) and np.all(gSd[outside] == 0)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_helium3_populated_block_forward(prec):
    g = _gold()["he3_block"]
    L, T = g["L"], g["T"]
    Su, Sd = synth.iid(T, L ** 3, seed=g["seed"])
    Su, Sd = keep_block(Su, Sd, [0], block_sites(L, g["block"]))
    C = forward(HE3, Su, Sd, prec)
    assert np.all(C[:, 1:] == 0)
    check(C[:, 0], _c(g["C"]), g["A"], 5, 4, prec, "3He batch, 64-site block of 32^3x8")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["f32c", "f64"])
def test_helium3_batch_gradients_32x32x32x8_every_site(prec):
    """Config 5's backward: the 8 3He correlators in one launch on 32^3 x 8,
    every site populated; grad_S at 3 sampled sites and grad_W at 2 sampled
    entries per correlator (each a sum over all 262144 sites)."""
    api = _api()
    g = _gold()["he3_grad"]
    L, T = g["L"], g["T"]
    Su, Sd = synth.iid(T, L ** 3, seed=g["seed"])
    plan = api.Plan(api.IndexSet(HE3), prec)
    gC = _c(g["gC"])
    su, sd, gc = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(), torch.from_numpy(gC).cuda()
    print(f"3He batch backward {prec} on 32^3x8: grad_W", flush=True)
    gW, _, _ = api.contract_backward(plan, su, sd, None, gc, need_W=True, need_S=False)
    gW = gW.cpu().numpy()
    print(f"3He batch backward {prec} on 32^3x8: grad_S", flush=True)
    _, gSu, gSd = api.contract_backward(plan, su, sd, None, gc, need_W=False, need_S=True)
    gSu, gSd = gSu.cpu().numpy(), gSd.cpu().numpy()
    ent = np.asarray(g["entries"])
    ref, scl = _c(g["gW"]), np.asarray(g["sW"])
    err = np.abs(gW[ent] - ref)
    print(f"3He batch grad_W {prec}: max |err|/scale = {float(np.max(err / scl)):.3e}", flush=True)
    assert np.all(err <= grad_tol(ref, scl, 5, 4, prec) + 1e-300)
    worst = 0.0
    for (t, v), rSu, rSd, sSu, sSd in zip(g["sites"], g["gSu"], g["gSd"], g["sSu"], g["sSd"]):
        for got, r, s in ((gSu[t, v], _c(rSu), np.asarray(sSu)), (gSd[t, v], _c(rSd), np.asarray(sSd))):
            e = np.abs(got - r)
            worst = max(worst, float(np.max(e / np.maximum(s, 1e-300))))
            assert np.all(e <= grad_tol(r, s, 5, 4, prec) + 1e-300), (prec, t, v)
    print(f"3He batch grad_S {prec}: max |err|/scale = {worst:.3e}", flush=True)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_neutron_forward_and_backward(prec):
    """The (n_u, n_d) = (1, 2) family on a populated 4^3 x 4 lattice."""
    api = _api()
    ods = [dict(op="neutron", snk_spin=1, src_spin=1), dict(op="neutron", snk_spin=2, src_spin=3)]
    T, V = 4, 64
    Su, Sd = synth.iid(T, V, seed=6)
    rs = O.build_index_set(ods)
    ref = CO.correlator(Su, Sd, rs)
    A = CO.sum_abs_terms(Su, Sd, rs)
    C = forward(ods, Su, Sd, prec)
    check(C, ref, A, 1, 2, prec, "neutron 4^3x4")
    rng = np.random.default_rng(61)
    gC = rng.standard_normal((2, T)) + 1j * rng.standard_normal((2, T))
    plan = api.Plan(api.IndexSet(ods), prec)
    gW, gSu, gSd = api.contract_backward(plan, torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(), None,
                                         torch.from_numpy(gC).cuda())
    gW, gSu, gSd = gW.cpu().numpy(), gSu.cpu().numpy(), gSd.cpu().numpy()
    r = CO.gradients(Su, Sd, rs, gC)
    s = CO.gradient_abs_scales(Su, Sd, rs, gC)
    for name, got in (("W", gW), ("S_u", gSu), ("S_d", gSd)):
        assert np.all(np.abs(got - r[name]) <= grad_tol(r[name], s[name], 1, 2, prec) + 1e-300), (prec, name)

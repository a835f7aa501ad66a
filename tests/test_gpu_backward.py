"""GPU parity of the backward (adjoint) contraction against the oracle's gradients."""
import numpy as np
import pytest

from oracle import correlator as CO
from oracle import operators as O
from paper_2201_04269_amd import synth
from tests.parity import kappa

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_2201_04269_amd import api
    return api


CASES = {
    "proton": ([dict(op="proton")], 2, 3, "iid"),
    "proton_two_spins": ([dict(op="proton", snk_spin=1, src_spin=2), dict(op="proton", snk_spin=3, src_spin=3)],
                         1, 2, "iid"),
    "DI": ([dict(op="DI")], 2, 2, "su3"),
    "DI_DII_mix": ([dict(op="DI"), dict(op="DII"), dict(op="DII", sign_mode="r2")], 1, 2, "iid"),
    "He3": ([dict(op="HE3_I", snk_spin=2, src_spin=2), dict(op="HE3_II", snk_spin=0, src_spin=0, sign_mode="r2")],
            1, 1, "iid"),
}


def _inputs(name):
    ods, T, V, kind = CASES[name]
    Su, Sd = (synth.su3_spin if kind == "su3" else synth.iid)(T, V, seed=31)
    rs = O.build_index_set(ods)
    rng = np.random.default_rng(5)
    gC = rng.standard_normal((rs.n_corr, T)) + 1j * rng.standard_normal((rs.n_corr, T))
    return ods, Su, Sd, rs, gC


def _gpu_backward(ods, Su, Sd, gC, precision, W=None):
    api = _api()
    plan = api.Plan(api.IndexSet(ods), precision)
    su, sd = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda()
    w = None if W is None else torch.from_numpy(W).cuda()
    gW, gSu, gSd = api.contract_backward(plan, su, sd, w, torch.from_numpy(gC).cuda())
    torch.cuda.synchronize()
    return gW.cpu().numpy(), gSu.cpu().numpy(), gSd.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_backward_matches_oracle(name, precision):
    ods, Su, Sd, rs, gC = _inputs(name)
    got = dict(zip(("W", "S_u", "S_d"), _gpu_backward(ods, Su, Sd, gC, precision)))
    ref = CO.gradients(Su, Sd, rs, gC)
    scl = CO.gradient_abs_scales(Su, Sd, rs, gC)
    u = 2.0 ** -53 if precision == "f64" else 2.0 ** -24
    k = kappa(rs.nu, rs.nd)
    for key in ("W", "S_u", "S_d"):
        err = np.abs(got[key] - ref[key])
        tol = k * u * scl[key]
        if precision == "f64":
            tol = np.maximum(tol, 1e-12 * np.abs(ref[key]))
        ratio = float(np.max(err / np.maximum(scl[key], 1e-300)))
        print(name, precision, key, "max err / sum|terms|", ratio)
        assert np.all(err <= tol + 1e-300), (key, ratio)


def test_backward_user_weights_and_linearity_in_W():
    ods = [dict(op="DI")]
    Su, Sd = synth.iid(1, 2, seed=7)
    rs = O.build_index_set(ods)
    rng = np.random.default_rng(9)
    W = rng.standard_normal(rs.nnz) + 1j * rng.standard_normal(rs.nnz)
    gC = np.array([[0.3 - 1.1j]])
    gW, gSu, gSd = _gpu_backward(ods, Su, Sd, gC, "f64", W)
    rs.weights = lambda: W
    ref = CO.gradients(Su, Sd, rs, gC)
    for got, key in ((gW, "W"), (gSu, "S_u"), (gSd, "S_d")):
        assert np.max(np.abs(got - ref[key])) <= 1e-11 * np.max(np.abs(ref[key]))


def test_backward_empty_index_set_gives_zero():
    api = _api()
    plan = api.Plan(api.IndexSet([dict(op="DII")]), "f64")
    Su, Sd = synth.iid(2, 2, seed=1)
    su, sd = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda()
    gW, gSu, gSd = api.contract_backward(plan, su, sd, None, torch.ones(1, 2, dtype=torch.complex128).cuda())
    assert gW.numel() == 0
    assert torch.all(gSu == 0) and torch.all(gSd == 0)


def test_autograd_function_and_central_differences():
    """dC/dc for W(c) = c1 W_DI + c2 W_DII(R2), and dL/dS, against FD (h = 1e-4, FP64)."""
    api = _api()
    Su, Sd = synth.iid(2, 1, seed=3)
    both = api.IndexSet([dict(op="DI"), dict(op="DII", sign_mode="r2")])
    w = both.weights()
    n = both.nnz // 2
    W1 = torch.from_numpy(w[:n]).cuda()
    W2 = torch.from_numpy(w[n:]).cuda()
    plan = api.Plan(api.IndexSet([dict(op="DI")]), "f64")
    rng = np.random.default_rng(3)
    v = torch.from_numpy(rng.standard_normal((1, 2)) + 1j * rng.standard_normal((1, 2))).cuda()
    c = torch.tensor([1.0, 0.5], dtype=torch.float64, device="cuda", requires_grad=True)
    su = torch.from_numpy(Su).cuda().requires_grad_(True)
    sd = torch.from_numpy(Sd).cuda().requires_grad_(True)

    def loss(c_, su_, sd_):
        W = c_[0].to(torch.complex128) * W1 + c_[1].to(torch.complex128) * W2
        C = api.Contract.apply(su_, sd_, W, plan)
        return torch.real(torch.sum(torch.conj(v) * C))

    L = loss(c, su, sd)
    L.backward()
    h = 1e-4
    with torch.no_grad():
        for i in range(2):
            e = torch.zeros(2, dtype=torch.float64, device="cuda")
            e[i] = h
            fd = (loss(c + e, su, sd) - loss(c - e, su, sd)) / (2 * h)
            assert abs(float(fd) - float(c.grad[i])) <= 1e-9 * max(1.0, abs(float(fd)))
        # under R2, W_DII = 2 W_DI exactly, so dL/dc2 = 2 dL/dc1
        assert abs(float(c.grad[1]) - 2 * float(c.grad[0])) <= 1e-9 * abs(float(c.grad[0]))
        # C is a cubic polynomial in S_u (and in S_d): the five-point stencil
        # (8 [L(h) - L(-h)] - [L(2h) - L(-2h)]) / 12h is exact for it up to rounding
        E = torch.from_numpy(rng.standard_normal(Su.shape) + 1j * rng.standard_normal(Su.shape)).cuda()

        def fd5(f):
            return (8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)

        fd = fd5(lambda d: loss(c, su + d * E, sd))
        an = torch.real(torch.sum(torch.conj(su.grad) * E))
        assert abs(float(fd) - float(an)) <= 1e-8 * max(1.0, abs(float(an)))
        fd = fd5(lambda d: loss(c, su, sd + d * E))
        an = torch.real(torch.sum(torch.conj(sd.grad) * E))
        assert abs(float(fd) - float(an)) <= 1e-8 * max(1.0, abs(float(an)))
        # the plain central difference agrees to its O(h^2) truncation error
        fd2 = (loss(c, su + h * E, sd) - loss(c, su - h * E, sd)) / (2 * h)
        an = torch.real(torch.sum(torch.conj(su.grad) * E))
        assert abs(float(fd2) - float(an)) <= 1e-5 * max(1.0, abs(float(an)))


def test_backward_reproducible():
    ods, Su, Sd, rs, gC = _inputs("DI")
    a = _gpu_backward(ods, Su, Sd, gC, "f32c")
    b = _gpu_backward(ods, Su, Sd, gC, "f32c")
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.float64), y.view(np.float64))

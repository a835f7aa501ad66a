"""GPU parity of the forward contraction (through the C ABI) against the oracle."""
import numpy as np
import pytest

from oracle import correlator as CO
from oracle import operators as O
from paper_2201_04269_amd import synth
from tests.parity import f64_branch, kappa, tol_f32c, tol_f64

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_2201_04269_amd import api
    return api


def run(ods, Su, Sd, precision, W=None, c64=False):
    api = _api()
    iset = api.IndexSet(ods)
    plan = api.Plan(iset, precision)
    dt = torch.complex64 if c64 else torch.complex128
    su = torch.from_numpy(Su).to(dt).cuda()
    sd = torch.from_numpy(Sd).to(dt).cuda()
    w = None if W is None else torch.from_numpy(W).cuda()
    C = api.contract(plan, su, sd, w)
    torch.cuda.synchronize()
    return C.cpu().numpy(), plan


def oracle(ods, Su, Sd, W=None):
    ref_set = O.build_index_set(ods)
    if W is not None:
        ref_set.weights = lambda: W
    return CO.correlator(Su, Sd, ref_set), CO.sum_abs_terms(Su, Sd, ref_set), ref_set


CASES = {
    # configuration 1: proton alpha = alpha' = 0, 4^3 x 8, i.i.d. seed 0
    "proton_4x4x4x8": ([dict(op="proton")], lambda: synth.iid(8, 64, seed=0)),
    # dinucleon I on a small lattice, SU(3) (x) spin propagators (configuration 2's recipe)
    "DI_2x2x2x2_su3": ([dict(op="DI")], lambda: synth.su3_spin(2, 8, seed=1)),
    # several correlators in one launch, including an empty one (D_II exact)
    "DI_DII_mix": ([dict(op="DI"), dict(op="DII"), dict(op="DII", sign_mode="r2")],
                   lambda: synth.iid(2, 2, seed=2)),
    # 3He batch: I and II (R2), two spins
    "He3_batch": ([dict(op="HE3_I", snk_spin=0, src_spin=0), dict(op="HE3_I", snk_spin=2, src_spin=2),
                   dict(op="HE3_II", snk_spin=1, src_spin=1, sign_mode="r2")],
                  lambda: synth.iid(1, 2, seed=4)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_forward_f64_matches_oracle(name):
    ods, gen = CASES[name]
    Su, Sd = gen()
    C, plan = run(ods, Su, Sd, "f64")
    ref, A, rs = oracle(ods, Su, Sd)
    err = np.abs(C - ref)
    tol = tol_f64(ref, A, rs.nu, rs.nd)
    print(name, "max err/A", float(np.max(err / np.maximum(A, 1e-300))), "max err/|C|",
          float(np.max(err / np.maximum(np.abs(ref), 1e-300))), f64_branch(ref, A, rs.nu, rs.nd))
    assert np.all(err <= tol)


@pytest.mark.parametrize("name", list(CASES))
def test_forward_f32c_within_bound(name):
    ods, gen = CASES[name]
    Su, Sd = gen()
    C, plan = run(ods, Su, Sd, "f32c")
    ref, A, rs = oracle(ods, Su, Sd)
    err = np.abs(C - ref)
    print(name, "f32c err/A", float(np.max(err / np.maximum(A, 1e-300))),
          "bound", kappa(rs.nu, rs.nd) * 2.0 ** -24)
    assert np.all(err <= tol_f32c(A, rs.nu, rs.nd))


@pytest.mark.parametrize("name", ["DI_2x2x2x2_su3", "He3_batch"])
@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_factored_and_unfactored_schedules_agree(name, precision):
    """The exact weights (W = None) take the factored forward; the same
    weights passed as a user W take the unfactored one. Both must give the
    oracle's correlator within the precision's bound, and each other."""
    ods, gen = CASES[name]
    Su, Sd = gen()
    rs = O.build_index_set(ods)
    Cf, plan = run(ods, Su, Sd, precision)
    assert plan.stats["fwd_factored"] == 1 and plan.stats["rank1"] == 1
    Cu, _ = run(ods, Su, Sd, precision, W=np.asarray(rs.weights(), dtype=np.complex128))
    ref, A, _ = oracle(ods, Su, Sd)
    tol = tol_f64(ref, A, rs.nu, rs.nd) if precision == "f64" else tol_f32c(A, rs.nu, rs.nd)
    print(name, precision, "factored vs unfactored max |diff|/A",
          float(np.max(np.abs(Cf - Cu) / np.maximum(A, 1e-300))))
    assert np.all(np.abs(Cf - ref) <= tol)
    assert np.all(np.abs(Cu - ref) <= tol)
    assert np.all(np.abs(Cf - Cu) <= 2 * tol)


def test_empty_index_set_gives_zero():
    Su, Sd = synth.iid(3, 2, seed=9)
    C, plan = run([dict(op="DII"), dict(op="DII", snk_spin=1)], Su, Sd, "f64")
    assert plan.stats["n_tiles"] == 0
    assert np.all(C == 0)


def test_user_weights_and_complex64_input():
    ods = [dict(op="DI")]
    Su, Sd = synth.iid(2, 2, seed=6)
    rs = O.build_index_set(ods)
    rng = np.random.default_rng(8)
    W = rng.standard_normal(rs.nnz) + 1j * rng.standard_normal(rs.nnz)
    C, _ = run(ods, Su, Sd, "f64", W=W)
    ref, _, _ = oracle(ods, Su, Sd, W)
    rs.weights = lambda: np.abs(W)
    A = CO.sum_abs_terms(Su, Sd, rs)
    assert np.all(np.abs(C - ref) <= tol_f64(ref, A, 3, 3))
    # complex64 propagators: the FP64 kernel sees exactly the rounded inputs
    S32u, S32d = Su.astype(np.complex64), Sd.astype(np.complex64)
    C32, _ = run(ods, S32u, S32d, "f64", W=W, c64=True)
    ref32, _, _ = oracle(ods, S32u.astype(np.complex128), S32d.astype(np.complex128), W)
    assert np.all(np.abs(C32 - ref32) <= tol_f64(ref32, A, 3, 3) * 2)


def test_run_to_run_bitwise_reproducible():
    ods = [dict(op="DI")]
    Su, Sd = synth.iid(2, 4, seed=10)
    api = _api()
    plan = api.Plan(api.IndexSet(ods), "f64")
    su, sd = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda()
    a = api.contract(plan, su, sd).cpu().numpy()
    b = api.contract(plan, su, sd).cpu().numpy()
    assert np.array_equal(a.view(np.float64), b.view(np.float64))


def test_identity_closed_forms_on_gpu():
    """S = 1 gives sigma s^2 sum |w|^2 exactly (integers) in both precisions."""
    I = np.broadcast_to(np.eye(12, dtype=complex), (2, 3, 12, 12)).copy()
    for ods, val in (([dict(op="proton")], -30), ([dict(op="DI")], -4320),
                     ([dict(op="HE3_I", snk_spin=2, src_spin=2)], 4608)):
        for prec in ("f64", "f32c"):
            C, _ = run(ods, I, I, prec)
            assert np.all(C == 3 * val), (ods, prec, C)


def test_invalid_pointer_is_rejected():
    api = _api()
    plan = api.Plan(api.IndexSet([dict(op="proton")]), "f64")
    from paper_2201_04269_amd import _binding as B
    import ctypes
    host = np.zeros(288, dtype=np.complex128)
    C = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = B.lib().mbc_contract(plan._h, ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(host.ctypes.data),
                              0, 1, 1, None, ctypes.c_void_p(C.data_ptr()), None, 0, None)
    assert st == 1 and b"device" in B.lib().mbc_last_error()

"""mbc_contract_noalloc (fixed per-GPU scratch, no allocation) against
mbc_contract (caller workspace) through the C ABI: identical results on two
calls in a row, the second with a smaller input, and a clear error when the
intermediates exceed the scratch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2201_04269_amd import _binding as B
from paper_2201_04269_amd import api, synth

pytestmark = pytest.mark.gpu


def _noalloc(plan, su, sd, W, C):
    L = B.lib()
    dt = B.C128 if su.dtype == torch.complex128 else B.C64
    T, V = su.shape[:2]
    st = L.mbc_contract_noalloc(plan._h, ctypes.c_void_p(su.data_ptr()), ctypes.c_void_p(sd.data_ptr()), dt, int(T),
                                int(V), ctypes.c_void_p(W.data_ptr() if W is not None else 0),
                                ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_noalloc_equals_the_workspace_entry_point_on_two_calls(prec):
    dev = torch.device("cuda:0")
    plan = api.Plan(api.IndexSet([dict(op="DI")]), prec)
    rng = np.random.default_rng(7)
    W = torch.from_numpy(rng.standard_normal(plan.iset.nnz) + 1j * rng.standard_normal(plan.iset.nnz)).to(dev)
    for (T, V, seed) in ((2, 64, 3), (1, 16, 4)):  # second call smaller
        Su, Sd = synth.iid(T, V, seed=seed)
        su, sd = torch.from_numpy(Su).to(dev), torch.from_numpy(Sd).to(dev)
        for w in (W, None):
            print(f"noalloc {prec} T={T} V={V} W={'user' if w is not None else 'exact'}", flush=True)
            ref = api.contract(plan, su, sd, w)
            C = torch.full((plan.n_corr, T), float("nan"), dtype=torch.complex128, device=dev)
            assert _noalloc(plan, su, sd, w, C) == B.MBC_OK, B.lib().mbc_last_error().decode()
            torch.cuda.synchronize()
            # the same kernels on the same launch shape: bit-identical
            assert torch.equal(C, ref)


def test_noalloc_rejects_intermediates_beyond_the_scratch():
    dev = torch.device("cuda:0")
    ops = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)]
    plan = api.Plan(api.IndexSet(ops), "f32c")
    W = torch.zeros(plan.iset.nnz, dtype=torch.complex128, device=dev)  # 3.2M weights: 25.7 MB plan-ordered
    Su, Sd = synth.iid(1, 2, seed=5)
    su, sd = torch.from_numpy(Su).to(dev), torch.from_numpy(Sd).to(dev)
    C = torch.zeros((plan.n_corr, 1), dtype=torch.complex128, device=dev)
    print("noalloc 3He_I batch with a caller W: exact weights fit, caller weights in F64 do not", flush=True)
    assert _noalloc(plan, su, sd, None, C) == B.MBC_OK
    plan64 = api.Plan(api.IndexSet(ops), "f64")
    st = _noalloc(plan64, su, sd, W, C)
    assert st == B.MBC_ERR_UNSUPPORTED
    assert "scratch" in B.lib().mbc_last_error().decode()

"""Host-side checks of libmbc (no GPU): exported symbols, bit-exact index sets
against the oracle, argument validation, and the compiled schedule walked on
the host (mbc_debug_eval_host) against the oracle's correlator."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import correlator as CO
from oracle import operators as O
from paper_2201_04269_amd import _binding as B
from paper_2201_04269_amd import synth
from paper_2201_04269_amd.api import IndexSet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(mbc_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    B.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(mbc_[a-z0-9_]+)$", out, flags=re.M))
    declared = _declared_symbols()
    assert declared, "no declarations found"
    assert declared <= exported, declared - exported
    # and the binding knows every one of them
    assert declared <= {n for n, _, _ in B.SIGNATURES}


CASES = [("proton", 0, 0, "exact", True), ("proton", 2, 1, "exact", True), ("neutron", 3, 3, "exact", True),
         ("DI", 0, 0, "exact", True), ("DII", 0, 0, "exact", True), ("DII", 0, 0, "r2", True),
         ("HE3_I", 0, 0, "exact", True), ("HE3_I", 3, 3, "exact", True), ("HE3_II", 1, 1, "exact", True),
         ("HE3_II", 2, 2, "r2", True), ("proton", 0, 0, "exact", False), ("DI", 0, 0, "exact", False)]


@pytest.mark.parametrize("op,s,sp,mode,sym", CASES, ids=lambda *a: None)
def test_index_set_bit_exact_vs_oracle(op, s, sp, mode, sym):
    od = dict(op=op, snk_spin=s, src_spin=sp, sign_mode=mode, symmetrise=sym)
    ref = O.build_index_set([od])
    got = IndexSet([od]).export()
    assert got["snk_u"].shape == ref.snk_u.shape
    if sym:
        for k, rk in (("snk_u", "snk_u"), ("src_u", "src_u"), ("snk_d", "snk_d"), ("src_d", "src_d"),
                      ("corr_id", "corr_id"), ("w_re", "w_re"), ("w_im", "w_im"), ("w_den", "w_den")):
            assert np.array_equal(got[k], getattr(ref, rk)), k
    else:
        # raw sets: order of written terms is not canonical; compare as multisets
        def rows(d):
            m = np.concatenate([d["snk_u"], d["src_u"], d["snk_d"], d["src_d"],
                                d["w_re"][:, None], d["w_im"][:, None]], 1).astype(np.int64)
            return m[np.lexsort(m.T[::-1])]
        r = dict(snk_u=ref.snk_u, src_u=ref.src_u, snk_d=ref.snk_d, src_d=ref.src_d, w_re=ref.w_re, w_im=ref.w_im)
        assert np.array_equal(rows(got), rows(r))


def test_index_set_batch_of_correlators_bit_exact():
    ods = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
          [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]
    ref = O.build_index_set(ods)
    got = IndexSet(ods).export()
    assert got["corr_id"].shape[0] == ref.nnz == 8352810
    for k in ("snk_u", "src_u", "snk_d", "src_d", "corr_id", "w_re", "w_im", "w_den"):
        assert np.array_equal(got[k], getattr(ref, k)), k


def test_invalid_arguments_return_status():
    L = B.lib()
    h = ctypes.c_void_p()
    bad = (B.OpDesc * 1)()
    bad[0].op = 99
    assert L.mbc_build_index_set(bad, 1, ctypes.byref(h)) == 1
    assert b"operator" in L.mbc_last_error()
    assert L.mbc_build_index_set(bad, 0, ctypes.byref(h)) == 1
    bad[0].op = 0
    bad[0].snk_spin = 4
    assert L.mbc_build_index_set(bad, 1, ctypes.byref(h)) == 1
    two = (B.OpDesc * 2)()
    two[0].op = B.OPS["proton"]
    two[1].op = B.OPS["DI"]
    assert L.mbc_build_index_set(two, 2, ctypes.byref(h)) == 1  # mixed (n_u, n_d)
    assert L.mbc_index_set_dims(None, None, None, None, None) == 1
    L.mbc_index_set_free(None)
    L.mbc_plan_destroy(None)
    assert L.mbc_contract(None, None, None, 0, 1, 1, None, None, None, 0, None) == 1
    # a raw (unsymmetrised) set has no plan
    good = (B.OpDesc * 1)()
    good[0].op = B.OPS["proton"]
    good[0].symmetrise = 0
    assert L.mbc_build_index_set(good, 1, ctypes.byref(h)) == 0
    C = np.zeros(2)
    S = np.zeros(288)
    assert L.mbc_debug_eval_host(h, 0, S.ctypes.data, S.ctypes.data, 1, 1, None, C.ctypes.data, None) == 1
    L.mbc_index_set_free(h)


def host_walk(ods, Su, Sd, W=None, precision=B.F64):
    iset = IndexSet(ods)
    T, V = Su.shape[:2]
    C = np.zeros((iset.n_corr, T), dtype=np.complex128)
    st = B.PlanStats()
    Wc = None if W is None else np.ascontiguousarray(W, dtype=np.complex128)
    B.check(B.lib().mbc_debug_eval_host(iset._h, precision, np.ascontiguousarray(Su).ctypes.data,
                                        np.ascontiguousarray(Sd).ctypes.data, T, V,
                                        None if Wc is None else Wc.ctypes.data, C.ctypes.data,
                                        ctypes.byref(st)))
    return C, st


@pytest.mark.parametrize("ods", [
    [dict(op="proton", snk_spin=0, src_spin=0)],
    [dict(op="proton", snk_spin=1, src_spin=2), dict(op="proton", snk_spin=3, src_spin=3)],
    [dict(op="DI")],
    [dict(op="DI"), dict(op="DII", sign_mode="r2"), dict(op="DII")],
    [dict(op="HE3_I", snk_spin=2, src_spin=2), dict(op="HE3_II", snk_spin=0, src_spin=0, sign_mode="r2")],
    [dict(op="neutron", snk_spin=1, src_spin=1)],
], ids=["proton", "p+n", "DI", "DI+DII", "He3", "neutron"])
def test_plan_walk_matches_oracle(ods):
    """W = NULL walks the factored forward (every correlator's exact weights
    are a sink vector times a source vector: per run, sum over top d columns
    of (sum_b u[b] Dd) (sum_s v[s] Du)); the same weights passed explicitly
    walk the forward tiles that stage the weights. Both against the oracle."""
    Su, Sd = synth.iid(2, 1, seed=17)
    ref_set = O.build_index_set(ods)
    ref = CO.correlator(Su, Sd, ref_set)
    A = CO.sum_abs_terms(Su, Sd, ref_set) if ref_set.nnz < 300000 else None
    scale = A if A is not None else np.abs(ref) + 1.0
    for W in (None, ref_set.weights()):
        C, st = host_walk(ods, Su, Sd, W)
        assert np.all(np.abs(C - ref) <= 1e-12 * np.maximum(scale, 1e-300) + 1e-300), (C, ref, W is None)
    assert st.rank1 == 1 and st.fwd_factored == 1
    assert st.n_tiles >= 1 and st.f_n_tiles >= 1
    assert st.exec_flops_per_site >= st.alg_flops_per_site * 0.5


def test_plan_walk_user_weights():
    Su, Sd = synth.iid(1, 2, seed=5)
    ods = [dict(op="DI")]
    ref_set = O.build_index_set(ods)
    rng = np.random.default_rng(3)
    W = rng.standard_normal(ref_set.nnz) + 1j * rng.standard_normal(ref_set.nnz)
    C, _ = host_walk(ods, Su, Sd, W)
    ref_set.weights = lambda: W
    ref = CO.correlator(Su, Sd, ref_set)
    assert np.allclose(C, ref, rtol=1e-11, atol=1e-9)


def test_plan_statistics_dinucleon():
    Su, Sd = synth.iid(1, 1, seed=0)
    _, st = host_walk([dict(op="DI")], Su, Sd)
    # global minor DAG: 2 x (52*66*14 + 208*208*22) + 8*(520^2 + 208^2)
    assert st.alg_flops_per_site == 2 * (52 * 66 * 14 + 208 * 208 * 22) + 8 * (520 ** 2 + 208 ** 2)
    assert st.lds_bytes <= 160 * 1024


def host_backward(ods, Su, Sd, gC, W=None):
    iset = IndexSet(ods)
    gW = np.zeros(iset.nnz, dtype=np.complex128)
    gSu = np.zeros_like(Su)
    gSd = np.zeros_like(Sd)
    T, V = Su.shape[:2]
    Wc = None if W is None else np.ascontiguousarray(W, dtype=np.complex128)
    gC = np.ascontiguousarray(gC, dtype=np.complex128)
    B.check(B.lib().mbc_debug_backward_host(iset._h, B.F64, np.ascontiguousarray(Su).ctypes.data,
                                            np.ascontiguousarray(Sd).ctypes.data, T, V,
                                            None if Wc is None else Wc.ctypes.data, gC.ctypes.data,
                                            gW.ctypes.data, gSu.ctypes.data, gSd.ctypes.data))
    return gW, gSu, gSd


@pytest.mark.parametrize("ods,T,V", [
    ([dict(op="proton", snk_spin=0, src_spin=0)], 2, 2),
    ([dict(op="proton", snk_spin=1, src_spin=2), dict(op="proton", snk_spin=3, src_spin=3)], 1, 2),
    ([dict(op="DI")], 2, 1),
    ([dict(op="DI"), dict(op="DII", sign_mode="r2"), dict(op="DII")], 1, 1),
    ([dict(op="HE3_I", snk_spin=1, src_spin=1)], 1, 1),
], ids=["proton", "p2", "DI", "DI+DII", "He3"])
def test_backward_walk_matches_oracle_gradients(ods, T, V):
    Su, Sd = synth.iid(T, V, seed=23)
    rs = O.build_index_set(ods)
    rng = np.random.default_rng(4)
    gC = rng.standard_normal((rs.n_corr, T)) + 1j * rng.standard_normal((rs.n_corr, T))
    ref = CO.gradients(Su, Sd, rs, gC)
    # W = NULL walks the factored dS schedule (the exact weights as a product
    # of a sink and a source vector); the same weights passed explicitly walk
    # the schedule that stages the weights
    for W in (None, rs.weights()):
        gW, gSu, gSd = host_backward(ods, Su, Sd, gC, W)
        for name, got in (("W", gW), ("S_u", gSu), ("S_d", gSd)):
            r = ref[name]
            scale = np.max(np.abs(r)) + 1e-300
            assert np.max(np.abs(got - r)) <= 1e-11 * scale, (name, W is None)


def test_mbc_log_writes_one_line_per_handle():
    code = ("from paper_2201_04269_amd import api\n"
            "api.IndexSet([dict(op='proton')])\n"
            "b = api.BlockSet([dict(op='DI', moms=[(0, 0, 0)] * 2)])\n"
            "api.TensorEGraph.for_blocks(b, 0, 0)\n")
    env = dict(os.environ, MBC_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[mbc] ")]
    assert [ln.split(":")[0] for ln in lines] == ["[mbc] index set", "[mbc] block set", "[mbc] e-graph"]
    assert "441 entries" in lines[0]
    env["MBC_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert "[mbc]" not in r.stderr


HE3_BATCH = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
            [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]


@pytest.mark.parametrize("ods", [[dict(op="DI")], HE3_BATCH], ids=["DI", "He3_batch"])
def test_bench_plans_fit_the_kernel_instantiations(ods):
    """mbc_plan_create checks a compiled plan against the kernels' compiled
    limits (source keys per thread, columns per level, dW keys per tile, the
    S-bar bins' lanes x registers, source-key lists) before it touches the
    device: the bench workloads' plans must pass in both precisions (without
    a device the call then fails at the device lookup, never as unsupported)."""
    L = B.lib()
    s = IndexSet(ods)
    for prec in (B.F64, B.F32C):
        h = ctypes.c_void_p()
        st = L.mbc_plan_create(s._h, prec, None, ctypes.byref(h))
        assert st != B.MBC_ERR_UNSUPPORTED, L.mbc_last_error()
        if st == B.MBC_OK:
            L.mbc_plan_destroy(h)

"""GPU parity of the hadron blocks and block-level correlators (through the C
ABI) against the oracle; correlators by factor trees (Sec. 4) and by the flat
term sum.

Tolerances (FP64 throughout):
* a block entry is a sum over sites; the kernel's and the oracle's sums differ
  in order and in the factorisation through B, so each entry may differ by a
  few units of 2^-53 times the sum of the magnitudes of its site terms, which
  the tests bound by 1e-13 * V * max|f| (per block type and timeslice);
* a correlator is sum_k w_k prod_i f_i with heavy cancellation; its error is
  bounded by n_slots times the block error times the sum of the magnitudes of
  its products, A[t] = sum_k |w_k| prod_i |f_i|, so the tests require
  |C_gpu - C_oracle| <= 1e-12 A[t] + 1e-12 |C_oracle|.
"""
import numpy as np
import pytest

from oracle import blocks as OB
from oracle import correlator as CO
from oracle import operators as O
from paper_2201_04269_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAME = {("p", 0): "p", ("n", 0): "n", ("p", 1): "p+", ("p", -1): "p-", ("n", 1): "n+", ("n", -1): "n-"}


def _api():
    from paper_2201_04269_amd import api
    return api


def gpu_blocks(corrs, Su, Sd, dims, c64=False):
    """(C by factor trees, blocks, block set); C by the flat term sum must agree
    with the trees to rounding (checked here)."""
    api = _api()
    bset = api.BlockSet(corrs)
    plan = api.BlockPlan(bset)
    dt = torch.complex64 if c64 else torch.complex128
    su = torch.from_numpy(Su).to(dt).cuda()
    sd = torch.from_numpy(Sd).to(dt).cuda()
    C, blk = api.block_correlators(plan, su, sd, dims)
    Ct = api.block_contract(plan, blk, method="terms")
    torch.cuda.synchronize()
    C, Ct = C.cpu().numpy(), Ct.cpu().numpy()
    assert np.all(np.abs(C - Ct) <= 1e-12 * np.abs(Ct).max(axis=1, keepdims=True) + 1e-300)
    return C, blk.cpu().numpy().reshape(Su.shape[0], bset.n_types, 4, 1728), bset


def oracle_blocks(bset, Su, Sd, dims):
    return {(NAME[(f, p)], m, z): OB.block(Su, Sd, NAME[(f, p)], m, dims, srcs=z)
            for f, p, m, z in bset.types(with_points=True)}


def abs_scale(bset, blocks):
    """A[c, t] = sum_k |w_k| prod_i |f_i| over the library's terms."""
    e = bset.export()
    T = next(iter(blocks.values())).shape[0]
    flat = np.stack([np.abs(blocks[(NAME[(f, p)], m, z)]) for f, p, m, z in bset.types(with_points=True)],
                    axis=1).reshape(T, -1)
    w = np.abs((e["num_re"] + 1j * e["num_im"]) / e["den"][e["corr_id"]])
    prod = np.ones((T, bset.n_terms)) * w[None, :]
    for s in range(bset.n_slots):
        f = e["factor"][:, s]
        used = f >= 0
        prod[:, used] *= flat[:, f[used]]
    return np.stack([prod[:, e["corr_id"] == c].sum(axis=1) for c in range(bset.n_corr)])


def check_blocks(blk, ref, bset, V):
    for k, (f, p, m) in enumerate(bset.types()):
        want = ref[(NAME[(f, p)], m, (0, 0, 0))]
        for t in range(blk.shape[0]):
            scale = np.abs(want[t]).max()
            err = np.abs(blk[t, k] - want[t]).max()
            assert err <= 1e-13 * V * scale, (f, p, m, t, err, scale)


def check_corr(C, ref, A):
    err = np.abs(C - ref)
    assert np.all(err <= 1e-12 * A + 1e-12 * np.abs(ref)), (err.max(), A.max())


BATCH = [
    dict(op="proton", snk_spin=1, src_spin=2, moms=[(1, 1, 0)]),
    dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)]),
    dict(op="DII", sign_mode="r2", moms=[(0, 1, 0), (0, -1, 0)]),
    dict(op="HE3_I", snk_spin=2, src_spin=2, moms=[(1, 0, 0), (0, 0, 0), (-1, 0, 0)]),
]


@pytest.mark.parametrize("c64", [False, True])
def test_blocks_and_correlators_of_a_mixed_batch(c64):
    dims, T = (4, 2, 2), 2
    Su, Sd = synth.iid(T, 16, seed=41)
    if c64:  # both sides see the same complex64-rounded propagators
        Su, Sd = Su.astype(np.complex64).astype(np.complex128), Sd.astype(np.complex64).astype(np.complex128)
    C, blk, bset = gpu_blocks(BATCH, Su, Sd, dims, c64=c64)
    assert bset.n_slots == 3 and bset.n_types == 10
    ref = oracle_blocks(bset, Su, Sd, dims)
    check_blocks(blk, ref, bset, 16)
    A = abs_scale(bset, ref)
    for c, corr in enumerate(BATCH):
        want = OB.block_correlator(Su, Sd, corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0),
                                   corr.get("sign_mode", "exact"), corr["moms"], dims, blocks=ref)
        check_corr(C[c], want, A[c])


def test_blocks_are_exactly_antisymmetric_with_zero_diagonal():
    dims, T = (3, 2, 1), 1
    Su, Sd = synth.iid(T, 6, seed=42)
    _, blk, _ = gpu_blocks([dict(op="DI", moms=[(1, 0, 0), (2, 1, 0)])], Su, Sd, dims)
    f = blk.reshape(T, -1, 4, 12, 12, 12)
    assert np.array_equal(f, -f.transpose(0, 1, 2, 5, 4, 3))
    assert np.all(np.einsum("tkaiyi->tkay", f) == 0)


def test_one_site_equals_the_determinant_form_kernels():
    # V = 1: the block path and mbc_contract compute the same local correlator
    api = _api()
    T = 3
    Su, Sd = synth.su3_spin(T, 1, seed=43)
    corrs = [dict(op="DI", moms=[(0, 0, 0)] * 2), dict(op="HE3_I", snk_spin=1, src_spin=1, moms=[(0, 0, 0)] * 3)]
    C, _, _ = gpu_blocks(corrs, Su, Sd, (1, 1, 1))
    for c, (op, spin) in enumerate([("DI", 0), ("HE3_I", 1)]):
        iset = api.IndexSet([dict(op=op, snk_spin=spin, src_spin=spin)])
        det = api.contract(api.Plan(iset, "f64"), torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda())
        det = det.cpu().numpy()[0]
        ref = CO.correlator(Su, Sd, O.build_index_set([dict(op=op, snk_spin=spin, src_spin=spin)]))[0]
        A = CO.sum_abs_terms(Su, Sd, O.build_index_set([dict(op=op, snk_spin=spin, src_spin=spin)]))[0]
        assert np.all(np.abs(C[c] - ref) <= 1e-12 * A)
        assert np.all(np.abs(C[c] - det) <= 2e-12 * A)


def test_ragged_site_chunks_sampled_entries():
    # 105 sites, 4 timeslices, 5 block types: the launch uses chunks of 2
    # sites with a one-site tail; checked on sampled entries of every type
    api = _api()
    dims, T = (7, 5, 3), 4
    corrs = [dict(op="DI", moms=[(1, 2, 0), (-1, 0, 1)]),
             dict(op="HE3_I", moms=[(0, 0, 1), (3, 0, 0), (0, 0, 0)])]
    assert api.BlockSet(corrs).n_types == 5
    Su, Sd = synth.iid(T, 105, seed=44)
    _, blk, bset = gpu_blocks(corrs, Su, Sd, dims)
    rng = np.random.default_rng(5)
    for k, (f, p, m) in enumerate(bset.types()):
        ent = [tuple(int(v) for v in rng.integers(0, [4, 12, 12, 12])) for _ in range(12)]
        ent = [(a, A, Y, C) if A != C else (a, A, Y, (C + 1) % 12) for a, A, Y, C in ent]
        want = OB.block_entries(Su, Sd, NAME[(f, p)], m, dims, ent)
        got = np.stack([blk[:, k, a, (A * 12 + Y) * 12 + C] for a, A, Y, C in ent], axis=1)
        assert np.abs(got - want).max() <= 1e-13 * 105 * np.abs(want).max()


def test_exact_sign_dii_gives_zero_and_empty_sets_are_fine():
    C, blk, bset = gpu_blocks([dict(op="DII", moms=[(0, 0, 0)] * 2)], *synth.iid(2, 4, seed=45), (2, 2, 1))
    assert bset.n_terms == 0
    assert np.all(C == 0)
    assert np.all(np.isfinite(blk))


def test_bad_arguments_are_rejected():
    api = _api()
    bset = api.BlockSet([dict(op="proton", moms=[(0, 0, 0)])])
    plan = api.BlockPlan(bset)
    su = torch.zeros((1, 4, 12, 12), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        api.blocks(plan, su, su, (2, 1, 1))  # V does not match dims
    with pytest.raises(api.B.MbcError):
        api.blocks(plan, su, su, (2, 2, 1), workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    host = torch.zeros((1, 4, 12, 12), dtype=torch.complex128)
    import ctypes
    d = (ctypes.c_int32 * 3)(2, 2, 1)
    assert api.B.lib().mbc_blocks_compute(plan._h, ctypes.c_void_p(host.data_ptr()),
                                          ctypes.c_void_p(host.data_ptr()), 0, 1, d, None, None, 0, None) == 1


def test_block_example_from_the_readme():
    # the README's block-path snippet, checked against the oracle
    api = _api()
    bset = api.BlockSet([dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)])])
    bplan = api.BlockPlan(bset)
    Su, Sd = synth.iid(T=4, V=64, seed=2)
    C, blocks = api.block_correlators(bplan, torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(),
                                      dims=(4, 4, 4))
    factors, children = bset.factor_tree(0)
    assert factors[0] == -1 and children.sum() == len(factors) - 1
    n_terms, n_distinct, hist = api.block_multiplicities(dict(op="DI", moms=[(0, 0, 0)] * 2))
    assert n_terms == 4 * 2304 * 9 and (np.arange(hist.shape[0]) * hist).sum() == n_terms
    eg = api.TensorEGraph.for_blocks(bset, 0, node_limit=100000)
    C_eg = eg.execute_blocks(blocks)
    ref = OB.block_correlator(Su, Sd, "DI", 0, 0, "exact", [(1, 0, 0), (-1, 0, 0)], (4, 4, 4))
    assert np.abs(C.cpu().numpy()[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(C_eg.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert eg.stats["saturated"] == 1 and eg.stats["flops_plan"] < eg.stats["flops_direct"]


def test_blocks_and_correlators_are_bitwise_reproducible():
    api = _api()
    corrs = [dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)]), dict(op="HE3_I", moms=[(0, 0, 0)] * 3)]
    plan = api.BlockPlan(api.BlockSet(corrs))
    Su, Sd = synth.iid(3, 60, seed=46)
    su, sd = torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda()
    runs = []
    for _ in range(2):
        blk = api.blocks(plan, su, sd, (5, 4, 3))
        runs.append([blk.cpu().numpy(), api.block_contract(plan, blk, method="tree").cpu().numpy(),
                     api.block_contract(plan, blk, method="terms").cpu().numpy()])
    for x, y in zip(*runs):
        assert np.array_equal(x.view(np.float64), y.view(np.float64))


def test_displaced_sources_mixed_source_blocks_and_correlators():
    # two source points (a propagator set each); D_I and exact-sign D_II with
    # the source baryons displaced, and a proton from the second point
    api = _api()
    dims, T = (3, 2, 1), 2
    corrs = [dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)], src_pts=(0, 1)),
             dict(op="DII", moms=[(1, 0, 0), (-1, 0, 0)], src_pts=(0, 1)),
             dict(op="proton", snk_spin=1, src_spin=3, moms=[(0, 1, 0)], src_pts=(1,))]
    S = [synth.iid(T, 6, seed=90 + p) for p in range(2)]
    Su, Sd = np.stack([x[0] for x in S]), np.stack([x[1] for x in S])
    bset = api.BlockSet(corrs)
    assert bset.n_points == 2
    plan = api.BlockPlan(bset)
    assert plan.stats["n_gmats"] > bset.n_types  # mixed-source types take two G matrices
    C, blk = api.block_correlators(plan, torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(), dims)
    Ct = api.block_contract(plan, blk, method="terms")
    torch.cuda.synchronize()
    C, Ct, blk = C.cpu().numpy(), Ct.cpu().numpy(), blk.cpu().numpy().reshape(T, bset.n_types, 4, 1728)
    ref = {}
    for k, (f, p, m, z) in enumerate(bset.types(with_points=True)):
        want = OB.block(Su, Sd, NAME[(f, p)], m, dims, srcs=z)
        ref[(NAME[(f, p)], m, z)] = want
        assert np.abs(blk[:, k] - want).max() <= 1e-13 * 6 * np.abs(want).max(), (f, p, m, z)
    for c, corr in enumerate(corrs):
        want = OB.block_correlator(Su, Sd, corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0), "exact",
                                   corr["moms"], dims, src_pts=corr["src_pts"], blocks=ref)
        for got in (C[c], Ct[c]):
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (c, np.abs(got - want).max())
    assert np.abs(C[1]).max() > 1.0  # exact-sign D_II survives displaced sources

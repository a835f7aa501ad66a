"""Host side of the block path: libmbc's block-level term expansion and
multiplicity count against the oracle (no GPU).

The library's terms are contracted here, in NumPy, with blocks the oracle
computes from their definition; the sum must equal the oracle's own
block-level correlator, which is pinned in test_oracle_blocks.py.
"""
import ctypes

import numpy as np
import pytest

from oracle import blocks as OB
from paper_2201_04269_amd import _binding as B
from paper_2201_04269_amd import api, synth

NAME = {("p", 0): "p", ("n", 0): "n", ("p", 1): "p+", ("p", -1): "p-", ("n", 1): "n+", ("n", -1): "n-"}


def contract_terms_with_oracle_blocks(bset, S_u, S_d, dims):
    """C [n_corr, T] = sum over the library's terms of w_k prod_i f[t][factor_i].

    S_u, S_d: [T, V, 12, 12] or [P, T, V, 12, 12] (one set per source point)."""
    T = S_u.shape[-4]
    blk = np.stack([OB.block(S_u, S_d, NAME[(fam, proj)], mom, dims, srcs=z)
                    for fam, proj, mom, z in bset.types(with_points=True)], axis=1).reshape(T, -1)
    e = bset.export()
    w = (e["num_re"] + 1j * e["num_im"]) / e["den"][e["corr_id"]]
    prod = np.ones((T, bset.n_terms), dtype=np.complex128) * w[None, :]
    for s in range(bset.n_slots):
        f = e["factor"][:, s]
        used = f >= 0
        prod[:, used] *= blk[:, f[used]]
    C = np.zeros((bset.n_corr, T), dtype=np.complex128)
    for c in range(bset.n_corr):
        C[c] = prod[:, e["corr_id"] == c].sum(axis=1)
    return C


@pytest.mark.parametrize("corr,dims,T", [
    (dict(op="proton", snk_spin=1, src_spin=2, moms=[(1, 1, 0)]), (2, 2, 1), 2),
    (dict(op="neutron", snk_spin=0, src_spin=3, moms=[(0, 1, 0)]), (2, 2, 1), 1),
    (dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)]), (2, 2, 1), 2),
    (dict(op="DII", sign_mode="r2", moms=[(1, 0, 0), (0, 1, 0)]), (2, 2, 1), 1),
    (dict(op="HE3_I", snk_spin=1, src_spin=3, moms=[(1, 0, 0), (0, 0, 0), (-1, 0, 0)]), (2, 1, 1), 1),
])
def test_library_terms_reproduce_the_oracle_correlator(corr, dims, T):
    V = dims[0] * dims[1] * dims[2]
    S_u, S_d = synth.iid(T, V, seed=31)
    bset = api.BlockSet([corr])
    got = contract_terms_with_oracle_blocks(bset, S_u, S_d, dims)[0]
    ref = OB.block_correlator(S_u, S_d, corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0),
                              corr.get("sign_mode", "exact"), corr["moms"], dims)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_mixed_batch_pads_unused_slots_and_shares_types():
    corrs = [dict(op="proton", moms=[(0, 0, 0)]), dict(op="DI", moms=[(0, 0, 0), (0, 0, 0)]),
             dict(op="DII", sign_mode="exact", moms=[(0, 0, 0), (0, 0, 0)])]
    bset = api.BlockSet(corrs)
    assert bset.n_slots == 2 and bset.n_corr == 3
    assert bset.types() == [("p", 0, (0, 0, 0)), ("n", 0, (0, 0, 0))]
    e = bset.export()
    assert np.all(e["factor"][e["corr_id"] == 0, 1] == -1)
    assert np.all(e["factor"][e["corr_id"] == 1] >= 0)
    assert not np.any(e["corr_id"] == 2)  # exact-sign D_II: empty source, no terms
    assert list(e["den"]) == [1, 1, 2]
    # every factor names a block entry with its two like antiquarks in order
    f = e["factor"][e["factor"] >= 0]
    A, C = (f // 144) % 12, f % 12
    assert np.all(A < C)
    S_u, S_d = synth.iid(2, 1, seed=32)
    got = contract_terms_with_oracle_blocks(bset, S_u, S_d, (1, 1, 1))
    for c, corr in enumerate(corrs):
        ref = OB.block_correlator(S_u, S_d, corr["op"], 0, 0, corr.get("sign_mode", "exact"), corr["moms"],
                                  (1, 1, 1))
        assert np.abs(got[c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_dinucleon_terms_are_products_of_nine_partitions():
    # 4 sink spin products x 9 partitions x 520 canonical source keys; no two
    # coincide after ordering the factors
    bset = api.BlockSet([dict(op="DI", moms=[(0, 0, 0), (0, 0, 0)])])
    assert bset.n_terms == 4 * 9 * 520


@pytest.mark.parametrize("corr", [dict(op="proton", snk_spin=2, src_spin=1),
                                  dict(op="DI"), dict(op="DII", sign_mode="exact"),
                                  dict(op="DII", sign_mode="r2"), dict(op="DI", src_pts=(0, 1))])
def test_multiplicity_histogram_matches_the_oracle_exactly(corr):
    A = 1 if corr["op"] == "proton" else 2
    c = dict(corr, moms=[(0, 0, 0)] * A)
    n, n_distinct, hist = api.block_multiplicities(c)
    on, ohist = OB.multiplicity_histogram(corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0),
                                          corr.get("sign_mode", "exact"), src_pts=corr.get("src_pts"))
    assert n == on
    assert n_distinct == sum(ohist.values())
    assert {m: int(k) for m, k in enumerate(hist) if k} == dict(ohist)


def test_multiplicity_guard_and_errors():
    L = B.lib()
    d = api._block_descs([dict(op="HE3_II", sign_mode="r2", moms=[(0, 0, 0)] * 3)])
    nt, nd, mm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.mbc_block_multiplicities(d, 1000, ctypes.byref(nt), ctypes.byref(nd), ctypes.byref(mm),
                                      None, 0) == 2
    assert nt.value == 24 * 41472 * 360  # sink products x written source terms x partitions
    assert b"max_terms" in L.mbc_last_error()
    bad = api._block_descs([dict(op="DI")])
    bad[0].op = 9
    h = ctypes.c_void_p()
    assert L.mbc_block_set_build(bad, 1, ctypes.byref(h)) == 1
    assert L.mbc_block_set_build(api._block_descs([dict(op="DI")]), 0, ctypes.byref(h)) == 1
    bad = api._block_descs([dict(op="proton", snk_spin=4)])
    assert L.mbc_block_set_build(bad, 1, ctypes.byref(h)) == 1
    assert L.mbc_block_set_dims(None, None, None, None, None, None) == 1
    bad = api._block_descs([dict(op="DI", src_pts=(0, 3))])
    assert L.mbc_block_set_build(bad, 1, ctypes.byref(h)) == 1
    assert b"source point" in L.mbc_last_error()
    L.mbc_block_set_free(None)
    L.mbc_block_plan_destroy(None)
    assert L.mbc_blocks_compute(None, None, None, 0, 1, None, None, None, 0, None) == 1
    assert L.mbc_block_contract(None, None, 1, 1, None, None, 0, None) == 1
    s = api.BlockSet([dict(op="DI", moms=[(0, 0, 0)] * 2)])
    n = ctypes.c_int64()
    assert L.mbc_block_set_factor_tree(s._h, 1, ctypes.byref(n), None, None) == 1
    assert L.mbc_block_set_factor_tree(s._h, -1, ctypes.byref(n), None, None) == 1


@pytest.mark.parametrize("corrs", [
    [dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)])],
    [dict(op="proton", moms=[(0, 0, 0)]), dict(op="DII", sign_mode="r2", moms=[(0, 1, 0), (0, 0, 0)]),
     dict(op="DII", moms=[(0, 0, 0)] * 2), dict(op="HE3_I", snk_spin=1, src_spin=2, moms=[(0, 0, 0)] * 3)],
])
def test_factor_trees_equal_the_oracle_construction_and_value(corrs):
    # the library's linearised trees (Sec. 4) against the oracle's prefix-tree
    # construction on the same terms, and their depth-first value against the
    # flat sum over the terms, with oracle blocks as factor values
    from oracle import factor_tree as FT
    dims, T = (2, 1, 1), 1
    S_u, S_d = synth.iid(T, 2, seed=33)
    bset = api.BlockSet(corrs)
    e = bset.export()
    blk = np.stack([OB.block(S_u, S_d, NAME[(fam, proj)], mom, dims) for fam, proj, mom in bset.types()],
                   axis=1).reshape(T, -1)[0]
    flat = contract_terms_with_oracle_blocks(bset, S_u, S_d, dims)[:, 0]
    for c in range(bset.n_corr):
        m = e["corr_id"] == c
        w = (e["num_re"][m] + 1j * e["num_im"][m]) / e["den"][c]
        terms = [(wk, tuple(int(x) for x in f if x >= 0)) for wk, f in zip(w, e["factor"][m])]
        factors, children, coefficients = FT.build(terms)
        fac, ch = bset.factor_tree(c)
        assert [None if x < 0 else int(x) for x in fac] == factors
        assert list(ch) == children
        val = FT.evaluate(factors, children, coefficients, lambda f: blk[f])
        assert abs(val - flat[c]) <= 1e-13 * max(1.0, abs(flat[c]))
        if m.any():
            A = int((e["factor"][m][0] >= 0).sum())
            assert len(fac) == 1 + len({tuple(f[:k]) for f in e["factor"][m].tolist() for k in range(1, A + 1)})


@pytest.mark.parametrize("corr", [
    dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)], src_pts=(0, 1)),
    dict(op="DII", moms=[(1, 0, 0), (-1, 0, 0)], src_pts=(1, 0)),
    dict(op="proton", snk_spin=2, src_spin=1, moms=[(1, 0, 0)], src_pts=(1,)),
])
def test_displaced_sources_reproduce_the_oracle_correlator(corr):
    # one propagator set per source point; mixed-source block types
    dims, T = (3, 1, 1), 1
    P = 1 + max(corr["src_pts"])
    S = [synth.iid(T, 3, seed=80 + p) for p in range(P)]
    S_u, S_d = np.stack([x[0] for x in S]), np.stack([x[1] for x in S])
    bset = api.BlockSet([corr])
    assert bset.n_points == P
    got = contract_terms_with_oracle_blocks(bset, S_u, S_d, dims)[0]
    ref = OB.block_correlator(S_u, S_d, corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0), "exact",
                              corr["moms"], dims, src_pts=corr["src_pts"])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    if corr["op"] == "DII":
        assert np.abs(ref).max() > 1.0
        assert any(z[0] != z[2] for *_, z in bset.types(with_points=True))  # mixed-source types occur

"""Linearised factor trees over arbitrary factor sets (Sec. 4) through the C
ABI (include/mbc_tree.h): validation of the paper's three arrays on the host
(no GPU), and GPU evaluation against the oracle's depth-first evaluator, the
Fig. 4 example's factorised form, and the block path's own tree kernel.
"""
import ctypes
import json
import os

import numpy as np
import pytest

from oracle import factor_tree as FT
from paper_2201_04269_amd import _binding as B

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "factor_tree_fig4.json")


def _create(factors, children, coefs, n_values):
    L = B.lib()
    f = np.ascontiguousarray(factors, dtype=np.int32)
    ch = np.ascontiguousarray(children, dtype=np.int32)
    c = np.asarray(coefs, dtype=np.complex128)
    cc = np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1).reshape(-1))
    h = ctypes.c_void_p()
    st = L.mbc_factor_tree_create(f.ctypes.data_as(ctypes.c_void_p), ch.ctypes.data_as(ctypes.c_void_p), f.shape[0],
                                  cc.ctypes.data_as(ctypes.c_void_p), c.shape[0], n_values, None, ctypes.byref(h))
    return st, L.mbc_last_error()


@pytest.mark.parametrize("factors,children,coefs,n_values,msg", [
    ([0, 1, 2], [1, 1, 0], [1], 3, b"root"),                     # root with a factor
    ([-1, 1, -1], [1, 1, 0], [1], 3, b"out of range"),           # a second -1
    ([-1, 0, 5], [1, 1, 0], [1], 3, b"out of range"),            # factor past the table
    ([-1, 0, 1], [2, 0, 0], [1, 2, 3], 3, b"leaves"),            # 2 leaves, 3 coefficients
    ([-1, 0, 1], [3, 0, 0], [1, 2], 3, b"more vertices"),        # children need a 4th vertex
    ([-1, 0, 1], [1, 0, 0], [1], 3, b"left over"),               # vertex 2 outside the tree
    ([-1, 0], [1, -1], [1], 3, b"negative"),
])
def test_inconsistent_arrays_are_rejected(factors, children, coefs, n_values, msg):
    st, err = _create(factors, children, coefs, n_values)
    assert st == 1 and msg in err, err
    L = B.lib()
    assert L.mbc_factor_tree_create(None, None, 0, None, 0, 0, None, None) == 1
    assert L.mbc_factor_tree_stats(None, None, None) == 1
    assert L.mbc_factor_tree_evaluate(None, None, 1, None, None, 0, None) == 1
    L.mbc_factor_tree_destroy(None)


def _fig4():
    g = json.load(open(GOLDEN))
    names = sorted({n for n in g["factors"] if n})
    idx = {n: i for i, n in enumerate(names)}
    return g, names, [-1 if n is None else idx[n] for n in g["factors"]]


@pytest.mark.gpu
def test_fig4_example_on_the_gpu():
    import torch
    from paper_2201_04269_amd import api
    g, names, factors = _fig4()
    t = api.FactorTree(factors, g["children"], g["coefficients"], len(names))
    assert t.depth == 2 and t.flops == 8 * 5
    rng = np.random.default_rng(3)
    vals = rng.standard_normal((3, len(names))) + 1j * rng.standard_normal((3, len(names)))
    got = t.evaluate(torch.from_numpy(vals).cuda()).cpu().numpy()
    v = {n: vals[:, i] for i, n in enumerate(names)}
    want = 5 * v["T1_122"] * v["T2_232"] + v["T1_123"] * (v["T2_232"] - v["T2_323"])
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(6))
def test_random_trees_equal_the_oracle(seed):
    import torch
    from paper_2201_04269_amd import api
    rng = np.random.default_rng(900 + seed)
    n_values = int(rng.integers(3, 40))
    depth = int(rng.integers(1, 8))
    terms = {}
    for _ in range(int(rng.integers(1, 60))):
        # strings of one length, so no string is a prefix of another
        terms[tuple(int(x) for x in rng.integers(0, n_values, size=depth))] = complex(*rng.standard_normal(2))
    factors, children, coefficients = FT.build([(c, f) for f, c in terms.items()])
    t = api.FactorTree([-1 if x is None else x for x in factors], children, coefficients, n_values)
    batch = 4
    vals = rng.standard_normal((batch, n_values)) + 1j * rng.standard_normal((batch, n_values))
    got = t.evaluate(torch.from_numpy(vals).cuda()).cpu().numpy()
    for b in range(batch):
        want = FT.evaluate(factors, children, coefficients, lambda f: vals[b, f])
        assert abs(got[b] - want) <= 1e-13 * max(1.0, abs(want))


@pytest.mark.gpu
def test_degenerate_trees():
    import torch
    from paper_2201_04269_amd import api
    t = api.FactorTree([-1], [0], [], 0)  # the root alone: no paths, value 0
    out = t.evaluate(torch.zeros((2, 0), dtype=torch.complex128, device="cuda"))
    assert torch.equal(out, torch.zeros(2, dtype=torch.complex128, device="cuda"))
    n = 60  # a chain: the product of 59 factors times the coefficient
    t = api.FactorTree([-1] + list(range(n - 1)), [1] * (n - 1) + [0], [2.0], n - 1)
    assert t.depth == n - 1
    vals = np.exp(1j * np.linspace(0, 1, n - 1))[None, :]
    got = t.evaluate(torch.from_numpy(vals).cuda()).item()
    assert abs(got - 2 * np.prod(vals)) <= 1e-13


@pytest.mark.gpu
def test_block_set_trees_equal_the_block_tree_kernel():
    # the generic evaluator on a block set's trees, with the blocks as the
    # factor table, against the block path's specialised tree kernel
    import torch
    from paper_2201_04269_amd import api, synth
    corrs = [dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)]), dict(op="proton", snk_spin=1, src_spin=2, moms=[(0, 0, 0)])]
    bset = api.BlockSet(corrs)
    plan = api.BlockPlan(bset)
    Su, Sd = synth.iid(3, 8, seed=11)
    blk = api.blocks(plan, torch.from_numpy(Su).cuda(), torch.from_numpy(Sd).cuda(), (2, 2, 2))
    ref = api.block_contract(plan, blk, method="tree").cpu().numpy()
    e = bset.export()
    table = blk.reshape(blk.shape[0], -1).contiguous()
    for c in range(bset.n_corr):
        fac, ch = bset.factor_tree(c)
        m = e["corr_id"] == c
        w = (e["num_re"][m] + 1j * e["num_im"][m]) / e["den"][c]
        t = api.FactorTree(fac, ch, w, table.shape[1])
        got = t.evaluate(table).cpu().numpy()
        assert np.abs(got - ref[c]).max() <= 1e-12 * np.abs(ref[c]).max()

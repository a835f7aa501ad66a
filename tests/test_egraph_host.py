"""Host side of the tensor e-graph (Sec. 5): libmbc's canonical forms, e-graph
and extracted plan against the oracle's, exactly (no GPU).

Classes, canonical codes, e-nodes, term classes and signs, and the plan steps
must be identical: both sides follow the same documented construction order,
the oracle by brute force over every arrangement.
"""
import ctypes

import numpy as np
import pytest

from oracle import egraph as E
from paper_2201_04269_amd import _binding as B
from paper_2201_04269_amd import api

from test_oracle_egraph import _random_expr, _tensors


def _lib_tensors(T):
    out = []
    for t in sorted(T):
        vals, group, ext = T[t]
        gens = [(p, s) for p, s in group[1:]][:4]
        out.append((ext, gens))
    return out


def _compare(g, og, objective):
    ex = g.export()
    assert len(ex["classes"]) == len(og.cls)
    for c, oc in zip(ex["classes"], og.cls):
        assert c["code"] == tuple(oc["code"])
        assert c["n_factors"] == len(oc["factors"]) and c["n_open"] == oc["n_open"]
        assert c["nodes"] == [(a, b, s, tuple(o1), tuple(o2)) for a, b, s, o1, o2 in oc["nodes"]]
    assert [(c, o) for c, o in ex["terms"]] == [(c, tuple(o)) for c, _, o in og.roots]
    assert np.allclose(ex["coefs"], [c for _, c, _ in og.roots], rtol=0, atol=0)
    steps, _ = og.plan(objective)
    got = [(c, ex["classes"][c]["nodes"][i]) for c, i in ex["steps"]]
    assert got == [(c, (a, b, s, tuple(o1), tuple(o2))) for c, (a, b, s, o1, o2) in steps]
    assert g.stats["saturated"] == int(og.saturated)
    assert g.stats["n_nodes"] == og.n_nodes


def test_paper_example_matches_the_oracle():
    groups = {0: E.closure(E.EPS_GENS, 3), 1: E.closure([], 3)}
    expr = [(0, (0, 1, 2)), (0, (3, 4, 5)), (1, (0, 1, 3)), (1, (5, 4, 2))]
    og = E.EGraph(groups, {0: (3, 3, 3), 1: (3, 3, 3)}).build([(1.0, expr)], 1000)
    g = api.TensorEGraph([((3, 3, 3), E.EPS_GENS), ((3, 3, 3), [])], [(1.0, expr)], 1000, "reuse")
    _compare(g, og, "reuse")
    gf = api.TensorEGraph([((3, 3, 3), E.EPS_GENS), ((3, 3, 3), [])], [(1.0, expr)], 1000, "flops")
    _compare(gf, og, "flops")
    gs = api.TensorEGraph([((3, 3, 3), E.EPS_GENS), ((3, 3, 3), [])], [(1.0, expr)], 1000, "shared")
    _compare(gs, og, "shared")
    assert gs.export()["steps"] == gf.export()["steps"]  # B_kl B_lk is already the cheapest
    assert gf.stats["n_steps"] == 2 and gf.stats["flops_plan"] < g.stats["flops_direct"]


@pytest.mark.parametrize("seed", range(16))
@pytest.mark.parametrize("objective", ["reuse", "flops", "shared"])
def test_random_sums_match_the_oracle_exactly(seed, objective):
    rng = np.random.default_rng(300 + seed)
    T = _tensors(rng)
    groups = {t: v[1] for t, v in T.items()}
    ext = {t: v[2] for t, v in T.items()}
    n_open = int(rng.integers(0, 3))
    terms = [(complex(rng.standard_normal(), rng.standard_normal()), _random_expr(rng, int(rng.integers(2, 6)), n_open))
             for _ in range(int(rng.integers(1, 4)))]
    opens = {tuple(sorted(x for _, l in e for x in l if x >= 40)) for _, e in terms}
    if len(opens) != 1:
        pytest.skip("terms with different open labels")
    limit = int(rng.choice([3, 1000]))
    try:
        og = E.EGraph(groups, ext).build(terms, limit)
    except ValueError:
        with pytest.raises(B.MbcError):
            api.TensorEGraph(_lib_tensors(T), terms, limit, objective)
        return
    g = api.TensorEGraph(_lib_tensors(T), terms, limit, objective)
    _compare(g, og, objective)


def test_generator_lists_give_the_same_groups():
    # the library gets generators (the first elements past the identity);
    # their closure must be the oracle's group
    T = _tensors(np.random.default_rng(0))
    for t, (vals, group, ext) in T.items():
        gens = [(p, s) for p, s in group[1:]][:4]
        assert sorted(E.closure(gens, len(ext))) == sorted(group)


def test_bad_input_is_rejected():
    L = B.lib()
    eps = ((3, 3, 3), E.EPS_GENS)
    with pytest.raises(B.MbcError, match="more than twice"):
        api.TensorEGraph([eps], [(1.0, [(0, (0, 0, 0))])])
    with pytest.raises(B.MbcError, match="different open labels"):
        api.TensorEGraph([eps], [(1.0, [(0, (0, 1, 2))]), (1.0, [(0, (0, 1, 3))])])
    with pytest.raises(B.MbcError, match="permutation"):
        api.TensorEGraph([((3, 3, 3), [((0, 0, 1), 1)])], [(1.0, [(0, (0, 1, 2))])])
    with pytest.raises(B.MbcError, match="vanishes"):
        api.TensorEGraph([((3, 3), [((1, 0), -1), ((1, 0), 1)])], [(1.0, [(0, (0, 1))])])
    with pytest.raises(B.MbcError, match="two extents"):
        api.TensorEGraph([eps, ((4, 4), [])], [(1.0, [(0, (0, 1, 2)), (1, (0, 1))])])
    with pytest.raises(B.MbcError, match="label out of range"):
        api.TensorEGraph([eps], [(1.0, [(0, (0, 1, 64))])])
    h = ctypes.c_void_p()
    assert L.mbc_egraph_build(None, 0, None, None, None, 0, 0, 0, ctypes.byref(h)) == 1
    assert L.mbc_egraph_get_stats(None, None) == 1
    assert L.mbc_egraph_execute(None, None, None, 1, None, None, 0, None) == 1
    L.mbc_egraph_free(None)
    # a vanishing term is dropped: eps_ijk S_ij with S symmetric
    g = api.TensorEGraph([eps, ((3, 3), [((1, 0), 1)])], [(1.0, [(0, (0, 1, 2)), (1, (0, 1))])])
    assert g.stats["n_roots"] == 0 and g.stats["out_elems"] == 3


def _oracle_ids(bset):
    ids = {}
    for k, (fam, proj, mom, z) in enumerate(bset.types(with_points=True)):
        name = {("p", 0): "p", ("n", 0): "n", ("p", 1): "p+", ("p", -1): "p-", ("n", 1): "n+", ("n", -1): "n-"}[(fam, proj)]
        ids[("block", name, tuple(mom), tuple(z))] = k
    n = bset.n_types
    ids[("eps",)] = n
    for j, p in enumerate((0, 1, -1)):
        ids[("gamma", p)] = n + 1 + j
    for j in range(4):
        ids[("unit", j)] = n + 4 + j
    return ids


@pytest.mark.parametrize("corr", [dict(op="proton", snk_spin=1, src_spin=2, moms=[(1, 0, 0)]),
                                  dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)])])
def test_block_expressions_match_the_oracle_canonically(corr):
    # every term of the library's expansion has the canonical class and sign of
    # the oracle's expression for it (oracle canonical forms by brute force)
    bset = api.BlockSet([corr])
    g = api.TensorEGraph.for_blocks(bset, 0, node_limit=0)
    ex = g.export()
    terms = E.block_expressions(corr["op"], corr.get("snk_spin", 0), corr.get("src_spin", 0), "exact", corr["moms"])
    ids = _oracle_ids(bset)
    groups = {}
    n = bset.n_types
    for k in range(n):
        groups[k] = E.closure([E.BLOCK_SWAP], 7)
    groups[n] = E.closure(E.EPS_GENS, 3)
    for j in range(3):
        groups[n + 1 + j] = E.closure(E.ANTISYM2, 2)
    for j in range(4):
        groups[n + 4 + j] = E.closure([], 1)
    assert len(ex["terms"]) == len(terms)
    for (cls, _), coef, (ocoef, factors) in zip(ex["terms"], ex["coefs"], terms):
        code, sign, _, _ = E.canonical([(ids[nm], lab) for nm, lab in factors], groups)
        assert ex["classes"][cls]["code"] == tuple(code)
        assert abs(coef - ocoef * sign) < 1e-15


def _bset_with_types(corr):
    # exact-sign D_II adds no block types of its own; D_I supplies them
    return api.BlockSet([corr, dict(op="DI", moms=[(0, 0, 0)] * 2)])


def test_exact_dii_cancels_and_r2_is_twice_di_by_canonical_forms():
    # Appendix-C-type identities found structurally: at one source point the
    # 36 terms of exact-sign D_II fall into 9 canonical classes whose summed
    # coefficients are exactly zero, and under R2 every class carries exactly
    # twice D_I's coefficient (C_DII = 2 C_DI)
    roots = {}
    for name, corr in (("exact", dict(op="DII", moms=[(0, 0, 0)] * 2)),
                       ("r2", dict(op="DII", sign_mode="r2", moms=[(0, 0, 0)] * 2)),
                       ("di", dict(op="DI", moms=[(0, 0, 0)] * 2))):
        g = api.TensorEGraph.for_blocks(_bset_with_types(corr), 0, 100000)
        ex = g.export()
        acc = {}
        for (c, o), k in zip(ex["terms"], ex["coefs"]):
            acc[(ex["classes"][c]["code"], o)] = acc.get((ex["classes"][c]["code"], o), 0) + k
        roots[name] = (acc, g.stats)
    acc, st = roots["exact"]
    assert st["n_terms"] == 36 and len(acc) == 9 and all(v == 0 for v in acc.values())
    assert st["n_roots"] == 0 and st["n_steps"] == 0
    r2, di = roots["r2"][0], roots["di"][0]
    assert set(r2) == set(di) and all(r2[k] == 2 * di[k] for k in di)


def test_sharing_aware_extraction_lowers_the_dinucleon_plan():
    bset = api.BlockSet([dict(op="DI", moms=[(1, 0, 0), (-1, 0, 0)])])
    f = api.TensorEGraph.for_blocks(bset, 0, 100000, "flops").stats["flops_plan"]
    s = api.TensorEGraph.for_blocks(bset, 0, 100000, "shared").stats["flops_plan"]
    assert s < 0.95 * f


def test_the_papers_dii_subexpressions_are_shared_classes():
    # Sec. 5 names two common sub-expressions of the D_II correlator: B1 (both
    # blocks, two eps, two C gamma5; four open spins) and B2 (both blocks,
    # four C gamma5; six open colours).  The saturated e-graph holds classes
    # of both shapes, each with several parent classes.
    bset = _bset_with_types(dict(op="DII", sign_mode="r2", moms=[(0, 0, 0)] * 2))
    g = api.TensorEGraph.for_blocks(bset, 0, 100000)
    assert g.stats["saturated"] == 1
    ex = g.export()
    n = bset.n_types
    rank = {**{t: 7 for t in range(n)}, n: 3, n + 1: 2, n + 2: 2, n + 3: 2, **{n + 4 + j: 1 for j in range(4)}}
    ext = lambda t, k: (4, 3, 4, 3, 4, 3, 4)[k] if t < n else (3 if t == n else 4)
    parents = {}
    for cid, c in enumerate(ex["classes"]):
        for nd in c["nodes"]:
            for k in set(nd[:2]):
                parents.setdefault(k, set()).add(cid)
    shapes = {"B1": [], "B2": []}
    for cid, c in enumerate(ex["classes"]):
        code, p, kinds, opens = c["code"], 0, [], []
        while p < len(code):
            t = code[p]
            kinds.append("blk" if t < n else ("eps" if t == n else "gam" if t < n + 4 else "unit"))
            opens += [ext(t, k) for k in range(rank[t]) if code[p + 1 + k] & 1]
            p += 1 + rank[t]
        kinds, opens = sorted(kinds), sorted(opens)
        if kinds == ["blk", "blk", "eps", "eps", "gam", "gam"] and opens == [4] * 4:
            shapes["B1"].append(len(parents.get(cid, ())))
        if kinds == ["blk", "blk", "gam", "gam", "gam", "gam"] and opens == [3] * 6:
            shapes["B2"].append(len(parents.get(cid, ())))
    assert shapes["B1"] and max(shapes["B1"]) >= 2
    assert shapes["B2"] and max(shapes["B2"]) >= 2


def _random_expr_with_traces(rng, n_factors, n_open):
    """Like _random_expr, but with a factor that repeats a label (a trace)
    whenever the shape allows one (else the last draw is returned)."""
    for attempt in range(400):
        fac = [int(rng.choice((0, 1, 3, 4, 5))) for _ in range(n_factors)]
        ranks = [3 if t in (0, 3, 4) else 2 for t in fac]
        slots = sum(ranks)
        if (slots - n_open) % 2 or slots < n_open:
            continue
        labels = list(range((slots - n_open) // 2)) * 2 + list(range(40, 40 + n_open))
        rng.shuffle(labels)
        out, p = [], 0
        for t, r in zip(fac, ranks):
            out.append((t, tuple(int(x) for x in labels[p:p + r])))
            p += r
        if any(len(set(l)) < len(l) for _, l in out):
            return out
    return _random_expr(rng, max(n_factors, 2), n_open)


@pytest.mark.parametrize("seed", range(12))
def test_sums_with_traces_match_the_oracle_exactly(seed):
    rng = np.random.default_rng(700 + seed)
    T = _tensors(rng)
    groups = {t: v[1] for t, v in T.items()}
    ext = {t: v[2] for t, v in T.items()}
    n_open = int(rng.integers(0, 3))
    terms = [(complex(rng.standard_normal(), rng.standard_normal()),
              _random_expr_with_traces(rng, int(rng.integers(1, 5)), n_open)) for _ in range(2)]
    if len({tuple(sorted(x for _, l in e for x in l if x >= 40)) for _, e in terms}) != 1:
        pytest.skip("terms with different open labels")
    try:
        og = E.EGraph(groups, ext).build(terms, 500)
    except ValueError:
        with pytest.raises(B.MbcError):
            api.TensorEGraph(_lib_tensors(T), terms, 500, "flops")
        return
    g = api.TensorEGraph(_lib_tensors(T), terms, 500, "flops")
    _compare(g, og, "flops")

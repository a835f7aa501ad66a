"""Pins of the oracle's tensor e-graph (Sec. 5).

Each check takes a route that does not reuse the canonicalisation: the
paper's worked example (tests/golden/egraph_sec5_example.json), numeric
evaluation of expressions against their canonical forms and of extracted
plans against the direct contraction, group orders of the symmetries, and the
block-level correlator of oracle.blocks (itself pinned against a determinant
brute force) for the correlator expressions.
"""
import json
import os

import numpy as np
import pytest

from oracle import blocks as OB
from oracle import egraph as E
from paper_2201_04269_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "egraph_sec5_example.json")


def _eps():
    return E.constant_tensor(("eps",))


def _tensors(rng):
    """id -> (values, closure, extents): eps, an antisymmetric 3x3, a symmetric
    3x3, two generic rank-3 and one generic rank-2 tensor."""
    a = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    return {0: (_eps(), E.closure(E.EPS_GENS, 3), (3, 3, 3)),
            1: (a - a.T, E.closure(E.ANTISYM2, 2), (3, 3)),
            2: (a + a.T, E.closure([((1, 0), 1)], 2), (3, 3)),
            3: (rng.standard_normal((3, 3, 3)) + 1j * rng.standard_normal((3, 3, 3)), E.closure([], 3), (3, 3, 3)),
            4: (rng.standard_normal((3, 3, 3)) + 1j * rng.standard_normal((3, 3, 3)), E.closure([], 3), (3, 3, 3)),
            5: (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)), E.closure([], 2), (3, 3))}


def _random_expr(rng, n_factors, n_open, tids=(0, 1, 3, 4, 5)):
    """A product of n_factors tensors whose slots pair up, leaving n_open open labels."""
    while True:
        fac = [int(rng.choice(tids)) for _ in range(n_factors)]
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
        if all(len(set(l)) == len(l) for _, l in out):
            return out


def _value(expr, T, out):
    args = []
    for t, lab in expr:
        args += [T[t][0], list(lab)]
    return np.einsum(*args, list(out))


def test_symmetry_groups_have_the_expected_orders_and_signs():
    g = E.closure(E.EPS_GENS, 3)
    assert len(g) == 6
    for p, s in g:
        inv = sum(p[i] > p[j] for i in range(3) for j in range(i + 1, 3))
        assert s == (-1) ** inv
    assert len(E.closure([E.BLOCK_SWAP], 7)) == 2
    with pytest.raises(ValueError):
        E.closure([((0, 1), -1)], 2)  # T = -T: the tensor vanishes


def test_paper_example_finds_the_common_subexpression():
    gold = json.load(open(GOLD))
    tid = {"eps": 0, "T": 1}
    expr = [(tid[n], tuple(l)) for n, l in gold["factors"]]
    groups = {0: E.closure(E.EPS_GENS, 3), 1: E.closure([], 3)}
    g = E.EGraph(groups, {0: (3, 3, 3), 1: (3, 3, 3)}).build([(1.0, expr)], 1000)
    # the two sub-expressions of the example canonicalise to one class with
    # the relative sign of the example
    subs = [E.canonical([(tid[n], tuple(l)) for n, l in part], groups) for part in gold["subexpressions"]]
    assert subs[0][0] == subs[1][0]
    assert [list(x[2]) for x in subs] == gold["subexpression_open_labels"]
    assert subs[0][1] * subs[1][1] == gold["subexpression_sign_product"]
    root, coef, _ = g.roots[0]
    shared = [n for n in g.cls[root]["nodes"] if n[0] == n[1]]
    assert shared, "the root class has an e-node whose two children are one class"
    B_cls = g.cls[shared[0][0]]
    assert [t for t, _ in B_cls["factors"]] == [0, 1] and B_cls["n_open"] == 2
    # numerically: E = -B_kl B_lk with B_kl = eps_ijk T_ijl
    rng = np.random.default_rng(1)
    T = rng.standard_normal((3, 3, 3)) + 1j * rng.standard_normal((3, 3, 3))
    B = np.einsum("ijk,ijl->kl", _eps(), T)
    direct = E.evaluate([(1.0, expr)], {0: _eps(), 1: T}, [])
    assert abs(direct - (-np.einsum("kl,lk->", B, B))) <= 1e-13 * abs(direct)
    for objective in ("reuse", "flops"):
        assert abs(g.evaluate_plan({0: _eps(), 1: T}, [], objective) - direct) <= 1e-13 * abs(direct)
    # the cheapest plan is the example's: B once, then the root from B_kl B_lk
    steps, flops = g.plan("flops")
    assert len(steps) == 2 and steps[0][0] == shared[0][0]
    assert flops == 8 * 81 + 8 * 9


@pytest.mark.parametrize("seed", range(12))
def test_canonical_form_is_invariant_and_equal_in_value(seed):
    rng = np.random.default_rng(100 + seed)
    T = _tensors(rng)
    groups = {t: v[1] for t, v in T.items()}
    expr = _random_expr(rng, int(rng.integers(2, 5)), int(rng.integers(0, 3)))
    code, sign, opens, arr = E.canonical(expr, groups)
    if sign == 0:
        assert np.abs(_value(expr, T, sorted({x for _, l in expr for x in l if sum(x in m for _, m in expr) == 1}))).max() < 1e-12
        return
    # value: E[opens] = sign x canonical expression[open codes]
    cf = E.relabelled(expr, arr, code)
    v = _value(expr, T, list(opens))
    w = sign * _value(cf, T, [2 * k + 1 for k in range(len(opens))])
    assert np.abs(v - w).max() <= 1e-12 * max(1.0, np.abs(v).max())
    # a relabelled, reordered, symmetry-rewritten copy has the same code, and
    # the sign and open map describe it correctly
    perm = {x: int(y) for x, y in zip(sorted({x for _, l in expr for x in l}), rng.permutation(50))}
    copy, tracked = [], 1
    for t, lab in expr:
        p, s = T[t][1][int(rng.integers(len(T[t][1])))]
        copy.append((t, tuple(perm[lab[p[k]]] for k in range(len(p)))))
        tracked *= s
    order = rng.permutation(len(copy))
    copy = [copy[i] for i in order]
    code2, sign2, opens2, _ = E.canonical(copy, groups)
    assert code2 == code
    v2 = _value(copy, T, list(opens2))
    assert np.abs(v2 - sign2 * _value(cf, T, [2 * k + 1 for k in range(len(opens2))])).max() <= 1e-12 * max(1.0, np.abs(v2).max())
    # and the copy is the original times the signs of the symmetries applied
    cv = _value(copy, T, [perm[x] for x in opens])
    assert np.abs(cv - tracked * v).max() <= 1e-12 * max(1.0, np.abs(v).max())


def test_vanishing_expressions_are_detected():
    rng = np.random.default_rng(3)
    T = _tensors(rng)
    groups = {t: v[1] for t, v in T.items()}
    # eps_ijk S_ij with S symmetric, and A_ij S_ij with A antisymmetric
    for expr in ([(0, (0, 1, 9)), (2, (0, 1))], [(1, (0, 1)), (2, (0, 1))]):
        assert E.canonical(expr, groups)[1] == 0
        out = [x for _, l in expr for x in l if sum(x in m for _, m in expr) == 1]
        assert np.abs(_value(expr, T, out)).max() < 1e-12


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("objective", ["reuse", "flops", "shared"])
def test_extracted_plan_equals_the_direct_contraction(seed, objective):
    rng = np.random.default_rng(200 + seed)
    T = _tensors(rng)
    groups = {t: v[1] for t, v in T.items()}
    ext = {t: v[2] for t, v in T.items()}
    n_open = int(rng.integers(0, 3))
    terms = []
    exprs = [_random_expr(rng, int(rng.integers(2, 6)), n_open) for _ in range(3)]
    outs = [sorted(x for _, l in e for x in l if x >= 40) for e in exprs]
    for e, o in zip(exprs, outs):
        terms.append((complex(rng.standard_normal(), rng.standard_normal()), e))
    out = outs[0]
    if any(o != out for o in outs):
        pytest.skip("terms with different open labels")
    vals = {t: v[0] for t, v in T.items()}
    try:
        g = E.EGraph(groups, ext).build(terms, 400)
    except ValueError:
        return  # a vanishing sub-expression
    direct = E.evaluate(terms, vals, out)
    got = g.evaluate_plan(vals, out, objective)
    assert np.abs(np.asarray(got) - direct).max() <= 1e-12 * max(1.0, np.abs(direct).max())


@pytest.mark.parametrize("op,s,sp,mode,moms,pts", [
    ("DI", 0, 0, "exact", [(1, 0, 0), (-1, 0, 0)], None),
    ("DII", 0, 0, "r2", [(1, 0, 0), (0, 0, 0)], None),
    ("proton", 1, 2, "exact", [(1, 0, 0)], None),
    ("DII", 0, 0, "exact", [(1, 0, 0), (-1, 0, 0)], (0, 1)),
    ("HE3_I", 1, 3, "exact", [(1, 0, 0), (0, 0, 0), (-1, 0, 0)], None),
])
def test_block_expressions_equal_the_block_level_correlator(op, s, sp, mode, moms, pts):
    P = 1 if pts is None else 2
    S = [synth.iid(1, 3, seed=40 + p) for p in range(P)]
    Su = S[0][0] if P == 1 else np.stack([x[0] for x in S])
    Sd = S[0][1] if P == 1 else np.stack([x[1] for x in S])
    dims = (3, 1, 1)
    terms = E.block_expressions(op, s, sp, mode, moms, pts)
    cache = {}

    def value(name):
        if name[0] != "block":
            return E.constant_tensor(name)
        if name not in cache:
            cache[name] = OB.block(Su, Sd, name[1], name[2], dims, srcs=name[3])[0].reshape(E.BLOCK_EXT)
        return cache[name]

    got = E.evaluate_named(terms, value)
    ref = OB.block_correlator(Su, Sd, op, s, sp, mode, moms, dims, src_pts=pts)[0]
    assert abs(got - ref) <= 1e-13 * abs(ref)
    assert abs(ref) > 1e-3


# ---------------------------------------------------------------------------
# Extraction choices pinned on hand-worked examples (Sec. 5 objective)
# ---------------------------------------------------------------------------
def _chain_graph(ext, labels, node_limit=1000):
    groups = {t: E.closure([], len(e)) for t, e in ext.items()}
    expr = [(t, lab) for t, lab in labels]
    return E.EGraph(groups, ext).build([(1.0, expr)], node_limit), expr


def test_tree_cost_picks_the_cheapest_order_of_a_three_factor_chain():
    # A_ij (2 x 8) B_jk (8 x 8) C_kl (8 x 8), open i, l.  By hand, at 8 flops
    # per complex multiply-add over the labels of the two operands:
    #   (A B) C: 8 (2*8*8) + 8 (2*8*8)       =  2048
    #   A (B C): 8 (8*8*8) + 8 (2*8*8)       =  5120
    #   (A C) B: 8 (2*8*8*8) + 8 (2*8*8*8)   = 16384  (A C is an outer product)
    # catches a cost model that counts only the result's labels, or a pick of
    # the first admitted split instead of the cheapest tree
    g, expr = _chain_graph({0: (2, 8), 1: (8, 8), 2: (8, 8)}, [(0, (0, 1)), (1, (1, 2)), (2, (2, 3))])
    steps, flops = g.plan("flops")
    assert flops == 2048 and len(steps) == 2
    first = g.cls[steps[0][0]]
    assert sorted(t for t, _ in first["factors"]) == [0, 1]  # A B first
    rng = np.random.default_rng(5)
    T = {t: rng.standard_normal(e) + 1j * rng.standard_normal(e) for t, e in ((0, (2, 8)), (1, (8, 8)), (2, (8, 8)))}
    direct = E.evaluate([(1.0, expr)], T, [0, 3])
    assert np.allclose(g.evaluate_plan(T, [0, 3], "flops"), direct, rtol=1e-13, atol=0)


def test_tree_cost_of_a_vector_matrix_chain():
    # v_i M_ij N_jk u_k (all extents 8), a scalar.  Every order that never
    # forms M N costs 8 (64 + 64 + 8) = 1088 by hand (v M, then with N, then
    # with u; or v M and N u, then their dot product); forming M N first
    # costs 8 (512 + ...) and more
    ext = {0: (8,), 1: (8, 8), 2: (8, 8), 3: (8,)}
    g, expr = _chain_graph(ext, [(0, (0,)), (1, (0, 1)), (2, (1, 2)), (3, (2,))])
    steps, flops = g.plan("flops")
    assert flops == 1088 and len(steps) == 3


def test_reuse_objective_scores_on_the_paper_example_by_hand():
    """The reuse objective (excess parents from distinct e-classes x flops,
    read per child class) on E = eps_ijk eps_lmn T_ijl T_nmk, by hand.

    Saturated, the e-graph holds these 2-factor classes, with their parent
    classes (classes that have an e-node using them) and direct costs:
      eps eps (outer, 3^6 points):   parents E, eps eps T         -> 2, 8*729 = 5832
      T T (outer, 3^6 points):       parents E, eps T T           -> 2, 5832
      B_kl = eps_ijk T_ijl (3^4):    parents E, eps eps T, eps T T -> 3, 8*81 = 648
      eps_ijk T_nmk (one shared, 3^5): parents E, eps eps T, eps T T -> 3, 8*243 = 1944
    so the root's e-nodes score (eps eps)(T T): 5832 + 5832 = 11664,
    (eps T_nmk)^2: 2*1944 = 3888, B_kl B_lk: 2*648 = 1296, and splits with a
    3-factor child (one parent each) 0: the objective picks (eps eps)(T T),
    not the example's B_kl B_lk, which the smallest tree cost picks.
    """
    gold = json.load(open(GOLD))
    tid = {"eps": 0, "T": 1}
    expr = [(tid[n], tuple(l)) for n, l in gold["factors"]]
    groups = {0: E.closure(E.EPS_GENS, 3), 1: E.closure([], 3)}
    g = E.EGraph(groups, {0: (3, 3, 3), 1: (3, 3, 3)}).build([(1.0, expr)], 1000)
    npar = g.n_parents()
    two = {}
    for cid in range(len(g.cls)):
        c = g.cls[cid]
        if g.find(cid) == cid and len(c["factors"]) == 2:
            key = (tuple(sorted(t for t, _ in c["factors"])), c["n_open"])
            two[key] = (npar[cid], g.naive_flops(cid))
    assert two == {((0, 0), 6): (2, 5832), ((1, 1), 6): (2, 5832), ((0, 1), 2): (3, 648), ((0, 1), 4): (3, 1944)}
    root = g.roots[0][0]
    choice = g.extract("reuse")
    n = g.cls[root]["nodes"][choice[root]]
    kids = sorted(tuple(sorted(t for t, _ in g.cls[g.find(k)]["factors"])) for k in n[:2])
    assert kids == [(0, 0), (1, 1)]  # (eps eps)(T T)
    n = g.cls[root]["nodes"][g.extract("flops")[root]]
    assert n[0] == n[1] and g.cls[g.find(n[0])]["n_open"] == 2  # B_kl B_lk

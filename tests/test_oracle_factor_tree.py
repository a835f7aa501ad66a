"""Pins of the oracle's linearised factor trees (Sec. 4).

The worked example of Fig. 4 (its printed factors / children / coefficients
arrays, tests/golden/factor_tree_fig4.json) fixes the construction; the
evaluation is checked against the term-by-term sum and against the
factorised form the figure prints.
"""
import json
import os

import numpy as np
import pytest

from oracle import factor_tree as FT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "factor_tree_fig4.json")


def test_fig4_linearised_arrays():
    g = json.load(open(GOLDEN))
    terms = [(c, tuple(f)) for c, f in g["terms"]]
    factors, children, coefficients = FT.build(terms)
    assert factors == g["factors"]
    assert children == g["children"]
    assert coefficients == g["coefficients"]


def test_fig4_evaluation_equals_the_factorised_form():
    g = json.load(open(GOLDEN))
    rng = np.random.default_rng(1)
    T1 = rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4))
    T2 = rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4))

    def value(name):
        T = T1 if name.startswith("T1") else T2
        i, j, k = (int(d) for d in name.split("_")[1])
        return T[i, j, k]

    tree = FT.evaluate(g["factors"], g["children"], g["coefficients"], value)
    factorised = 5 * T1[1, 2, 2] * T2[2, 3, 2] + T1[1, 2, 3] * (T2[2, 3, 2] - T2[3, 2, 3])
    assert abs(tree - factorised) <= 1e-14 * abs(factorised)
    assert abs(FT.direct([(c, tuple(f)) for c, f in g["terms"]], value) - factorised) <= 1e-14 * abs(factorised)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_expressions_tree_equals_direct_sum(seed):
    rng = np.random.default_rng(seed)
    depth = 1 + seed
    terms = []
    for _ in range(300):
        fac = tuple(int(v) for v in rng.integers(0, 6, size=depth))
        terms.append((int(rng.integers(-3, 4)), fac))
    vals = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    factors, children, coefficients = FT.build(terms)
    prefixes = {fac[:k] for _, fac in terms for k in range(1, depth + 1)}
    assert len(factors) == 1 + len(prefixes)
    assert sum(children) == len(factors) - 1
    assert len(coefficients) == len({fac for _, fac in terms})
    got = FT.evaluate(factors, children, coefficients, lambda f: vals[f])
    want = FT.direct(terms, lambda f: vals[f])
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_a_string_that_prefixes_another_is_rejected():
    with pytest.raises(ValueError):
        FT.build([(1, ("a", "b")), (2, ("a",))])
    with pytest.raises(ValueError):
        FT.build([(2, ("a",)), (1, ("a", "b"))])

"""Linearised factor trees (Sec. 4), plain Python.

TEST INFRASTRUCTURE ONLY: like the rest of ``oracle``, nothing in the library
imports or calls this module.

A factor tree represents a sum of products sum_k w_k prod_i F_{k,i}: every
term is a root-to-leaf path whose vertices carry the factors, and the leaf
carries the coefficient; the sum of the coefficient-weighted products of all
root-to-leaf paths is the expression.  Terms that begin with the same
factors share those vertices, so the shared factors are multiplied once.

The linearised form (Sec. 4) is three arrays in depth-first order of the
vertices: ``factors`` (None for the root), ``children`` (the number of
children of each vertex) and ``coefficients`` (the leaf coefficients).

Here the tree of a list of terms is their prefix tree: the children of a
vertex appear in the order in which the terms first use them.
"""


def build(terms):
    """Linearised factor tree of terms [(coef, (F_1, .., F_n)), ...].

    Identical factor strings are merged (coefficients added).  A string may
    not be a proper prefix of another (the paths end at leaves).
    Returns (factors, children, coefficients).
    """
    root = {"f": None, "kids": [], "index": {}, "coef": None}
    for coef, fac in terms:
        node = root
        for f in fac:
            if node["coef"] is not None:
                raise ValueError("a factor string is a prefix of another")
            if f not in node["index"]:
                child = {"f": f, "kids": [], "index": {}, "coef": None}
                node["index"][f] = child
                node["kids"].append(child)
            node = node["index"][f]
        if node["kids"]:
            raise ValueError("a factor string is a prefix of another")
        node["coef"] = coef if node["coef"] is None else node["coef"] + coef
    factors, children, coefficients = [], [], []

    def visit(node):
        factors.append(node["f"])
        children.append(len(node["kids"]))
        if not node["kids"] and node is not root:
            coefficients.append(node["coef"])
        for k in node["kids"]:
            visit(k)

    visit(root)
    return factors, children, coefficients


def evaluate(factors, children, coefficients, value):
    """Sum over root-to-leaf paths of coefficient x product of factor values.

    Depth-first over the linearised arrays: a vertex's value is its factor's
    value (1 for the root) times the sum of its children's values, a leaf's
    the factor's value times its coefficient.  ``value`` maps a factor to a
    number.
    """
    pos = 0
    leaf = 0

    def visit():
        nonlocal pos, leaf
        i = pos
        pos += 1
        if children[i] == 0 and i != 0:
            s = coefficients[leaf]
            leaf += 1
        else:
            s = sum(visit() for _ in range(children[i]))
        return s if factors[i] is None else value(factors[i]) * s

    total = visit()
    if pos != len(factors) or leaf != len(coefficients):
        raise ValueError("inconsistent linearised tree")
    return total


def direct(terms, value):
    """The same expression term by term: sum_k w_k prod_i value(F_{k,i})."""
    tot = 0
    for coef, fac in terms:
        p = coef
        for f in fac:
            p = p * value(f)
        tot += p
    return tot

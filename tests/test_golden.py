"""The oracle against the committed fixtures under tests/golden/."""
import json
import os

import pytest

from oracle import operators as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_hand_derived_proton_identity_fixture():
    vals = {}
    for line in open(os.path.join(HERE, "proton_identity.txt")):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=")
            vals[k.strip()] = int(v)
    w = O.sink_tensor("proton", 0)
    sw2 = sum(c[0] ** 2 + c[1] ** 2 for c in w.values())
    assert O.grassmann_sigma(2, 1) * sw2 == vals["C_identity"]


@pytest.mark.parametrize("case", json.load(open(os.path.join(HERE, "index_sets.json"))),
                         ids=lambda c: f"{c['op']}-{c['snk_spin']}-{c['src_spin']}-{c['sign_mode']}")
def test_index_set_regression(case):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    iset = O.build_index_set([dict(op=case["op"], snk_spin=case["snk_spin"],
                                   src_spin=case["src_spin"], sign_mode=case["sign_mode"])])
    assert iset.nnz == case["nnz"]
    assert (iset.nu, iset.nd) == (case["n_u"], case["n_d"])
    assert mg.digest(iset) == case["sha256"]

"""Write the index-set regression fixtures from the FP64 oracle.

Run from the repository root:  python tests/golden/make_golden.py
Calls only ``oracle/``; nothing here comes from the GPU path.  For every
operator used by the correlator workloads it records the raw-term count, the
canonical key counts, sum |w|^2, the value C(S = 1) = sigma s^2 sum |w|^2, and
a SHA-256 of the canonical index set (int32 keys, int64 weight numerators) in
its canonical order, so that a change of any bit of the index set shows up.
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import operators as O  # noqa: E402

CASES = [("proton", 0, 0, "exact"), ("proton", 1, 3, "exact"), ("neutron", 2, 2, "exact"),
         ("DI", 0, 0, "exact"), ("DII", 0, 0, "exact"), ("DII", 0, 0, "r2")]
CASES += [("HE3_I", j, j, "exact") for j in range(4)]
CASES += [("HE3_II", j, j, "exact") for j in range(4)]
CASES += [("HE3_II", j, j, "r2") for j in range(4)]


def digest(iset):
    h = hashlib.sha256()
    for a in (iset.snk_u, iset.src_u, iset.snk_d, iset.src_d):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(iset.corr_id, dtype=np.int32).tobytes())
    for a in (iset.w_re, iset.w_im, iset.w_den):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    return h.hexdigest()


def main():
    out = []
    for op, s, sp, mode in CASES:
        iset = O.build_index_set([dict(op=op, snk_spin=s, src_spin=sp, sign_mode=mode)])
        terms, s2 = O.operator_terms(op, s, mode)
        w = O.sink_tensor(op, s, mode)
        nu, nd = O.quark_counts(op)
        sw2 = sum(c[0] ** 2 + c[1] ** 2 for c in w.values())
        cI = O.grassmann_sigma(nu, nd) * sw2 * s2 if s == sp else None
        out.append(dict(op=op, snk_spin=s, src_spin=sp, sign_mode=mode, n_u=nu, n_d=nd,
                        raw_terms=len(terms), canonical_keys=len(w),
                        distinct_snk_u=len({k[0] for k in w}), distinct_snk_d=len({k[1] for k in w}),
                        sum_abs_w2=sw2, w_den=int(s2.denominator), nnz=iset.nnz,
                        C_identity=(str(cI) if cI is not None else None),
                        sha256=digest(iset)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "index_sets.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path, len(out), "cases")


if __name__ == "__main__":
    main()

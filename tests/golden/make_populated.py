"""Write the fixtures of the populated-lattice GPU parity tests from the FP64 oracle.

Run from the repository root:  python tests/golden/make_populated.py
Calls only ``oracle/`` (and the seeded input generators of ``synth``, which
hold none of the method's arithmetic); nothing here comes from the GPU path.
Work is spread over the host's cores with a process pool.

Cases (the GPU launches run at these full lattice sizes, every site listed
as populated carrying its seeded propagators):
  di8        D_I on 8^3 x 16, SU(3) x spin propagators (seed 1), all 8192
             sites populated: C[t] and A[t] (sum of |Wick terms|) per timeslice.
  di_block   16^3 x 32, i.i.d. (seed 3), a fully populated 4^3 x 4 block
             (x, y, z < 4, t < 4; 256 sites), every other site zero:
             forward C, A for D_II (exact and R2) and D_I, and for the
             mixed weights W = W_DI + 0.5 W_DII(R2) on D_I's index set; the
             mixed-weight gradients for grad_C drawn with seed 33: grad_W and
             its scale at 64 sampled entries, grad_S_u/grad_S_d and scales at
             8 sampled block sites.
  he3_block  32^3 x 8, i.i.d. (seed 4), the 8 3He correlators, a populated
             4^3 block at t = 0 (64 sites), every other site zero: C[0], A[0].
  he3_grad   the same 32^3 x 8 lattice, every site populated, grad_C drawn
             with seed 44: grad_S_u/grad_S_d and scales at 3 sampled sites;
             grad_W and its scale at 16 sampled entries (2 per correlator),
             summed over all 262144 sites.
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import correlator as CO  # noqa: E402
from oracle import operators as O  # noqa: E402
from paper_2201_04269_amd import synth  # noqa: E402

HE3 = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
      [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]
DI_BLOCK_OPS = [dict(op="DII"), dict(op="DII", sign_mode="r2"), dict(op="DI")]

_CACHE = {}


def iset_for(key):
    if key not in _CACHE:
        if key == "he3":
            _CACHE[key] = O.build_index_set(HE3)
        elif key == "di_block":
            _CACHE[key] = O.build_index_set(DI_BLOCK_OPS)
        elif key == "di":
            _CACHE[key] = O.build_index_set([dict(op="DI")])
        elif key == "di_mixed":
            rs = O.build_index_set([dict(op="DI")])
            both = O.build_index_set([dict(op="DI"), dict(op="DII", sign_mode="r2")])
            w = both.weights()
            n = rs.nnz
            W = w[:n] + 0.5 * w[n:]
            rs.weights = lambda: W
            _CACHE[key] = rs
    return _CACHE[key]


def block_sites(L, n):
    """Sites v = x + L (y + L z) with x, y, z < n."""
    return [x + L * (y + L * z) for z in range(n) for y in range(n) for x in range(n)]


def job_forward(args):
    """C[c] and A[c] summed over the given sites of one timeslice."""
    key, Su, Sd = args
    rs = iset_for(key)
    su, sd = Su[None], Sd[None]
    return CO.correlator(su, sd, rs)[:, 0], CO.sum_abs_terms(su, sd, rs)[:, 0]


def job_site_grad(args):
    key, Su1, Sd1, g = args
    rs = iset_for(key)
    su, sd = Su1[None, None], Sd1[None, None]
    ref = CO.gradients(su, sd, rs, g, want=("S_u", "S_d"))
    scl = CO.gradient_abs_scales(su, sd, rs, g)
    return ref["S_u"][0, 0], ref["S_d"][0, 0], scl["S_u"][0, 0], scl["S_d"][0, 0]


def job_site_grad_w(args):
    """grad_W and its scale of one site for the whole index set (small sets)."""
    key, Su1, Sd1, g = args
    rs = iset_for(key)
    su, sd = Su1[None, None], Sd1[None, None]
    ref = CO.gradients(su, sd, rs, g)
    scl = CO.gradient_abs_scales(su, sd, rs, g)
    return ref, scl


def sub_index_set(rs, entries):
    """Every sampled entry as a correlator of its own (same exact weight)."""
    e = np.asarray(entries)
    return O.IndexSet(rs.nu, rs.nd, rs.snk_u[e], rs.src_u[e], rs.snk_d[e], rs.src_d[e], np.arange(len(e)),
                      rs.w_re[e], rs.w_im[e], rs.w_den[rs.corr_id[e]])


def job_entries(args):
    """Per sampled entry k (its own correlator): C_k[t] = W_k sum_{x in t} Du Dd and
    A_k[t] = |W_k| sum_{x in t} perm|Su sub| perm|Sd sub| over one timeslice."""
    key, entries, Su_t, Sd_t = args
    sub = sub_index_set(iset_for(key), entries)
    return CO.correlator(Su_t[None], Sd_t[None], sub)[:, 0], CO.sum_abs_terms(Su_t[None], Sd_t[None], sub)[:, 0]


def cx(a):
    a = np.asarray(a)
    return np.stack([a.real, a.imag], axis=-1).tolist()


def main():
    nproc = min(os.cpu_count() or 1, 16)
    pool = mp.get_context("fork").Pool(nproc)
    out = {}

    # di8: D_I on 8^3 x 16, SU(3) x spin (seed 1), every site
    T, V = 16, 8 ** 3
    Su, Sd = synth.su3_spin(T, V, seed=1)
    jobs = [("di", Su[t, a:a + 64], Sd[t, a:a + 64]) for t in range(T) for a in range(0, V, 64)]
    res = pool.map(job_forward, jobs, chunksize=1)
    C = np.zeros(T, complex)
    A = np.zeros(T)
    for (_, su, _), (c, a), (t, _) in zip(jobs, res, [(t, a) for t in range(T) for a in range(0, V, 64)]):
        C[t] += c[0]
        A[t] += a[0]
    out["di8"] = dict(T=T, V=V, seed=1, C=cx(C), A=A.tolist())
    print("di8 done", flush=True)

    # di_block: 16^3 x 32 i.i.d. (seed 3), the 4^3 x 4 block populated
    L, T = 16, 32
    V = L ** 3
    Su, Sd = synth.iid(T, V, seed=3)
    sites = block_sites(L, 4)
    blk = {}
    for key in ("di_block", "di_mixed"):
        res = pool.map(job_forward, [(key, Su[t, sites], Sd[t, sites]) for t in range(4)], chunksize=1)
        blk[key] = dict(C=cx([r[0] for r in res]), A=[r[1].tolist() for r in res])
    rng = np.random.default_rng(33)
    gC = rng.standard_normal((1, T)) + 1j * rng.standard_normal((1, T))
    rs = iset_for("di_mixed")
    ent = sorted(rng.choice(rs.nnz, size=64, replace=False).tolist())
    site_picks = sorted({(int(t), int(sites[i])) for t, i in zip(rng.integers(0, 4, 8), rng.integers(0, 64, 8))})
    # grad_W over the 256 block sites: per site, the oracle's full gradient, summed
    res = pool.map(job_site_grad_w, [("di_mixed", Su[t, v], Sd[t, v], gC[:, t:t + 1]) for t in range(4) for v in sites],
                   chunksize=4)
    gW = sum(r[0]["W"] for r in res)
    sW = sum(r[1]["W"] for r in res)
    by_site = {(t, v): r for (t, v), r in zip([(t, v) for t in range(4) for v in sites], res)}
    blk["grad"] = dict(gC=cx(gC), entries=ent, gW=cx(gW[ent]), sW=sW[ent].tolist(), grad_W_dot=None,
                       sites=[list(p) for p in site_picks],
                       gSu=[cx(by_site[p][0]["S_u"][0, 0]) for p in site_picks],
                       gSd=[cx(by_site[p][0]["S_d"][0, 0]) for p in site_picks],
                       sSu=[by_site[p][1]["S_u"][0, 0].tolist() for p in site_picks],
                       sSd=[by_site[p][1]["S_d"][0, 0].tolist() for p in site_picks])
    # sum_k W_k conj(grad_W_k) over every entry, and its scale (checks all entries at once)
    W = rs.weights()
    blk["grad"]["grad_W_dot"] = cx(np.sum(W * np.conj(gW)))
    blk["grad"]["grad_W_dot_scale"] = float(np.sum(np.abs(W) * sW))
    out["di_block"] = dict(L=L, T=T, seed=3, block=4, **blk)
    print("di_block done", flush=True)

    # he3_block: 32^3 x 8 i.i.d. (seed 4), 4^3 block at t = 0
    L, T = 32, 8
    V = L ** 3
    Su, Sd = synth.iid(T, V, seed=4)
    sites = block_sites(L, 4)
    res = pool.map(job_forward, [("he3", Su[0, sites[i:i + 4]], Sd[0, sites[i:i + 4]]) for i in range(0, 64, 4)],
                   chunksize=1)
    out["he3_block"] = dict(L=L, T=T, seed=4, block=4, C=cx(sum(r[0] for r in res)),
                            A=sum(r[1] for r in res).tolist())
    print("he3_block done", flush=True)

    # he3_grad: every site populated
    rng = np.random.default_rng(44)
    gC = rng.standard_normal((8, T)) + 1j * rng.standard_normal((8, T))
    picks = [(0, 0), (3, 17000), (T - 1, V - 1)]
    res = pool.map(job_site_grad, [("he3", Su[t, v], Sd[t, v], gC[:, t:t + 1]) for t, v in picks], chunksize=1)
    rs = iset_for("he3")
    ent = []
    for c in range(rs.n_corr):
        idx = np.nonzero(rs.corr_id == c)[0]
        ent += sorted(rng.choice(idx, size=2, replace=False).tolist())
    eres = pool.map(job_entries, [("he3", ent, Su[t], Sd[t]) for t in range(T)], chunksize=1)
    Ck = np.stack([r[0] for r in eres], axis=1)     # [n_entries, T]
    Ak = np.stack([r[1] for r in eres], axis=1)
    W = rs.weights()[ent]
    g = gC[rs.corr_id[ent]]                          # [n_entries, T]
    gW = np.sum(g * np.conj(Ck / W[:, None]), axis=1)
    sW = np.sum(np.abs(g) * Ak / np.abs(W)[:, None], axis=1)
    out["he3_grad"] = dict(L=L, T=T, seed=4, gC=cx(gC), sites=[list(p) for p in picks],
                           gSu=[cx(r[0]) for r in res], gSd=[cx(r[1]) for r in res],
                           sSu=[r[2].tolist() for r in res], sSd=[r[3].tolist() for r in res],
                           entries=ent, gW=cx(gW), sW=sW.tolist())
    print("he3_grad done", flush=True)
    pool.close()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "populated.json")
    with open(path, "w") as f:
        json.dump(out, f)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()

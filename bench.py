"""Throughput of the multi-baryon correlator contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one pass of the hot path over one batch of synthetic propagators
resident in HBM: the forward contraction C[t] (eq. 1, per-timeslice sums)
and, when the library provides it, the backward pass (dC/dW, dC/dS).  The
index set and plan are built once, outside the timed region (the paper
amortises its tree construction over configurations the same way).

Workloads (synthetic inputs, the paper's propagators are not available):
  di_mixed   D_I and D_II (R2) mixed as W(c) = c1 W_DI + c2 W_DII, c = (1, 0.5),
             on the union index set (270400 entries), 16^3 x 32 sites,
             i.i.d. complex Gaussian propagators (seed 3) [default]
  di_8       D_I, 8^3 x 16 sites, SU(3) x spin propagators (seed 1)
  he3        3He_I^j and 3He_II^j (R2), j = 0..3, 8 correlators in one launch,
             32^3 x 64 sites, i.i.d. (seed 4)  [large: ~10 GB of propagators]

Prints one JSON line (rank 0).  `value` is index entries contracted per
second, sum over correlators of |I_c| times the number of sites, divided by
the time of one step, for the FP32-compensated path; the FP64 path is timed
beside it and reported under "fp64".
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "index-entry contractions/s (fwd, fwd+bwd) FP32-comp vs FP64, % vector peak"
PEAK = {"f32c": 157.3e12, "f64": 78.6e12}  # MI355X vector peaks (FP32 packed; FP64)


def workload(name):
    from paper_2201_04269_amd import synth
    if name == "di_mixed":
        L, T = 16, 32
        ops = [dict(op="DI"), dict(op="DII", sign_mode="r2")]
        gen = lambda: synth.iid(T, L ** 3, seed=3)  # noqa: E731
        desc = "D_I + D_II(R2) mixed W(c)=c1 W_DI + c2 W_DII, c=(1,0.5), 16^3x32, iid seed 3"
    elif name == "di_8":
        L, T = 8, 16
        ops = [dict(op="DI")]
        gen = lambda: synth.su3_spin(T, L ** 3, seed=1)  # noqa: E731
        desc = "D_I, 8^3x16, SU(3)xspin seed 1"
    elif name == "he3":
        L, T = 32, 64
        ops = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
              [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]
        gen = lambda: synth.iid(T, L ** 3, seed=4)  # noqa: E731
        desc = "3He_I^j + 3He_II^j (R2), j=0..3, 32^3x64, iid seed 4"
    else:
        raise SystemExit(f"unknown workload {name}")
    return dict(name=name, L=L, T=T, ops=ops, gen=gen, desc=desc)


_W_ISET = None


def _oracle_init(ops):
    global _W_ISET
    from oracle import operators as O
    _W_ISET = O.build_index_set(ops)


def _oracle_sites(args):
    """Oracle forward on a slice of sites (run in a worker process)."""
    Su, Sd = args
    from oracle import correlator as CO
    CO.site_values(Su, Sd, _W_ISET)
    return Su.shape[0]


def cpu_baseline(wl, Su, Sd, nnz, budget_s=15.0):
    """Time the FP64 oracle (as it stands) on a bounded sample of sites.

    The sample is the first n sites of the workload, n sized so that the run
    takes about budget_s seconds; the oracle's forward (determinants of every
    needed submatrix, then the sum over the index set) runs with one process
    per host core over sites.
    """
    ops = wl["ops"][:1] if wl["name"] == "di_mixed" else wl["ops"]
    nproc = min(os.cpu_count() or 1, 16)
    flat_u = Su.reshape(-1, 12, 12)
    flat_d = Sd.reshape(-1, 12, 12)
    _oracle_init(ops)
    _oracle_sites((flat_u[:1], flat_d[:1]))  # warm caches
    t0 = time.perf_counter()
    _oracle_sites((flat_u[1:2], flat_d[1:2]))
    one = time.perf_counter() - t0
    n = int(budget_s / max(one, 1e-6)) * nproc
    n = max(nproc, min(n, flat_u.shape[0]))
    chunks = [(flat_u[i:i + 1], flat_d[i:i + 1]) for i in range(n)]
    with mp.get_context("fork").Pool(nproc, initializer=_oracle_init, initargs=(ops,)) as pool:
        pool.map(_oracle_sites, chunks[:nproc], chunksize=1)  # build the worker caches
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_sites, chunks, chunksize=1))
        dt = time.perf_counter() - t0
    return {"value": nnz * done / dt, "unit": "index entries/s (fwd)", "cores": nproc, "kind": "oracle",
            "sample": f"oracle forward over the first {done} sites of this workload ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="di_mixed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="f32c,f64")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sites shard by timeslice; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_04269_amd import api

    wl = workload(args.workload)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    Su, Sd = wl["gen"]()
    T, V = Su.shape[:2]
    print(f"[bench] workload {wl['name']}: T={T} V={V} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    su = torch.from_numpy(Su).to(dev)
    sd = torch.from_numpy(Sd).to(dev)

    iset_ops = wl["ops"][:1] if wl["name"] == "di_mixed" else wl["ops"]
    iset = api.IndexSet(iset_ops)
    nnz = iset.nnz
    W = None
    if wl["name"] == "di_mixed":
        both = api.IndexSet(wl["ops"])
        e = both.export()
        w = both.weights()
        n1 = nnz
        assert np.array_equal(e["snk_u"][:n1], e["snk_u"][n1:]) and np.array_equal(e["src_d"][:n1], e["src_d"][n1:])
        W = torch.from_numpy(1.0 * w[:n1] + 0.5 * w[n1:]).to(dev)
    n_sites = T * V
    entries = float(nnz) * n_sites
    stream = torch.cuda.current_stream()

    results = {}
    for prec in args.precisions.split(","):
        t0 = time.perf_counter()
        plan = api.Plan(iset, prec)
        st = plan.stats
        print(f"[bench] plan {prec}: tiles={st['n_tiles']} lds={st['lds_bytes']} "
              f"alg={st['alg_flops_per_site']:.3e} exec={st['exec_flops_per_site']:.3e} "
              f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)

        def step():
            return api.contract(plan, su, sd, W)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        ms = ev0.elapsed_time(ev1) / args.steps
        alg = st["alg_flops_per_site"] * n_sites
        results[prec] = dict(ms_per_step=ms, wall_ms_per_step=1e3 * wall / args.steps,
                             value=entries / (ms * 1e-3), alg_tflops=alg / (ms * 1e-3) / 1e12,
                             exec_tflops=st["exec_flops_per_site"] * n_sites / (ms * 1e-3) / 1e12,
                             frac=alg / (ms * 1e-3) / PEAK[prec], tiles=st["n_tiles"],
                             lds_bytes=st["lds_bytes"])
        print(f"[bench] {prec}: {ms:.3f} ms/step  {entries / (ms * 1e-3):.3e} entries/s  "
              f"alg {alg / (ms * 1e-3) / 1e12:.2f} TFLOP/s", file=sys.stderr, flush=True)
        del plan

    head = "f32c" if "f32c" in results else list(results)[0]
    r = results[head]
    st_alg = None
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "index entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": wl["desc"], "pass": "fwd", "sites": n_sites, "nnz": nnz,
                   "index_entries_per_step": entries},
        "roofline": {"bound": "alu", "achieved": r["alg_tflops"], "peak": PEAK[head] / 1e12,
                     "unit": "TFLOP/s", "frac": r["frac"], "traffic": None},
    }
    for prec, rr in results.items():
        if prec != head:
            out[prec] = {"value": rr["value"], "ms_per_step": rr["ms_per_step"],
                         "roofline": {"bound": "alu", "achieved": rr["alg_tflops"], "peak": PEAK[prec] / 1e12,
                                      "unit": "TFLOP/s", "frac": rr["frac"]}}
    out["exec_tflops"] = {p: rr["exec_tflops"] for p, rr in results.items()}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, Su, Sd, nnz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

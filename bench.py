"""Throughput of the multi-baryon correlator contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one pass of the whole hot path over one batch of synthetic
propagators resident in HBM: the forward contraction C[t] (eq. 1,
per-timeslice sums) and the backward pass (dC/dW, then dC/dS).  The index
set and plan are built once, outside the timed region (the paper amortises
its tree construction over configurations the same way).

Workloads (synthetic inputs, the paper's propagators are not available):
  he3        3He_I^j and 3He_II^j (R2), j = 0..3, 8 correlators in one launch,
             32^3 x 64 sites, i.i.d. (seed 4), all 64 timeslices resident in
             HBM (9.7 GB).  A step is one timeslice (32^3 sites, the sites of
             one C[t]); step i takes timeslice i mod 64.  Beside the steps,
             the forward over the whole 32^3 x 64 lattice in one launch is
             timed once per precision.  [default]
  he3_shard  the same operators on one GPU's share of that lattice when it is
             split by timeslice over 8 GPUs: 32^3 x 8 sites (i.i.d., seed 4)
  di_mixed   D_I and D_II (R2) mixed as W(c) = c1 W_DI + c2 W_DII, c = (1, 0.5),
             on the union index set (270400 entries), 16^3 x 32 sites,
             i.i.d. complex Gaussian propagators (seed 3); a step is the whole
             lattice
  di_8       D_I, 8^3 x 16 sites, SU(3) x spin propagators (seed 1)

Beside each workload the hadron-block path (Sec. 2 blocks with sink
momentum projection, Sec. 3 block-level correlators; FP64) is timed on the
same propagators and reported under "blocks" (--no-blocks skips it); for
di_mixed also with displaced sources (a second propagator set), under
"blocks"/"displaced".

Prints one JSON line (rank 0).  `value` is index entries contracted per
second, sum over correlators of |I_c| times the number of sites of a step,
divided by the time of one step, for the FP32-compensated path; the FP64 path
is timed beside it and reported under "f64" (forward only for he3).
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
        desc = ("3He_I^j + 3He_II^j (R2), j=0..3, 8 correlators, 32^3x64 resident (iid seed 4); "
                "step = one timeslice (32^3 sites)")
        return dict(name=name, L=L, T=T, ops=ops, gen=gen, desc=desc, step_T=1, fwd_full=True, bwd_precs=("f32c",))
    elif name == "he3_shard":
        L, T = 32, 8
        ops = [dict(op="HE3_I", snk_spin=j, src_spin=j) for j in range(4)] + \
              [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2") for j in range(4)]
        gen = lambda: synth.iid(T, L ** 3, seed=4)  # noqa: E731
        desc = "3He_I^j + 3He_II^j (R2), j=0..3, 32^3x8 (one timeslice shard of 32^3x64), iid seed 4"
    else:
        raise SystemExit(f"unknown workload {name}")
    return dict(name=name, L=L, T=T, ops=ops, gen=gen, desc=desc, step_T=T, fwd_full=False,
                bwd_precs=("f32c", "f64"))


def block_corrs(name):
    """Block-level correlators timed beside a workload (same propagators).

    di_mixed: D_I and D_II (R2) with the two nucleons at relative momentum 0
    and back to back at +-(1, 0, 0); he3_shard: 3He_I^j and 3He_II^j (R2),
    j = 0..3, all three baryons at zero momentum.
    """
    if name == "di_mixed":
        out = []
        for op, mode in (("DI", "exact"), ("DII", "r2")):
            out.append(dict(op=op, sign_mode=mode, moms=[(0, 0, 0), (0, 0, 0)]))
            out.append(dict(op=op, sign_mode=mode, moms=[(1, 0, 0), (-1, 0, 0)]))
        return out
    if name in ("he3_shard", "he3"):
        return [dict(op="HE3_I", snk_spin=j, src_spin=j, moms=[(0, 0, 0)] * 3) for j in range(4)] + \
               [dict(op="HE3_II", snk_spin=j, src_spin=j, sign_mode="r2", moms=[(0, 0, 0)] * 3) for j in range(4)]
    return None


def displaced_corrs(name):
    """Block-level correlators with displaced sources timed beside a workload:
    di_mixed: D_I and exact-sign D_II with the source nucleons at two points
    (the second point's propagators drawn with seed 5) and the sink nucleons
    back to back at +-(1, 0, 0)."""
    if name == "di_mixed":
        return [dict(op=op, moms=[(1, 0, 0), (-1, 0, 0)], src_pts=(0, 1)) for op in ("DI", "DII")], 5
    return None, None


def bench_blocks(api, torch, name, su, sd, L, steps, warmup, corrs=None):
    """Hadron blocks (one launch pair) and their contraction, timed with HIP
    events on the launch stream; FP64.  su, sd: [T, V, 12, 12] or
    [n_points, T, V, 12, 12]."""
    corrs = block_corrs(name) if corrs is None else corrs
    if corrs is None:
        return None
    t0 = time.perf_counter()
    bset = api.BlockSet(corrs)
    plan = api.BlockPlan(bset)
    st = plan.stats
    T, V = su.shape[-4:-2]
    dims = (L, L, L)
    ws = torch.empty(plan.workspace_bytes(T, dims), dtype=torch.uint8, device=su.device)
    print(f"[bench] blocks: {bset.n_types} types, {bset.n_terms} terms ({time.perf_counter() - t0:.1f}s)",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        blk = api.blocks(plan, su, sd, dims, workspace=ws)
        api.block_contract(plan, blk, method="tree", workspace=ws)
        api.block_contract(plan, blk, method="terms", workspace=ws)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for e in ev:
        e[0].record(stream)
        blk = api.blocks(plan, su, sd, dims, workspace=ws)
        e[1].record(stream)
        api.block_contract(plan, blk, method="tree", workspace=ws)
        e[2].record(stream)
        api.block_contract(plan, blk, method="terms", workspace=ws)
        e[3].record(stream)
    torch.cuda.synchronize()
    ms_b = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    ms_tree = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    ms_terms = sum(e[2].elapsed_time(e[3]) for e in ev) / steps
    flops_b = st["block_flops_per_site"] * T * V
    print(f"[bench] blocks: {ms_b:.3f} ms ({flops_b / (ms_b * 1e-3) / 1e12:.2f} TF), contraction by factor trees "
          f"{ms_tree:.3f} ms, by terms {ms_terms:.3f} ms", file=sys.stderr, flush=True)
    # the same trees through the generic evaluator (mbc_tree.h), blocks as the factor table
    e = bset.export()
    table = blk.reshape(T, -1)
    trees = []
    for c in range(bset.n_corr):
        m = e["corr_id"] == c
        if m.any():
            fac, ch = bset.factor_tree(c)
            trees.append(api.FactorTree(fac, ch, (e["num_re"][m] + 1j * e["num_im"][m]) / e["den"][c],
                                        table.shape[1]))
    for _ in range(warmup):
        for tr in trees:
            tr.evaluate(table)
    torch.cuda.synchronize()
    evg = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a0, a1 in evg:
        a0.record(stream)
        for tr in trees:
            tr.evaluate(table)
        a1.record(stream)
    torch.cuda.synchronize()
    ms_generic = sum(a0.elapsed_time(a1) for a0, a1 in evg) / steps
    print(f"[bench] blocks: factor trees by the generic evaluator {ms_generic:.3f} ms", file=sys.stderr, flush=True)
    egraph = bench_egraph(api, torch, bset, blk, steps, warmup, node_limit=EGRAPH_NODE_LIMIT.get(name, 200))
    return {"correlators": len(corrs), "block_types": bset.n_types, "g_matrices": st["n_gmats"],
            "source_points": bset.n_points, "terms": bset.n_terms,
            "tree_vertices": st["tree_vertices"], "dtype": "f64",
            "ms_blocks": ms_b, "ms_contract_tree": ms_tree, "ms_contract_terms": ms_terms,
            "ms_contract_tree_generic": ms_generic,
            "flops_contract_tree": st["tree_flops_per_t"] * T, "flops_contract_terms": st["contract_flops_per_t"] * T,
            "sites_per_s": T * V / ((ms_b + ms_tree) * 1e-3),
            "roofline": {"bound": "alu", "kernel": "block_g", "achieved": flops_b / (ms_b * 1e-3) / 1e12,
                         "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                         "frac": flops_b / (ms_b * 1e-3) / PEAK["f64"]},
            "egraph": egraph}


# e-graph node limits: the dinucleon graphs saturate (about 74 000 e-nodes for
# the four di_mixed correlators); 3He's do not, and its admitted re-writes cost
# canonicalisation time without lowering the plan's flops
EGRAPH_NODE_LIMIT = {"di_mixed": 100000, "he3_shard": 200, "he3": 200}
EGRAPH_MAX_WS = 48 << 30


def bench_egraph(api, torch, bset, blk, steps, warmup, node_limit=1000):
    """The same correlators as tensor expressions over the blocks (Sec. 5):
    e-graph per correlator, plan extracted with the paper's reuse objective and
    with the smallest tree cost, evaluated on the GPU; HIP events around all
    correlators' plans.  A plan whose workspace exceeds 8 GiB (or that the
    executor cannot take) is reported, not run."""
    T = blk.shape[0]
    out = {"node_limit": node_limit}
    for objective in ("reuse", "flops", "shared"):
        t0 = time.perf_counter()
        try:
            graphs = [api.TensorEGraph.for_blocks(bset, c, node_limit, objective) for c in range(bset.n_corr)]
        except Exception as e:  # a plan step beyond the executor's label limits
            out[objective] = {"error": str(e)}
            print(f"[bench] e-graph ({objective}): {e}", file=sys.stderr, flush=True)
            continue
        t_build = time.perf_counter() - t0
        ws_bytes = sum(g.workspace_bytes(T) for g in graphs)
        if ws_bytes > EGRAPH_MAX_WS:
            out[objective] = {"not_run": f"workspace {ws_bytes / 2**30:.1f} GiB",
                              "flops_plan": sum(g.stats["flops_plan"] for g in graphs) * T,
                              "steps": sum(g.stats["n_steps"] for g in graphs), "build_s": t_build}
            print(f"[bench] e-graph ({objective}): plan {out[objective]['flops_plan']:.3e} flops, workspace "
                  f"{ws_bytes / 2**30:.1f} GiB: not run", file=sys.stderr, flush=True)
            continue
        wss = [torch.empty(max(g.workspace_bytes(T), 16), dtype=torch.uint8, device=blk.device) for g in graphs]
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            for g, ws in zip(graphs, wss):
                g.execute_blocks(blk, workspace=ws)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            for g, ws in zip(graphs, wss):
                g.execute_blocks(blk, workspace=ws)
            b.record(stream)
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        fl = sum(g.stats["flops_plan"] for g in graphs) * T
        out[objective] = {"ms": ms, "build_s": t_build, "steps": sum(g.stats["n_steps"] for g in graphs),
                          "classes": sum(g.stats["n_classes"] for g in graphs),
                          "nodes": sum(g.stats["n_nodes"] for g in graphs),
                          "saturated": all(g.stats["saturated"] for g in graphs),
                          "terms": sum(g.stats["n_terms"] for g in graphs),
                          "roots": sum(g.stats["n_roots"] for g in graphs),
                          "flops_plan": fl, "flops_direct": sum(g.stats["flops_direct"] for g in graphs) * T,
                          "gflops": fl / (ms * 1e-3) / 1e9}
        print(f"[bench] e-graph ({objective}): {out[objective]['steps']} steps, plan {fl:.3e} flops "
              f"(direct {out[objective]['flops_direct']:.3e}), {ms:.3f} ms, built in {t_build:.2f} s",
              file=sys.stderr, flush=True)
    return out


_W_ISET = None


def _oracle_init(ops):
    global _W_ISET
    from oracle import operators as O
    _W_ISET = O.build_index_set(ops)


def _oracle_sites(args):
    """Oracle forward and gradients on a slice of sites (in a worker process)."""
    Su, Sd = args
    import numpy as np
    from oracle import correlator as CO
    S4u, S4d = Su[None], Sd[None]
    CO.correlator(S4u, S4d, _W_ISET)
    gC = np.ones((_W_ISET.n_corr, 1), dtype=np.complex128)
    CO.gradients(S4u, S4d, _W_ISET, gC)
    return Su.shape[0]


def host_cores():
    """Cores this process may run on (the box's share of the host) and the
    CPU model name from lscpu."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except Exception:  # pragma: no cover
        pass
    return n, model


def cpu_baseline(wl, Su, Sd, nnz, budget_s=15.0):
    """Time the FP64 oracle (as it stands) on a bounded sample of sites.

    The sample is the first n sites of the workload, n sized so that the run
    takes about budget_s seconds; per site the oracle's forward (determinants
    of every needed submatrix, then the sum over the index set) and its
    gradients (dW, dS_u, dS_d by cofactors) run, one process per core of the
    host share this process may use (at most 16, the share of one GPU).
    """
    ops = wl["ops"][:1] if wl["name"] == "di_mixed" else wl["ops"]
    avail, model = host_cores()
    nproc = max(1, min(avail, 16))
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
    return {"value": nnz * done / dt, "unit": "index entries/s (fwd+bwd)", "cores": nproc, "kind": "oracle",
            "host_cores_available": avail, "cpu_model": model,
            "sample": f"oracle forward + gradients over the first {done} sites of this workload ({dt:.1f} s)"}


KERNEL_PREFIX = {"fwd": "fwd_kernel", "dS": "ds_kernel", "dW": "dw_kernel"}


def profiled_traffic(workload, kernel, prec):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    profile of this workload, or None when there is none or the kernel sources
    changed since it was taken."""
    from paper_2201_04269_amd.build import source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    lines = open(path).read().splitlines()
    if f"source_hash {source_hash()}" not in lines:
        return None
    want = KERNEL_PREFIX[kernel] + ("<float" if prec == "f32c" else "<double")
    for ln in lines:
        parts = ln.split()  # traffic <kernel> <dispatches> <fetch B> <write B> <total B>
        if len(parts) == 6 and parts[0] == "traffic" and parts[1].startswith(want):
            return float(parts[-1])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="he3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="f32c,f64")
    ap.add_argument("--fwd-only", action="store_true")
    ap.add_argument("--no-blocks", action="store_true")
    ap.add_argument("--no-full", action="store_true", help="skip the whole-lattice forward launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
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
    step_T = wl["step_T"]
    n_batches = T // step_T
    sites_step = step_T * V
    entries = float(nnz) * sites_step
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(11)
    n_corr = len(iset_ops)
    gC = torch.from_numpy(rng.standard_normal((n_corr, step_T)) + 1j * rng.standard_normal((n_corr, step_T))).to(dev)

    def batch(i):
        t = (i % n_batches) * step_T
        return su[t:t + step_T], sd[t:t + step_T]

    def ev():
        return torch.cuda.Event(enable_timing=True)

    results = {}
    plans = {}
    for prec in args.precisions.split(","):
        do_bwd = (not args.fwd_only) and prec in wl["bwd_precs"]
        t0 = time.perf_counter()
        plan = api.Plan(iset, prec)
        plans[prec] = plan
        st = plan.stats
        # algorithmic flops per site of what runs: the exact weights (W None)
        # go through their factors where the plan says so
        fwd_fact = W is None and bool(st["fwd_factored"])
        ds_fact = W is None and bool(st["ds_factored"])
        fl_fwd = st["fact_alg_flops_per_site"] if fwd_fact else st["alg_flops_per_site"]
        fl_ds = st["fact_ds_alg_flops_per_site"] if ds_fact else st["ds_alg_flops_per_site"]
        print(f"[bench] plan {prec}: tiles={st['n_tiles']}/{st['b_n_tiles']}/{st['w_n_tiles']} "
              f"factored tiles={st['f_n_tiles'] if st['rank1'] else None} (fwd {fwd_fact}, dS {ds_fact}) "
              f"lds={st['f_lds_bytes_fwd'] if fwd_fact else st['lds_bytes']}/"
              f"{st['f_lds_bytes_ds'] if ds_fact else st['b_lds_bytes_ds']}/{st['b_lds_bytes_dw']} "
              f"alg fwd={fl_fwd:.3e} dS={fl_ds:.3e} dW={st['dw_alg_flops_per_site']:.3e} "
              f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)

        # one step: forward, then the backward as its two launches (dW, then
        # dS: the work of one contract_backward with both gradients), with
        # HIP events on the launch stream between them
        def step(i, marks=None):
            bu, bd = batch(i)
            if marks:
                marks[0].record(stream)
            api.contract(plan, bu, bd, W)
            if marks:
                marks[1].record(stream)
            if do_bwd:
                api.contract_backward(plan, bu, bd, W, gC, need_W=True, need_S=False)
                if marks:
                    marks[2].record(stream)
                api.contract_backward(plan, bu, bd, W, gC, need_W=False, need_S=True)
                if marks:
                    marks[3].record(stream)

        for i in range(args.warmup):
            step(i)
            torch.cuda.synchronize()
            print(f"[bench] {prec}: warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
        marks = [[ev() for _ in range(4)] for _ in range(args.steps)]
        first, last = ev(), ev()
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        first.record(stream)
        for i in range(args.steps):
            step(i, marks[i])
            if args.steps > 1 and sites_step * nnz > 1e11:  # long steps: report progress
                torch.cuda.synchronize()
                print(f"[bench] {prec}: step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
        last.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_wall) / args.steps
        ms = first.elapsed_time(last) / args.steps
        kern = {"fwd": (sum(m[0].elapsed_time(m[1]) for m in marks) / args.steps, fl_fwd)}
        if do_bwd:
            kern["dW"] = (sum(m[1].elapsed_time(m[2]) for m in marks) / args.steps, st["dw_alg_flops_per_site"])
            kern["dS"] = (sum(m[2].elapsed_time(m[3]) for m in marks) / args.steps, fl_ds)
        dom = max(kern, key=lambda k: kern[k][0])
        r = dict(ms_per_step=ms, wall_ms_per_step=1e3 * wall, value=entries / (ms * 1e-3), dominant=dom,
                 pass_="fwd+bwd" if do_bwd else "fwd",
                 kernels={k: {"ms": v[0], "alg_tflops": v[1] * sites_step / (v[0] * 1e-3) / 1e12,
                              "frac": v[1] * sites_step / (v[0] * 1e-3) / PEAK[prec]} for k, v in kern.items()},
                 fwd_value=entries / (kern["fwd"][0] * 1e-3),
                 exec_tflops_fwd=(None if fwd_fact else
                                  st["exec_flops_per_site"] * sites_step / (kern["fwd"][0] * 1e-3) / 1e12))
        results[prec] = r
        print(f"[bench] {prec}: step {ms:.3f} ms ({entries / (ms * 1e-3):.3e} entries/s) " +
              " ".join(f"{k} {v['ms']:.2f} ms {v['alg_tflops']:.2f} TF" for k, v in r["kernels"].items()),
              file=sys.stderr, flush=True)

    # the forward over the whole lattice in one launch (one timed launch per
    # precision; the kernel was already run on the steps' batches above)
    full = None
    if wl["fwd_full"] and not args.no_full:
        full = {"steps": 1, "sites": T * V, "T": T}
        for prec, plan in plans.items():
            a0, a1 = ev(), ev()
            torch.cuda.synchronize()
            print(f"[bench] {prec}: forward over the whole {T}x{V} lattice in one launch ...", file=sys.stderr,
                  flush=True)
            a0.record(stream)
            api.contract(plan, su, sd, W)
            a1.record(stream)
            torch.cuda.synchronize()
            fms = a0.elapsed_time(a1)
            pst = plan.stats
            fl = (pst["fact_alg_flops_per_site"] if (W is None and pst["fwd_factored"]) else pst["alg_flops_per_site"]) * T * V
            full[prec] = {"ms": fms, "value": float(nnz) * T * V / (fms * 1e-3), "alg_tflops": fl / (fms * 1e-3) / 1e12,
                          "frac": fl / (fms * 1e-3) / PEAK[prec]}
            print(f"[bench] {prec}: whole-lattice forward {fms / 1e3:.2f} s ({full[prec]['value']:.3e} entries/s, "
                  f"{full[prec]['alg_tflops']:.2f} TF)", file=sys.stderr, flush=True)
    plans.clear()

    head = "f32c" if "f32c" in results else list(results)[0]
    r = results[head]
    dk = r["kernels"][r["dominant"]]
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
        "config": {"workload": wl["desc"], "pass": r["pass_"], "sites_per_step": sites_step,
                   "lattice_sites": T * V, "correlators": n_corr, "nnz": nnz, "index_entries_per_step": entries},
        "roofline": {"bound": "alu", "kernel": r["dominant"], "achieved": dk["alg_tflops"],
                     "peak": PEAK[head] / 1e12, "unit": "TFLOP/s", "frac": dk["frac"],
                     "traffic": profiled_traffic(wl["name"], r["dominant"], head)},
        "hbm": None,
        "kernels": r["kernels"],
        "fwd_only_value": r["fwd_value"],
    }
    # HBM rate of the dominant kernel: its profiled bytes per launch over its
    # launch time measured here (null when the profile is stale)
    tr = out["roofline"]["traffic"]
    if tr is not None:
        out["hbm"] = {"kernel": r["dominant"], "bytes": tr, "GBps": tr / (dk["ms"] * 1e-3) / 1e9,
                      "peak_GBps": 8000.0}
    for prec, rr in results.items():
        if prec != head:
            out[prec] = {"pass": rr["pass_"], "value": rr["value"], "ms_per_step": rr["ms_per_step"],
                         "fwd_only_value": rr["fwd_value"], "kernels": rr["kernels"]}
    if full is not None:
        out["whole_lattice_forward"] = full
    if not args.no_blocks:
        blk = bench_blocks(api, torch, wl["name"], su, sd, wl["L"], args.steps, args.warmup)
        if blk is not None:
            out["blocks"] = blk
            dcorrs, seed2 = displaced_corrs(wl["name"])
            if dcorrs is not None:
                from paper_2201_04269_amd import synth
                Su2, Sd2 = synth.iid(T, V, seed=seed2)
                su2 = torch.stack([su, torch.from_numpy(Su2).to(dev)])
                sd2 = torch.stack([sd, torch.from_numpy(Sd2).to(dev)])
                del Su2, Sd2
                out["blocks"]["displaced"] = bench_blocks(api, torch, wl["name"], su2, sd2, wl["L"], args.steps,
                                                          args.warmup, corrs=dcorrs)
                del su2, sd2
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, Su, Sd, nnz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

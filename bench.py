#!/usr/bin/env python3
"""IRLS s-t min-cut benchmark on one MI355X.

A step is one whole pass of the hot path on one synthetic instance already
resident in HBM: every IRLS round (reweight + Jacobi-PCG) followed by the
sweep cut, i.e. irls_mincut_solve + irls_mincut_cut.  The default workload is
the 256^3 6-connected segmentation grid (16,777,216 non-terminal nodes,
50,135,040 interior edges), plain FP64, 40 rounds with eps halved from 0.1, CG
to a relative residual of 1e-8; beside it the same instance in the precision
form (FP32 SpMV, FP64 dots and residual replacement).

Prints one JSON line with the throughput (cuts/s), the roofline of the SpMV
kernel (algorithmic bytes / its mean in-solve launch time, from HIP events
around each launch during the timed steps, vs 8 TB/s) and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (generator kwargs, solver options, description)
    "seg128": (dict(kind="seg", N=128, seed=1), dict(rounds=40, cg_rtol=1e-8),
               "3-D 6-connected 128^3 segmentation grid, smooth-field capacities, FP64, "
               "40 rounds, eps 0.1 halved per round, Jacobi-PCG to 1e-8"),
    "grid64": (dict(kind="grid2d", nx=64, ny=64, seed=0), dict(rounds=30, cg_rtol=1e-10),
               "2-D 4-connected 64x64 grid, FP64, 30 rounds, eps 0.1 halved, Jacobi-PCG to 1e-10"),
    "seg256": (dict(kind="seg", N=256, seed=2), dict(rounds=40, cg_rtol=1e-8),
               "3-D 6-connected 256^3 segmentation grid, FP64 (plain), 40 rounds, CG to 1e-8"),
    "rmat512": (dict(kind="rmat", count=512, seed=1000), dict(rounds=30, cg_rtol=1e-8),
                "512 R-MAT FlowImprove-style instances (2^10..2^17 nodes drawn, average degree 8 before "
                "the isolated nodes are dropped, about 14.5 after), FP64, 30 rounds, CG to 1e-8, one "
                "persistent launch"),
    "seg256-mixed": (dict(kind="seg", N=256, seed=2),
                     dict(rounds=40, cg_rtol=1e-8, precision=1, refine_every=20),
                     "3-D 256^3 segmentation grid, FP32 conductances/SpMV/CG vectors, FP64 "
                     "potentials, dots and residual replacement every 20 CG steps"),
    "seg256-slab": (dict(kind="slab", N=256, planes=32, seed=2), dict(rounds=40, cg_rtol=1e-8),
                    "one GPU's share of the 256^3 segmentation grid split into 8 z-slabs: its first "
                    "32 planes (256x256x32) as a graph of their own, FP64, 40 rounds, CG to 1e-8"),
    "seg128-bj": (dict(kind="seg", N=128, seed=1), dict(rounds=40, cg_rtol=1e-8, precond=1),
                  "3-D 128^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi "
                  "preconditioner (x-lines of 128 rows, tridiagonal blocks)"),
    "seg128-ilu": (dict(kind="seg", N=128, seed=1), dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=4),
                   "3-D 128^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                   "(4x4x4 tiles, each block by ILU(0))"),
    "seg256-ilu": (dict(kind="seg", N=256, seed=2), dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=4),
                   "3-D 256^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                   "(4x4x4 tiles, each block by ILU(0))"),
    "seg128-ilu-mixed": (dict(kind="seg", N=128, seed=1),
                         dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=4, precision=1, refine_every=20),
                         "3-D 128^3 segmentation grid, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                         "(4x4x4 tiles, each block by ILU(0)) in the precision form: FP32 conductances, pivots, "
                         "SpMV and CG vectors, FP64 potentials, dots and residual replacement every 20 CG steps"),
    "seg256-ilu-mixed": (dict(kind="seg", N=256, seed=2),
                         dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=4, precision=1, refine_every=20),
                         "3-D 256^3 segmentation grid, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                         "(4x4x4 tiles, each block by ILU(0)) in the precision form: FP32 conductances, pivots, "
                         "SpMV and CG vectors, FP64 potentials, dots and residual replacement every 20 CG steps"),
    "seg128-ilu8": (dict(kind="seg", N=128, seed=1), dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=8),
                    "3-D 128^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                    "(8x8x8 tiles, each block by ILU(0))"),
    "seg256-ilu8": (dict(kind="seg", N=256, seed=2), dict(rounds=40, cg_rtol=1e-8, precond=2, block_size=8),
                    "3-D 256^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi preconditioner "
                    "(8x8x8 tiles, each block by ILU(0))"),
    "seg256-bj": (dict(kind="seg", N=256, seed=2), dict(rounds=40, cg_rtol=1e-8, precond=1),
                  "3-D 256^3 segmentation grid, FP64, 40 rounds, CG to 1e-8, block-Jacobi "
                  "preconditioner (x-lines of 128 rows, tridiagonal blocks solved exactly)"),
    "gnn192": (dict(kind="gnn", train64=96, train128=16, cost_graphs=48, eval_n=192, eval_seeds=8),
               dict(rounds=40, cg_rtol=1e-8),
               "learned warm start: network trained on 64^3 and 128^3 segmentation grids, "
               "evaluated on held-out 192^3 grids (seeds 20000..); time-to-cut at relative cut "
               "error <= 1e-6 vs the plain start (40 rounds, eps 0.1 halved, CG to 1e-8, FP64)"),
}


def make_graph(spec):
    import gen
    spec = dict(spec)
    kind = spec.pop("kind")
    if kind == "rmat":
        return gen.rmat_batch(spec["count"], first_seed=spec["seed"])
    if kind == "seg":
        return gen.grid3d_seg(spec["N"], seed=spec["seed"])
    if kind == "slab":
        return gen.grid3d_seg_slab(spec["N"], spec["planes"], seed=spec["seed"])
    return gen.grid2d(spec["nx"], spec["ny"], seed=spec["seed"])


def spmv_bytes(info, precision, variant):
    """Algorithmic bytes of one SpMV launch (each array element touched once)."""
    nt, nnz, K = info["n_nonterminal"], info["nnz_offdiag"], info["n_diagonals"]
    ts = 4 if precision == 1 else 8
    if variant == 4:
        # scaled system: reads K scaled conductances, z, p_old; writes p_new, q
        return nt * (ts * (K + 2) + 2 * ts)
    if info["format"] == 2:
        # reads D, K conductances, z, p_old; writes p_new, q
        return nt * (ts * (K + 3) + 2 * ts)
    # CSR: values + column indices + row pointers, D, p, q
    return nnz * (ts + 4) + (nt + 1) * 4 + nt * 3 * ts


def code_sha(path):
    """SHA-256 prefix of a source file's code: // comments, trailing blanks and
    blank lines removed, so that editing a comment keeps a profile valid."""
    import hashlib
    import re
    lines = []
    for line in open(path, encoding="utf-8"):
        line = re.sub(r"//.*", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def profiled_traffic(kernel, workload, source="cg.hip"):
    """HBM bytes per launch from the committed rocprofv3 summary, if the kernel
    code (the source file that holds it) is still the one that was profiled
    (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    sha = code_sha(os.path.join(ROOT, "paper_1501_03105_amd", "csrc", source))
    if fields.get("code_sha256_prefix") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def golden_run(workload):
    """The oracle's full FP64 Jacobi run of this workload's instance, if one is
    stored (written on the CPU by tests/golden/make_golden_fullsize.py, which
    calls only the oracle); the precision form and the block-Jacobi forms of
    an instance are compared with it too."""
    for suffix in ("-mixed", "-ilu8", "-ilu", "-bj"):
        if workload.endswith(suffix):
            workload = workload[: -len(suffix)]
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, opts, gpu_iters_total, budget_s):
    """Oracle time per CG iteration on the first rounds of the same instance,
    scaled to the GPU run's total CG iterations, plus the oracle sweep."""
    import oracle
    rounds = 1
    t_total, it_total = 0.0, 0
    while True:
        t0 = time.perf_counter()
        x, R, _ = oracle.irls(g, rounds=rounds, eps0=0.1, eps_factor=0.5,
                              cg_rtol=opts.get("cg_rtol", 1e-8), allow_maxit=True)
        dt = time.perf_counter() - t0
        t_total, it_total = dt, sum(r["cg_iters"] for r in R)
        if dt > budget_s / 3 or rounds >= opts.get("rounds", 40):
            break
        rounds = min(opts.get("rounds", 40), rounds * 2)
    t0 = time.perf_counter()
    oracle.sweep(g, x)
    t_sweep = time.perf_counter() - t0
    per_it = t_total / max(it_total, 1)
    est = per_it * gpu_iters_total + t_sweep
    return {
        "value": 1.0 / est, "unit": "cuts/s", "cores": oracle.max_threads(), "kind": "oracle",
        "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "sample": (f"oracle IRLS rounds 0..{rounds} of the same instance ({it_total} CG iterations "
                   f"in {t_total:.1f} s) + one oracle sweep ({t_sweep:.1f} s); time-to-cut "
                   f"estimated as per-iteration cost x the GPU run's {gpu_iters_total} CG iterations "
                   f"+ sweep = {est:.1f} s"),
    }


def bench_batch(args, spec, opts, desc):
    """Batched form: cuts/s over the whole batch (solve + sweep of every graph)."""
    import numpy as np
    import torch

    import paper_1501_03105_amd as P
    t0 = time.perf_counter()
    gs = make_graph(spec)
    print(f"[bench] {len(gs)} graphs, {sum(g.n for g in gs)} nodes, generated in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    mb = P.MinCutBatch(gs, stream=torch.cuda.current_stream(), **opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    # rows per wavefront: measured per row-length bin on short solves (setup,
    # not part of a step)
    t0 = time.perf_counter()
    lanes = mb.autotune(rounds=2, reps=2)
    t_tune = time.perf_counter() - t0
    print(f"[bench] autotuned lanes per row by bin {lanes} in {t_tune:.1f}s", file=sys.stderr, flush=True)

    def step():
        rc, st = mb.solve()
        _, vals = mb.cut()
        return st, vals

    for i in range(args.warmup):
        st, vals = step()
        print(f"[bench] warmup {i}: CG iterations {sum(r['cg_iters'] for s in st for r in s)}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, vals = step()
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = [sum(r["cg_iters"] for r in s) for s in st]
    # the same steps with the default table, for the autotuner's gain
    default_lanes = [min(2 << b, 64) for b in range(len(lanes))]
    mb.set_row_lanes(default_lanes)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, vals_def = step()
    torch.cuda.synchronize()
    dt_def = time.perf_counter() - t0
    mb.close()
    # The plain FP64 GPU path (one multi-workgroup solve per graph, one graph
    # after another) on every 16th graph in size order, each after one untimed
    # solve; its summed time x 16 estimates that path's time for the whole
    # batch.  Its cuts are compared with the batch's.
    order = sorted(range(len(gs)), key=lambda i: gs[i].n)
    sample = order[8::16]
    t_plain, t_tuned, worst = 0.0, 0.0, 0.0
    for i in sample:
        with P.MinCut.from_graph(gs[i], stream=torch.cuda.current_stream(), solver=1, **opts) as mc:
            mc.solve()                                       # warm-up, as for the batch
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mc.solve()
            _, v1, _ = mc.cut()
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            worst = max(worst, abs(v1 - vals[i]) / max(abs(vals[i]), 1e-300))
            # the same path with its rows per wavefront measured (setup, untimed;
            # a graph in the diagonal format has none to tune)
            try:
                mc.autotune(reps=1)
            except P.IrlsError:
                pass
            mc.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mc.solve()
            _, v2, _ = mc.cut()
            torch.cuda.synchronize()
            t_tuned += time.perf_counter() - t0
            worst = max(worst, abs(v2 - vals[i]) / max(abs(vals[i]), 1e-300))
    plain_rate = len(sample) / min(t_plain, t_tuned)
    print(f"[bench] plain FP64 path, {len(sample)} sampled graphs one by one: {t_plain:.2f} s "
          f"({plain_rate:.1f} cuts/s); largest cut difference from the batch {worst:.1e}",
          file=sys.stderr, flush=True)
    rate = len(gs) * args.steps / dt
    # roofline of the persistent launch: its algorithmic bytes (per CG
    # iteration of a graph 12 B per stored CSR entry and 104 B per row, the
    # count of the multi-workgroup CSR path's SpMV, direction and update
    # kernels) over the batch's time per step (the launch plus the batched
    # sweep, a few per cent of it)
    nnz = [2 * g.meta["interior"] for g in gs]
    rows = [g.n - 2 for g in gs]
    batch_bytes = sum(it * (12 * z + 104 * r) for it, z, r in zip(iters, nnz, rows))
    achieved = batch_bytes / (dt / args.steps) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic("k_resident", "rmat512", "resident.hip"), "kernel": "k_resident",
            "bytes_per_launch": int(batch_bytes), "avg_launch_ms": round(1000 * dt / args.steps, 3),
            "note": "one launch solves every round of every graph; the largest graphs, one workgroup each, "
                    "set its length, so it is bound by their memory latency, not by bandwidth"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample_b = order[::32]
        t0 = time.perf_counter()
        for i in sample_b:
            oracle.irls(gs[i], rounds=opts["rounds"], cg_rtol=opts["cg_rtol"], allow_maxit=True)
        t_orc = time.perf_counter() - t0
        cpu = {"value": len(sample_b) / t_orc, "unit": "cuts/s", "cores": oracle.max_threads(), "kind": "oracle",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "sample": f"oracle IRLS ({opts['rounds']} rounds, CG to {opts['cg_rtol']}) of every 32nd graph "
                         f"in size order ({len(sample_b)} graphs) in {t_orc:.1f} s, one after another"}
        print(f"[bench] oracle on {len(sample_b)} sampled graphs: {t_orc:.1f} s", file=sys.stderr, flush=True)
    out = {
        "metric": "IRLS s-t min-cut throughput of the batched form (cuts per second)",
        "value": round(rate, 3), "unit": "cuts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "graphs": len(gs),
                   "nodes": int(sum(g.n for g in gs)),
                   "interior_edges": int(sum(g.meta["interior"] for g in gs)),
                   "average_degree_after_isolated_nodes_dropped":
                       round(2 * sum(g.meta["interior"] for g in gs) / sum(g.n - 2 for g in gs), 2),
                   "arithmetic": "FP64 (conductances, SpMV, CG vectors and dots)",
                   "cg_iters_total": int(sum(iters)), "cg_iters_max_graph": int(max(iters)),
                   "setup_s": round(t_setup, 3),
                   "autotune": {"lanes_per_row_by_bin": lanes, "seconds": round(t_tune, 3),
                                "default_lanes": default_lanes,
                                "default_cuts_per_s": round(len(gs) * args.steps / dt_def, 3),
                                "max_rel_cut_difference_from_default": float(
                                    np.max(np.abs(vals - vals_def) / np.maximum(np.abs(vals_def), 1e-300)))},
                   "plain_fp64_one_by_one": {
                       "cuts_per_s": round(plain_rate, 3),
                       "cuts_per_s_default_rows_per_wave": round(len(sample) / t_plain, 3),
                       "cuts_per_s_autotuned_rows_per_wave": round(len(sample) / t_tuned, 3),
                       "speedup_of_batch": round(rate / plain_rate, 2),
                       "max_rel_cut_difference": worst,
                       "sample": f"every 16th graph in size order ({len(sample)} graphs), "
                                 "multi-workgroup FP64 solver, solve + sweep each; the rate is the "
                                 "faster of its default and autotuned rows per wavefront"}},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_gnn(args, spec, opts, desc):
    """Learned warm start: train, then time-to-cut on held-out 192^3 grids for
    the plain start, the best constant first eps (chosen on the training
    graphs, no network) and the network's start.  Every start runs its rounds
    down to the plain schedule's last eps and is then cut (nothing knows the
    answer); its cut is then compared with the plain start's."""
    import numpy as np
    import torch

    import gen
    import paper_1501_03105_amd as P
    from paper_1501_03105_amd import warmstart as W

    stream = torch.cuda.current_stream()

    def seg(N, seed):
        g = gen.grid3d_seg(N, seed=seed, with_intensity=True)
        return g, np.concatenate([g.meta["I"], [0.0, 0.0]])

    say = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ex = []
    for N, cnt, base in ((64, spec["train64"], 100), (128, spec["train128"], 300)):
        for i in range(cnt):
            g, I = seg(N, base + i)
            ex.append(W.make_example(g, I, opts, stream=stream))
            if (i + 1) % 8 == 0:
                say(f"{i + 1} of {cnt} training graphs of {N}^3 solved")
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, gamma, costs = W.fit(ex, args.gnn_epochs, args.gnn_epochs // 2, stream=stream, log=say,
                              max_cost_graphs=spec["cost_graphs"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # the no-network baseline: the best constant first eps on (the same
    # subset of) the training graphs
    t0 = time.perf_counter()
    sub = [ex[int(i)] for i in np.linspace(0, len(ex) - 1, min(len(ex), spec["cost_graphs"]))]
    eps_c, table = W.best_constant_eps(sub, stream=stream, log=say)
    t_const = time.perf_counter() - t0
    say(f"best constant first eps on the training graphs: {eps_c:.3g} ({ {f'{k:.0e}': v for k, v in table.items()} })")
    for e in ex:
        e.mc.close()
    del ex
    rows = []
    tol = 1e-6
    for k in range(spec["eval_seeds"]):
        sd = 20000 + k
        g, I = seg(spec["eval_n"], sd)
        mc = P.MinCut.from_graph(g, stream=stream, solver=1, **opts)
        W.time_to_final(mc, stream=stream)                  # warm-up
        plain = W.time_to_final(mc, stream=stream)          # the plain schedule: its cut is the reference
        ref = plain["cut"]
        const = W.time_to_final(mc, eps_first=eps_c, stream=stream)
        warm = W.time_to_final(mc, net=net, gamma=gamma, intensity=I, stream=stream)
        # hindsight: the best constant for this graph (context, not a baseline)
        best_h = min((W.time_to_final(mc, eps_first=e, stream=stream) for e in W.EPS_GRID),
                     key=lambda r: (r["cut"] > ref * (1 + tol), r["seconds"]))
        mc.close()
        mc32 = P.MinCut.from_graph(g, stream=stream, solver=1, precision=1, refine_every=20, **opts)
        W.time_to_final(mc32, net=net, gamma=gamma, intensity=I, stream=stream)     # warm-up
        both = W.time_to_final(mc32, net=net, gamma=gamma, intensity=I, stream=stream)
        mc32.close()
        for r in (const, warm, best_h, both):
            r["rel_cut_error"] = (r["cut"] - ref) / ref
        rows.append((sd, ref, plain, const, warm, best_h, both))
        say(f"eval {spec['eval_n']}^3 seed {sd}: plain {plain['cg_iters']} CG {plain['seconds']:.3f}s | "
            f"constant eps_1 {eps_c:.2g} {const['cg_iters']} CG {const['seconds']:.3f}s err {const['rel_cut_error']:.1e} | "
            f"warm eps_1 {warm['eps_first']:.2g} {warm['cg_iters']} CG {warm['seconds']:.3f}s "
            f"err {warm['rel_cut_error']:.1e} | warm+FP32 {both['seconds']:.3f}s err {both['rel_cut_error']:.1e}")
    tot = lambda j: sum(r[j]["seconds"] for r in rows)
    its = lambda j: sum(r[j]["cg_iters"] for r in rows)
    ok = lambda j: all(r[j]["rel_cut_error"] <= tol for r in rows)
    sp, sc, sw, sh, sb = tot(2), tot(3), tot(4), tot(5), tot(6)
    out = {
        "metric": "learned warm start: end-to-end time-to-cut speedup vs the plain start (rounds down to the "
                  "plain schedule's last eps, then the sweep cut; cut relative error vs the plain start's)",
        "value": round(sp / sw, 4), "unit": "x", "n_gpus": 1, "steps": len(rows), "warmup": 1,
        "ms_per_step": round(1000 * sw / len(rows), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 solve, bf16/f32 network", "data": "synthetic",
        "config": {"workload": desc, "name": args.workload,
                   "train_graphs": {"64^3": spec["train64"], "128^3": spec["train128"],
                                    "start_costs_and_eps_targets_on": len(sub)},
                   "epochs": [args.gnn_epochs, args.gnn_epochs // 2], "gamma": gamma,
                   "data_s": round(t_data, 1), "train_s": round(t_train, 1), "constant_choice_s": round(t_const, 1),
                   "speedup_vs_best_constant_eps": round(sc / sw, 4),
                   "best_constant_eps": eps_c,
                   "best_constant": {"speedup_vs_plain": round(sp / sc, 4), "cg_iters": its(3),
                                     "all_within_1e-6": ok(3)},
                   "warm": {"cg_iters": its(4), "all_within_1e-6": ok(4),
                            "max_rel_cut_error": max(r[4]["rel_cut_error"] for r in rows)},
                   "hindsight_best_constant_per_graph": {"speedup_vs_plain": round(sp / sh, 4),
                                                         "all_within_1e-6": ok(5)},
                   "warm_start_with_precision_form": {"speedup_vs_plain_fp64": round(sp / sb, 4),
                                                      "all_within_1e-6": ok(6), "cg_iters": its(6)},
                   "plain": {"cg_iters": its(2), "rounds": rows[0][2]["rounds"]},
                   "per_graph": [{"seed": r[0], "cut": r[1], "plain_s": round(r[2]["seconds"], 4),
                                  "const_s": round(r[3]["seconds"], 4), "warm_s": round(r[4]["seconds"], 4),
                                  "plain_cg": r[2]["cg_iters"], "const_cg": r[3]["cg_iters"],
                                  "warm_cg": r[4]["cg_iters"], "warm_eps_1": r[4]["eps_first"],
                                  "warm_err": r[4]["rel_cut_error"], "const_err": r[3]["rel_cut_error"]}
                                 for r in rows]},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="seg256", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel-events", type=int, default=16, metavar="EVERY",
                    help="N >= 1: HIP events around the SpMV launches of CG iterations 0, N, 2N, ... of "
                         "every round of the timed steps (the roofline's launch time); 0: none (the "
                         "roofline then falls back to back-to-back launches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--gnn-epochs", type=int, default=30)
    ap.add_argument("--early-stop-gap", type=float, default=0.01,
                    help="also time the certified-gap stopping rule (stop_gap) on the same instance; 0: skip")
    ap.add_argument("--precision-form", type=int, default=1,
                    help="1: also time the precision form on the same instance; 0: skip")
    ap.add_argument("--march-tile", default="", metavar="THREADS,LINES",
                    help="tile shape of the marching SpMV (irls_mincut_set_march_tile); default: the "
                         "library's")
    ap.add_argument("--kernel-breakdown", type=int, default=1,
                    help="1: one extra step per other CG kernel (update; residual replacement; "
                         "block-Jacobi apply) timed in the solve as the SpMV is; 0: skip")
    ap.add_argument("--stream-probe", type=int, default=1,
                    help="1: also measure the GPU's streaming ceiling for the SpMV's mix of five read and "
                         "two write streams of n_nonterminal doubles (irls_stream_probe); 0: skip")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run 5 plain device copies of MIB MiB (reference for byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library solves on one GPU; run with --gpus 1 (multi-GPU runs are "
              "not supported)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1501_03105_amd as P

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    spec, opts, desc = WORKLOADS[args.workload]
    if spec["kind"] == "rmat":
        return bench_batch(args, spec, opts, desc)
    if spec["kind"] == "gnn":
        return bench_gnn(args, spec, opts, desc)
    t0 = time.perf_counter()
    g = make_graph(spec)
    t_gen = time.perf_counter() - t0
    print(f"[bench] workload {args.workload}: n={g.n} m={g.m} generated in {t_gen:.1f}s",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mc = P.MinCut.from_graph(g, stream=stream, **opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = mc.info()
    if args.march_tile:
        mc.set_march_tile(*[int(v) for v in args.march_tile.split(",")])
    mc_tile = mc.march_tile() if info["solver"] == 1 else None
    print(f"[bench] create {t_setup:.1f}s info {info}", file=sys.stderr, flush=True)

    def step():
        rc, st = mc.solve()
        _, val, k = mc.cut()
        return st, val

    warm_ms = []
    for i in range(args.warmup):
        ts = time.perf_counter()
        st, val = step()
        warm_ms.append(1000.0 * (time.perf_counter() - ts))
        print(f"[bench] warmup {i}: cut {val:.10g}, CG iterations {sum(r['cg_iters'] for r in st)}, "
              f"{warm_ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    # the SpMV's in-solve launch times: an event pair around each of its
    # launches in the timed steps (the warm-up steps run without them)
    events = args.kernel_events > 0 and info["solver"] == 1
    if events:
        mc.set_kernel_timing(0, args.kernel_events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        st, val = step()                     # the cut's readback synchronises the stream
        step_ms.append(1000.0 * (time.perf_counter() - ts))
        print(f"[bench] step {i} done ({step_ms[-1]:.1f} ms)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ktime = mc.kernel_timing() if events else None
    if events:
        mc.set_kernel_timing(-1)
    # the other CG kernels' in-solve launch times, one extra step each (after
    # the timed steps, which stay as they are)
    breakdown = {}
    if events and args.kernel_breakdown:
        # with ILU(0) of 4x4x4 tiles (the default tile) the application runs
        # inside the update kernel
        fused = opts.get("precond", 0) == 2 and opts.get("block_size", 0) in (0, 4) and info["format"] == 2
        kinds = [(1, "update_with_ilu0_apply" if fused else "update")]
        if opts.get("precision", 0) == 1:
            kinds.append((2, "residual_replacement"))
        if opts.get("precond", 0) >= 1 and not fused:
            kinds.append((3, "block_jacobi_apply"))
        # an odd stride, so that both parities of the scaled form's update
        # (odd iterations also move the potentials) are sampled
        stride = args.kernel_events | 1
        for which, nm in kinds:
            mc.set_kernel_timing(which, stride)
            step()
            kt = mc.kernel_timing()
            mc.set_kernel_timing(-1)
            if kt["n_working"]:
                breakdown[nm] = {"mean_ms": round(kt["ms_working"] / kt["n_working"], 5),
                                 "sampled_launches": kt["n_working"]}
        print(f"[bench] in-solve kernel means: {breakdown}", file=sys.stderr, flush=True)
    iters = sum(r["cg_iters"] for r in st)
    ms_step = 1000.0 * dt / args.steps
    # the two-level rounding of the same potentials, timed on its own (it is
    # the paper's alternative to the sweep, not part of the step)
    t0 = time.perf_counter()
    _, val2, info2 = mc.cut_two_level()
    torch.cuda.synchronize()
    two = {"cut_value": val2, "seconds": round(time.perf_counter() - t0, 4),
           "relative_to_sweep": (val2 - val) / val, "coarse_nodes": info2["n_sc"] + 2,
           "coarse_edges": info2["coarse_edges"], "gamma": [info2["gamma0"], info2["gamma1"]]}
    print(f"[bench] two-level rounding: cut {val2:.10g} ({two['relative_to_sweep']:.2e} vs the sweep) "
          f"in {two['seconds']:.3f} s, coarse graph {two['coarse_nodes']} nodes", file=sys.stderr, flush=True)

    roof = None
    if info["solver"] == 1:
        # back-to-back launches on the last round's system, for comparison
        b2b_ms = mc.time_kernel(0, args.kernel_reps)
        # the update alternates between odd and even iterations (they differ
        # on the scaled system): the mean of the two
        upd_ms = 0.5 * (mc.time_kernel(1, args.kernel_reps) + mc.time_kernel(2, args.kernel_reps))
        variant, spmv_grid = mc.spmv_variant()
        kname = mc.SPMV_KERNELS[variant]
        nbytes = spmv_bytes(info, opts.get("precision", 0), variant)
        if ktime and ktime["n_working"] > 0:
            spmv_ms = ktime["ms_working"] / ktime["n_working"]
            how = (f"mean of {ktime['n_working']} SpMV launches that did work in the {args.steps} "
                   f"timed steps: those of CG iterations 0, {args.kernel_events}, "
                   f"{2 * args.kernel_events}, ... of every round, each between two HIP events on the "
                   f"solve's stream ({ktime['n_all'] - ktime['n_working']} sampled launches queued past "
                   f"convergence, which return at once, are left out)")
        else:
            spmv_ms = b2b_ms
            how = f"mean of {args.kernel_reps} back-to-back launches on the last round's system"
        achieved = nbytes / (spmv_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(kname, args.workload), "kernel": kname,
                "bytes_per_launch": nbytes, "avg_launch_ms": round(spmv_ms, 5), "launch_time": how,
                "back_to_back_launch_ms": round(b2b_ms, 5), "workgroups": spmv_grid,
                "update_kernel_ms_back_to_back": round(upd_ms, 5), "other_kernels_in_solve": breakdown}
        print(f"[bench] spmv {spmv_ms*1e3:.1f} us in the solve ({achieved:.0f} GB/s; back to back "
              f"{b2b_ms*1e3:.1f} us), update {upd_ms*1e3:.1f} us", file=sys.stderr, flush=True)
    mc.close()
    gold = golden_run(args.workload)
    if roof and args.stream_probe and info["n_nonterminal"] % 2 == 0:
        # the bandwidth a kernel with the SpMV's mix of streams (five arrays
        # read, two written, one row each per step) and nothing else sustains
        # at this size, and a plain copy; the best of two grid sizes and of
        # plain and streaming (non-temporal) accesses
        probe = {}
        for nr, nw in ((5, 2), (1, 1)):
            best = 0.0
            for wg in (256, 1024):
                ms = P.stream_probe(info["n_nonterminal"], nr, nw, wg, 20, stream)
                best = max(best, (nr + nw) * info["n_nonterminal"] * 8 / (ms * 1e-3) / 1e9)
            probe[f"{nr}r{nw}w"] = round(best, 1)
        roof["stream_ceiling_GBps"] = probe
        roof["frac_of_stream_ceiling"] = round(roof["achieved"] / probe["5r2w"], 4)
        print(f"[bench] streaming ceiling at {info['n_nonterminal']} rows: 5 reads + 2 writes "
              f"{probe['5r2w']:.0f} GB/s, copy {probe['1r1w']:.0f} GB/s", file=sys.stderr, flush=True)

    # A mode of the library beside the configured run: the same instance with
    # the certified-gap stopping rule (rounds stop once ||CBx||_1 and the
    # round's lower bound on the minimum cut are within stop_gap), its
    # time-to-cut, and the two-level rounding of the stopped potentials.
    early = None
    if args.early_stop_gap > 0 and info["solver"] == 1:
        with P.MinCut.from_graph(g, stream=stream, stop_gap=args.early_stop_gap, **opts) as me:
            me.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ste = me.solve()
            _, vale, _ = me.cut()
            torch.cuda.synchronize()
            dte = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, vale2, _ = me.cut_two_level()
            torch.cuda.synchronize()
            dte2 = time.perf_counter() - t0
        L = max(l for l, r in enumerate(ste) if l == 0 or r["eps"] > 0)
        lb = ste[L]["lower_bound"]
        early = {"stop_gap": args.early_stop_gap, "last_round": L, "rounds_configured": opts["rounds"],
                 "cg_iters": int(sum(r["cg_iters"] for r in ste)), "seconds_to_cut": round(dte, 4),
                 "cuts_per_s": round(1.0 / dte, 3), "sweep_cut": vale, "lower_bound": lb,
                 "certified_sweep_delta_at_most": (vale - lb) / lb,
                 "two_level_cut": vale2, "two_level_seconds": round(dte2, 4),
                 "two_level_cut_equals_configured_run": vale2 == val2}
        print(f"[bench] stop_gap {args.early_stop_gap}: rounds 0..{L}, {early['cg_iters']} CG iterations, "
              f"{dte*1e3:.1f} ms to the sweep cut {vale:.10g}; two-level {vale2:.10g}", file=sys.stderr, flush=True)

    # The precision form (FP32 conductances, SpMV and CG vectors; FP64
    # potentials, dots and residual replacement) on the same instance, beside
    # the configured FP64 run: its time-to-cut and its cut against the FP64 cut.
    # Of the block-Jacobi forms only ILU(0) of 4x4x4 tiles has a precision form.
    # On a plain (Jacobi) 3-D segmentation workload the precision form with
    # block-Jacobi over 4x4x4 ILU(0) tiles is timed as well, against the same
    # plain FP64 run.
    def precision_leg(label, **kw):
        with P.MinCut.from_graph(g, stream=stream, **kw) as mp:
            mp.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, stp = mp.solve()
            _, valp, _ = mp.cut()
            torch.cuda.synchronize()
            dtp = time.perf_counter() - t0
            _, valp2, _ = mp.cut_two_level()             # untimed, as for the FP64 run
        out = {"seconds_to_cut": round(dtp, 4), "cuts_per_s": round(1.0 / dtp, 3),
               "speedup_vs_fp64": round(ms_step / 1000.0 / dtp, 3),
               "cg_iters": int(sum(r["cg_iters"] for r in stp)), "cut_value": valp,
               "relative_cut_difference_vs_fp64": abs(valp - val) / val,
               "two_level_cut": valp2, "two_level_cut_equals_fp64_run": valp2 == val2}
        if gold:
            ov = gold["sweep"]["value"]
            out["relative_cut_error_vs_fp64_oracle"] = abs(valp - ov) / ov
        print(f"[bench] {label}: {dtp*1e3:.1f} ms to the cut {valp:.10g} "
              f"({out['relative_cut_difference_vs_fp64']:.1e} from the FP64 cut)", file=sys.stderr, flush=True)
        return out

    precision = precision_ilu = None
    ilu4 = opts.get("precond", 0) == 2 and opts.get("block_size", 0) in (0, 4) and info["format"] == 2
    if (args.precision_form and info["solver"] == 1 and opts.get("precision", 0) == 0
            and (opts.get("precond", 0) == 0 or ilu4)):
        precision = precision_leg("precision form", precision=1, refine_every=20, **opts)
        if spec["kind"] == "seg" and opts.get("precond", 0) == 0:
            precision_ilu = precision_leg("precision form, ILU(0) tiles", precision=1, refine_every=20,
                                          precond=2, block_size=4, **opts)

    if args.calibrate_copy > 0:
        nel = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copies: 5 x {args.calibrate_copy} MiB read + written",
              file=sys.stderr, flush=True)
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(g, opts, iters, args.cpu_budget)
        if gold:
            cpu["full_run"] = {"seconds": round(gold["timing"]["seconds"], 1),
                               "threads": gold["timing"]["threads"], "cpu_model": gold["timing"]["cpu_model"],
                               "cg_iters": gold["cg_iters_total"], "cut_value": gold["sweep"]["value"],
                               "where": "the oracle's whole run of this instance (all rounds + sweep), "
                                        "timed when its golden file was written on the build host"}
    oracle_ref = None
    if gold:
        ov = gold["sweep"]["value"]
        oracle_ref = {"cut_value": ov, "k_star": gold["sweep"]["k_star"], "cg_iters": gold["cg_iters_total"],
                      "gpu_cut_equals_oracle": val == ov, "relative_cut_error": abs(val - ov) / ov}

    out = {
        "metric": "IRLS s-t min-cut time-to-cut, as cuts per second (solve + sweep, graph resident)",
        "value": round(args.steps / dt, 5), "unit": "cuts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if opts.get("precision", 0) == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "n_nonterminal": info["n_nonterminal"],
                   "march_tile": list(mc_tile) if mc_tile else None,
                   "interior_edges": info["nnz_offdiag"] // 2, "format": info["format"],
                   "solver": info["solver"], "cg_iters_per_cut": iters,
                   "step_ms": [round(t, 3) for t in step_ms],
                   "median_step_ms": round(sorted(step_ms)[len(step_ms) // 2], 3),
                   "warmup_step_ms_without_events": [round(t, 3) for t in warm_ms],
                   "oracle": oracle_ref,
                   "cg_iters_per_round": [int(r["cg_iters"]) for r in st], "cut_value": val,
                   "setup_s": round(t_setup, 3), "two_level": two,
                   # the last round's lower bound (its flow scaled to respect every
                   # capacity) and ||CBx||_1 bracket the minimum cut: delta of a cut
                   # is at most (cut - bound) / bound
                   "early_stop": early,
                   "precision_form": precision,
                   "precision_form_ilu0_tiles": precision_ilu,
                   "certified": {"lower_bound": st[-1]["lower_bound"], "l1": st[-1]["l1"],
                                 "sweep_delta_at_most": (val - st[-1]["lower_bound"]) / st[-1]["lower_bound"],
                                 "two_level_delta_at_most":
                                     (val2 - st[-1]["lower_bound"]) / st[-1]["lower_bound"]}},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Benchmark of the per-round decrease estimate on one MI355X.

Default workload (--workload rmat22): AdvancedGreedy rounds on the 4M-vertex R-MAT graph.
A step is one greedy round of the hot path: theta = 10,000 live-edge samples, each with
live-edge decisions, reachability from the merged seed, the dominator tree, subtree sizes
and the exact accumulation of the decrease counts, followed by the device-side argmax and
block of the round's winner (Algorithms 2 and 3 of arXiv 2302.13529).

--workload batched: 256 independent Chung-Lu instances (theta = 2,000, b = 20, TR). A step
is one batched AdvancedGreedy call over all of them (20 rounds); the same instances are
also run one plain call at a time, and the blockers of both forms must agree exactly.

Inputs are seeded synthetic data resident in HBM before the timed region starts. Prints
one JSON line: samples/s over the timed steps, the roofline figure of the dominant kernel
(algorithmic bytes per launch over its average launch time, against MI355X's 8 TB/s HBM
peak), and the CPU checker timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(stats: dict, n_seeds: int) -> float:
    """8 B per expanded vertex (its row_ptr pair; the seeds and every reached vertex), 8 B
    per scanned edge (target id + threshold), 8 B per reached vertex (counter update)."""
    expanded = stats["samples"] * n_seeds + stats["reached"]
    return 8.0 * expanded + 8.0 * stats["edges_scanned"] + 8.0 * stats["reached"]


def traffic_from_profile(path: str, kernel_source: str):
    """HBM bytes per launch from the committed counter summary, or None when there is none
    or when the kernel source changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.split()[0] if v.split() else ""
    if fields.get("kernel_source_sha256") != digest:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_workers() -> int:
    """Host cores the CPU checker runs on: this process's CPU affinity, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# What the forked checker processes work on; set before the pool forks, read in the workers.
_CPU_JOB: dict = {}


def _cpu_samples(js) -> tuple:
    """Samples js of greedy round 0 (key 0, no blockers) through the checker's one-sample
    call, subtree sizes accumulated into counts as its decrease call does."""
    import numpy as np
    from oracle import oracle as orc
    inst, model = _CPU_JOB["inst"], _CPU_JOB["model"]
    D = np.zeros(inst.n, dtype=np.uint64)
    reached = 0
    for j in js:
        r, c, _ = orc.sample(inst.n, inst.row_ptr, inst.col, inst.prob, inst.seeds, None, 0,
                             int(j), model=model)
        D += c.astype(np.uint64)
        reached += r
    return reached, len(js)


def _cpu_instances(ks) -> int:
    """Round 0 (full theta) of the listed batched instances; returns their samples."""
    from oracle import oracle as orc
    done = 0
    for k in ks:
        t = _CPU_JOB["insts"][k]
        _, st = orc.decrease(t.n, t.row_ptr, t.col, t.prob, t.seeds, None, t.theta, t.seed)
        done += st["samples"]
    return done


def _parallel(fn, parts):
    """fn over parts in forked processes (one per part, the checker unchanged); returns the
    results and the wall time of the work alone. Must run before this process touches the
    GPU."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(len(parts)) as pool:
        pool.map(abs, range(len(parts)))  # every worker up before the clock starts
        t0 = time.perf_counter()
        res = pool.map(fn, parts)
        dt = time.perf_counter() - t0
    return res, dt


def cpu_baseline(inst, theta_sample: int, model: str = "ic") -> dict:
    """The checker on samples 0..theta_sample-1 of greedy round 0, spread over the host
    cores (each process takes every k-th sample)."""
    from oracle import oracle as orc
    cores = min(cpu_workers(), theta_sample)
    _CPU_JOB.update(inst=inst, model=orc.LT if model == "lt" else orc.IC)
    res, dt = _parallel(_cpu_samples, [list(range(w, theta_sample, cores))
                                       for w in range(cores)])
    done = sum(k for _, k in res)
    return {"value": done / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} of the {inst.theta} samples of greedy round 0 "
                      f"(no blockers, key 0) on {inst.name}, C checker in {cores} processes "
                      f"(every {cores}-th sample each), {dt:.1f} s"}


def bench_batched(args) -> dict:
    import torch
    from paper_2302_13529_amd import binding, graphgen as gg

    print("[bench] generating 256 batched instances", file=sys.stderr, flush=True)
    insts = gg.batched_instances()
    cpu = None
    if not args.no_cpu:
        # the checker's processes fork before this process touches the GPU
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cores = cpu_workers()
        _CPU_JOB.update(insts=insts)
        res, cdt = _parallel(_cpu_instances, [list(range(w, len(insts), cores))
                                              for w in range(cores)])
        cpu = {"value": sum(res) / cdt, "unit": "samples/s", "cores": cores, "kind": "oracle",
               "sample": f"round 0 (full theta) of all {len(insts)} instances, C checker in "
                         f"{cores} processes (every {cores}-th instance each), {cdt:.1f} s"}
    graphs = [binding.Graph(t.row_ptr, t.col, t.prob) for t in insts]
    probs = [(g.handle, t.seeds, t.b, t.theta, t.seed) for g, t in zip(graphs, insts)]
    from paper_2302_13529_amd import autotune
    launch = dict(waves_per_cu=args.waves_per_cu, quad_limit=args.quad_limit,
                  pick_div=args.pick_div)
    tuned_key = None
    if not any(launch.values()):
        print("[bench] launch shape from the autotuner", file=sys.stderr, flush=True)
        tuned_key, tuned = autotune.tuned_batch_launch(insts, probs, tune_if_missing=args.tune)
        if tuned:
            launch = dict(tuned)
    launch["graph"] = 1 if args.graph else 0
    print(f"[bench] warmup: plain and batched, {args.warmup} each", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        for g, t in zip(graphs, insts):
            g.greedy(t.seeds, t.b, t.theta, t.seed, binding.IMIN_AG)
        binding.imin_greedy_batch(probs, binding.IMIN_AG, launch)
    torch.cuda.synchronize()
    print(f"[bench] plain: {len(insts)} greedy calls", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plain = [g.greedy(t.seeds, t.b, t.theta, t.seed, binding.IMIN_AG)
             for g, t in zip(graphs, insts)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain_samples = sum(st["samples"] for _, st in plain)
    print(f"[bench] batched: {args.steps} calls", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = binding.imin_greedy_batch(probs, binding.IMIN_AG, launch)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    identical = all(list(a[0]) == list(b[0]) for a, b in zip(plain, res))
    stats = {k: sum(st[k] for _, st in res) for k in
             ("samples", "reached", "edges_scanned", "live_edges", "wave_samples")}
    samples = stats["samples"] * args.steps
    kernel_ms = res[0][1]["kernel_ms"]  # the batch's sampling launches, last call
    alg = sum(algorithmic_bytes(st, len(t.seeds)) for (_, st), t in zip(res, insts))
    rounds = max(t.b for t in insts)
    achieved = alg / (kernel_ms / 1e3) / 1e9
    out = {
        "metric": "live-edge samples/sec incl. dominator decrease",
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "chunglu_batch256_tr", "instances": len(insts),
                   "theta": insts[0].theta, "b": insts[0].b,
                   "step": "one batched AdvancedGreedy call over all instances",
                   "parallelism": "none", "launch": launch, "tuned_key": tuned_key},
        "plain_value": plain_samples / plain_s,
        "speedup_vs_plain": (samples / dt) / (plain_samples / plain_s),
        "identical_to_plain": identical,
        "wave_share": stats["wave_samples"] / max(1, stats["samples"]),
        "teps": stats["edges_scanned"] * args.steps / dt,
        "reached_per_sample": stats["reached"] / max(1, stats["samples"]),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "decrease_small_kernel",
                     "algorithmic_bytes_per_launch": alg / rounds,
                     "avg_launch_ms": kernel_ms / rounds},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for g in graphs:
        g.close()
    return out


def bench_served(args) -> dict:
    import numpy as np
    import torch
    from paper_2302_13529_amd import binding, graphgen as gg, serve

    print("[bench] generating the served graph and queries", file=sys.stderr, flush=True)
    inst = gg.served_graph()
    queries = gg.served_queries(inst.n)[: args.queries]
    g = binding.Graph(inst.row_ptr, inst.col, inst.prob)
    budget = int(args.hbm_gib * (1 << 30))
    launch = {k: v for k, v in dict(waves_per_cu=args.waves_per_cu, quad_limit=args.quad_limit,
                                    pick_div=args.pick_div).items() if v}
    srv = binding.Server(g, hbm_budget=budget, max_active=args.max_active, max_theta=10000,
                         launch=launch or None)
    # plain form: one imin_greedy call per query, on a bounded prefix of the mix
    plain_n = min(args.plain_queries, len(queries))
    print(f"[bench] plain: warmup + {plain_n} queries", file=sys.stderr, flush=True)
    q0 = queries[0]
    g.greedy(q0["seeds"], 2, q0["theta"], q0["seed"], binding.IMIN_AG)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], binding.IMIN_AG)
             for q in queries[:plain_n]]
    plain_s = time.perf_counter() - t0
    plain_samples = sum(st["samples"] for _, st in plain)
    plain_qps = plain_n / plain_s
    # served, saturated: every query submitted at time 0
    print(f"[bench] served, saturated: {len(queries)} queries", file=sys.stderr, flush=True)
    res, lat_sat, span, steps = serve.run(srv, queries)
    served_samples = sum(st["samples"] for _, st in res)
    identical = all(list(res[i][0]) == list(plain[i][0]) and
                    res[i][1]["reached"] == plain[i][1]["reached"] for i in range(plain_n))
    # served, Poisson arrivals at 0.8x the plain form's query rate
    rate = 0.8 * plain_qps
    arrivals = serve.poisson_arrivals(len(queries), rate, seed=7)
    print(f"[bench] served, Poisson arrivals at {rate:.2f} queries/s", file=sys.stderr,
          flush=True)
    res2, lat, span2, steps2 = serve.run(srv, queries, arrivals)
    identical = identical and all(list(a[0]) == list(b[0]) for a, b in zip(res, res2))
    srv.close()
    g.close()
    out = {
        "metric": "live-edge samples/sec incl. dominator decrease",
        "value": served_samples / span,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": span * 1e3 / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": inst.name, "n": inst.n, "m": inst.m, "queries": len(queries),
                   "step": "one server step: a greedy round of every admitted query",
                   "hbm_budget_gib": args.hbm_gib, "max_active": args.max_active,
                   "launch": launch,
                   "parallelism": "none"},
        "plain_value": plain_samples / plain_s,
        "plain_queries": plain_n,
        "speedup_vs_plain": (served_samples / span) / (plain_samples / plain_s),
        "identical_to_plain": identical,
        "saturated_makespan_s": span,
        "poisson_rate_qps": rate,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "poisson_makespan_s": span2,
        "queries_per_s_served": len(queries) / span,
        "queries_per_s_plain": plain_qps,
    }
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-samples", type=int, default=256,
                    help="rmat22: samples the CPU checker times (an eighth of it under LT, whose "
                         "samples reach about 3x more vertices)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["rmat22", "batched", "served"], default="rmat22")
    ap.add_argument("--model", choices=["ic", "lt"], default="ic",
                    help="rmat22: propagation model (lt: WC weights as linear-threshold weights)")
    ap.add_argument("--queries", type=int, default=2000, help="served: queries of the mix")
    ap.add_argument("--plain-queries", type=int, default=40,
                    help="served: queries timed one plain call at a time")
    ap.add_argument("--hbm-gib", type=float, default=16.0, help="served: query-state budget")
    ap.add_argument("--max-active", type=int, default=256, help="served: admitted at once")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--quad-limit", type=int, default=0)
    ap.add_argument("--pick-div", type=int, default=0)
    ap.add_argument("--graph", action="store_true",
                    help="batched workload: capture each call's rounds into one HIP graph")
    ap.add_argument("--tune", action="store_true",
                    help="batched workload: tune the launch shape if no cached entry exists")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would shard across GPUs with one integer reduction of the counts "
              "per round; see the design notes)", file=sys.stderr)
        return 2
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0
    if args.workload == "served":
        print(json.dumps(bench_served(args)), flush=True)
        return 0

    import torch
    from paper_2302_13529_amd import binding, graphgen as gg

    print("[bench] generating rmat22 workload", file=sys.stderr, flush=True)
    inst = gg.large_plain()
    cpu = None
    if not args.no_cpu:
        # the checker's processes fork before this process touches the GPU
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        k = args.cpu_samples if args.model == "ic" else max(1, args.cpu_samples // 8)
        cpu = cpu_baseline(inst, k, args.model)
    torch.cuda.set_device(0)
    model = binding.IMIN_LT if args.model == "lt" else binding.IMIN_IC
    g = binding.Graph(inst.row_ptr, inst.col, inst.prob, model=model)
    theta = inst.theta
    print(f"[bench] warmup {args.warmup} rounds", file=sys.stderr, flush=True)
    if args.warmup > 0:
        g.greedy(inst.seeds, args.warmup, theta, 1000, binding.IMIN_AG)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} rounds", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    B, st = g.greedy(inst.seeds, args.steps, theta, 0, binding.IMIN_AG)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()

    samples = st["samples"]
    launches = args.steps
    alg = algorithmic_bytes(st, len(inst.seeds))
    kernel_s = st["kernel_ms"] / 1e3
    achieved = alg / kernel_s / 1e9
    traffic = traffic_from_profile(
        os.path.join(ROOT, "profiles", "decrease_kernel_rmat22_pmc.txt"),
        os.path.join(ROOT, "paper_2302_13529_amd", "csrc", "decrease.hip"))
    out = {
        "metric": "live-edge samples/sec incl. dominator decrease",
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": inst.name + ("_lt" if args.model == "lt" else ""),
                   "model": args.model.upper(), "n": inst.n, "m": inst.m, "seeds": len(inst.seeds),
                   "theta": theta, "step": "one AdvancedGreedy round", "parallelism": "none"},
        "teps": st["edges_scanned"] / dt,
        "reached_per_sample": st["reached"] / samples,
        "blockers": [int(x) for x in B],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "decrease_kernel",
                     "algorithmic_bytes_per_launch": alg / launches,
                     "avg_launch_ms": st["kernel_ms"] / launches},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark of the per-round decrease estimate on one MI355X.

Headline (default): AdvancedGreedy rounds on the 4M-vertex R-MAT graph. A step is one
greedy round of the hot path: theta = 10,000 live-edge samples, each with live-edge
decisions, reachability from the merged seed, the dominator tree, subtree sizes and the
exact accumulation of the decrease counts, followed by the device-side argmax and block of
the round's winner (Algorithms 2 and 3 of arXiv 2302.13529).

The default line also carries two sub-objects:
* "batched": 256 independent Chung-Lu instances (theta = 2,000, b = 20, TR); a step is one
  batched AdvancedGreedy call over all of them (20 rounds), against every instance run as a
  plain call (speed-up, identical blockers);
* "served": the 2^20-vertex R-MAT graph resident and the 2,000-query mix, saturated
  (samples/s against plain calls on a prefix), then a prefix under Poisson arrivals (p50 /
  p99 latency).
Each carries "verified": its blockers and work counters against the CPU oracle's stored
results at that configuration (tests/golden).

Inputs are seeded synthetic data resident in HBM before the timed region starts. Prints
one JSON line: samples/s over the timed steps, the roofline figure of the dominant kernel
(algorithmic bytes per launch over its average launch time, against MI355X's 8 TB/s HBM
peak), and the CPU oracle timed on a bounded sample of the same workload.
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
    per scanned edge (target id + threshold), 16 B per reached vertex (the read-modify-write
    of its 64-bit decrease counter)."""
    expanded = stats["samples"] * n_seeds + stats["reached"]
    return 8.0 * expanded + 8.0 * stats["edges_scanned"] + 16.0 * stats["reached"]


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden(name: str) -> dict:
    """A stored result of the CPU oracle at a benchmark configuration (tests/golden), read
    as text: blocker lists and work counters to compare the GPU's results with."""
    sys.path.insert(0, ROOT)
    from tests import helpers
    path = os.path.join(GOLDEN, name)
    return helpers.read_config_golden(name) if os.path.exists(path) else {}


def _stats4(st: dict) -> dict:
    return {k: int(st[k]) for k in ("samples", "reached", "edges_scanned", "live_edges")}


def traffic_from_profile(path: str, kernel_source: str):
    """HBM bytes per launch from the committed counter summary (rocprofv3 FETCH_SIZE and
    WRITE_SIZE of the same workload, scaled by a copy kernel's calibration), or None when
    there is none or when the kernel source changed since the counters were taken."""
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
    """Host cores the CPU oracle runs on: this process's CPU affinity, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# What the forked oracle processes work on; set before the pool forks, read in the workers.
_CPU_JOB: dict = {}


def _cpu_samples(js) -> tuple:
    """Samples js of greedy round 0 (key 0, no blockers) through the oracle's one-sample
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
    """fn over parts in forked processes (one per part, the oracle unchanged); returns the
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
    """The oracle on samples 0..theta_sample-1 of greedy round 0, spread over the host
    cores (each process takes every k-th sample)."""
    from oracle import oracle as orc
    cores = min(cpu_workers(), theta_sample)
    _CPU_JOB.update(inst=inst, model=orc.LT if model == "lt" else orc.IC)
    res, dt = _parallel(_cpu_samples, [list(range(w, theta_sample, cores))
                                       for w in range(cores)])
    done = sum(k for _, k in res)
    return {"value": done / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} of the {inst.theta} samples of greedy round 0 "
                      f"(no blockers, key 0) on {inst.name}, C oracle in {cores} processes "
                      f"(every {cores}-th sample each), {dt:.1f} s"}


def batched_cpu_baseline(insts) -> dict:
    """The oracle on round 0 (full theta) of every batched instance, in forked processes;
    call it before this process touches the GPU."""
    print("[bench] cpu baseline (batched instances)", file=sys.stderr, flush=True)
    cores = cpu_workers()
    _CPU_JOB.update(insts=insts)
    res, cdt = _parallel(_cpu_instances, [list(range(w, len(insts), cores))
                                          for w in range(cores)])
    return {"value": sum(res) / cdt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"round 0 (full theta) of all {len(insts)} instances, C oracle in "
                      f"{cores} processes (every {cores}-th instance each), {cdt:.1f} s"}


def bench_batched(args, with_cpu: bool, insts=None, cpu=None) -> dict:
    """256 Chung-Lu instances: every instance as a plain imin_greedy call, then args.steps
    batched calls over all of them; blockers compared with each other and with the oracle's
    stored results. `insts` and `cpu` may come from an earlier generation and oracle run."""
    import torch
    from paper_2302_13529_amd import binding, graphgen as gg

    if insts is None:
        print("[bench] generating 256 batched instances", file=sys.stderr, flush=True)
        insts = gg.batched_instances()
    if with_cpu and cpu is None:
        # the oracle's processes fork before this process touches the GPU
        cpu = batched_cpu_baseline(insts)
    graphs = [binding.Graph(t.row_ptr, t.col, t.prob) for t in insts]
    probs = [(g.handle, t.seeds, t.b, t.theta, t.seed) for g, t in zip(graphs, insts)]
    from paper_2302_13529_amd import autotune
    launch = dict(waves_per_cu=args.waves_per_cu, quad_limit=args.quad_limit,
                  pick_div=args.pick_div, pack_per_cu=args.pack_per_cu)
    tuned_key = None
    if not any(launch.values()):
        print("[bench] launch shape from the autotuner", file=sys.stderr, flush=True)
        tuned_key, tuned = autotune.tuned_batch_launch(insts, probs, tune_if_missing=args.tune)
        if tuned:
            launch = dict(tuned)
    launch["graph"] = int(args.graph)
    warm = max(1, args.warmup)
    print(f"[bench] warmup: plain and batched, {warm} each", file=sys.stderr, flush=True)
    for _ in range(warm):
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
    steps = max(1, args.batched_steps)
    print(f"[bench] batched: {steps} calls", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = binding.imin_greedy_batch(probs, binding.IMIN_AG, launch)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    identical = all(list(a[0]) == list(b[0]) and _stats4(a[1]) == _stats4(b[1])
                    for a, b in zip(plain, res))
    want = golden("config_c3.txt")
    verified = None
    if want:
        verified = all([int(x) for x in B] == want[("inst", i)][0] and
                       _stats4(st) == want[("inst", i)][1] for i, (B, st) in enumerate(res))
    stats = {k: sum(st[k] for _, st in res) for k in
             ("samples", "reached", "edges_scanned", "live_edges", "wave_samples",
              "pack_samples")}
    samples = stats["samples"] * steps
    kernel_ms = res[0][1]["kernel_ms"]  # the batch's sampling launches, last call
    alg = sum(algorithmic_bytes(st, len(t.seeds)) for (_, st), t in zip(res, insts))
    rounds = max(t.b for t in insts)
    achieved = alg / (kernel_ms / 1e3) / 1e9
    out = {
        "value": samples / dt,
        "unit": "samples/s",
        "steps": steps,
        "ms_per_step": dt * 1e3 / steps,
        "config": {"workload": "chunglu_batch256_tr", "instances": len(insts),
                   "theta": insts[0].theta, "b": insts[0].b,
                   "step": "one batched AdvancedGreedy call over all instances (20 rounds)",
                   "launch": launch, "tuned_key": tuned_key},
        "plain_value": plain_samples / plain_s,
        "speedup_vs_plain": (samples / dt) / (plain_samples / plain_s),
        "identical_to_plain": identical,
        "verified": {"vs_oracle": verified, "instances": len(insts), "rounds": rounds,
                     "source": "tests/golden/config_c3.txt"},
        "pack_share": stats["pack_samples"] / max(1, stats["samples"]),
        "wave_share": stats["wave_samples"] / max(1, stats["samples"]),
        "teps": stats["edges_scanned"] * steps / dt,
        "reached_per_sample": stats["reached"] / max(1, stats["samples"]),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "decrease_pack_kernel with the workgroup kernel for its "
                               "hand-overs (one round's sampling launches)",
                     "algorithmic_bytes_per_launch": alg / rounds,
                     "avg_launch_ms": kernel_ms / rounds},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for g in graphs:
        g.close()
    return out


def bench_served(args) -> dict:
    """The 2^20-vertex R-MAT graph resident, the served query mix: a prefix as plain calls,
    the whole mix saturated (every query submitted at time 0), then a prefix under Poisson
    arrivals at 0.8x the plain form's query rate for latency."""
    import numpy as np
    import torch
    from paper_2302_13529_amd import binding, graphgen as gg, serve

    print("[bench] generating the served graph and queries", file=sys.stderr, flush=True)
    inst = gg.served_graph()
    allq = gg.served_queries(inst.n)
    queries = allq[: args.queries]
    g = binding.Graph(inst.row_ptr, inst.col, inst.prob)
    budget = int(args.hbm_gib * (1 << 30))
    launch = {k: v for k, v in dict(waves_per_cu=args.waves_per_cu, quad_limit=args.quad_limit,
                                    pick_div=args.pick_div,
                                    pack_per_cu=args.pack_per_cu).items() if v}
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
                    _stats4(res[i][1]) == _stats4(plain[i][1]) for i in range(plain_n))
    want = golden("config_c5.txt")
    checked = [i for kind, i in want if kind == "query" and i < len(queries)]
    verified = None
    if checked:
        verified = all([int(x) for x in res[i][0]] == want[("query", i)][0] and
                       _stats4(res[i][1]) == want[("query", i)][1] for i in checked)
    # served, Poisson arrivals at 0.8x the plain form's query rate, on a prefix of the mix
    pq = queries[: min(args.poisson_queries, len(queries))]
    rate = 0.8 * plain_qps
    arrivals = serve.poisson_arrivals(len(pq), rate, seed=7)
    print(f"[bench] served, Poisson arrivals at {rate:.2f} queries/s, {len(pq)} queries",
          file=sys.stderr, flush=True)
    res2, lat, span2, steps2 = serve.run(srv, pq, arrivals)
    identical = identical and all(list(a[0]) == list(b[0]) and _stats4(a[1]) == _stats4(b[1])
                                  for a, b in zip(res, res2))
    srv.close()
    g.close()
    return {
        "value": served_samples / span,
        "unit": "samples/s",
        "steps": steps,
        "ms_per_step": span * 1e3 / max(steps, 1),
        "config": {"workload": inst.name, "n": inst.n, "m": inst.m, "queries": len(queries),
                   "step": "one server step: a greedy round of every admitted query",
                   "hbm_budget_gib": args.hbm_gib, "max_active": args.max_active,
                   "launch": launch},
        "plain_value": plain_samples / plain_s,
        "plain_queries": plain_n,
        "speedup_vs_plain": (served_samples / span) / (plain_samples / plain_s),
        "identical_to_plain": identical,
        "verified": {"vs_oracle": verified, "queries": len(checked),
                     "source": "tests/golden/config_c5.txt"},
        "saturated_makespan_s": span,
        "queries_per_s_served": len(queries) / span,
        "queries_per_s_plain": plain_qps,
        "poisson_queries": len(pq),
        "poisson_rate_qps": rate,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "poisson_makespan_s": span2,
    }


def line(value: float, unit: str, steps: int, warmup: int, ms_per_step: float,
         config: dict) -> dict:
    return {"metric": "live-edge samples/sec incl. dominator decrease", "value": value,
            "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": config}


def bench_headline(args) -> dict:
    """AdvancedGreedy rounds on the 4M-vertex R-MAT graph (or its LT variant)."""
    import torch
    from paper_2302_13529_amd import binding, graphgen as gg

    print("[bench] generating rmat22 workload", file=sys.stderr, flush=True)
    inst = gg.large_plain()
    cpu = None
    if not args.no_cpu:
        # the oracle's processes fork before this process touches the GPU
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
    prof = os.path.join("profiles", "decrease_kernel_rmat22_pmc.txt")
    src = os.path.join("paper_2302_13529_amd", "csrc", "decrease.hip")
    traffic = traffic_from_profile(os.path.join(ROOT, prof), os.path.join(ROOT, src))
    out = line(samples / dt, "samples/s", args.steps, args.warmup, dt * 1e3 / args.steps,
               {"workload": inst.name + ("_lt" if args.model == "lt" else ""),
                "model": args.model.upper(), "n": inst.n, "m": inst.m,
                "seeds": len(inst.seeds), "theta": theta, "counter_bits": 64,
                "step": "one AdvancedGreedy round", "parallelism": "none"})
    out.update({
        "teps": st["edges_scanned"] / dt,
        "reached_per_sample": st["reached"] / samples,
        "blockers": [int(x) for x in B],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": (f"{prof} (rocprofv3 FETCH_SIZE/WRITE_SIZE of this "
                                        f"kernel source, sha256 match)") if traffic else None,
                     "kernel": "decrease_kernel",
                     "algorithmic_bytes_per_launch": alg / launches,
                     "avg_launch_ms": st["kernel_ms"] / launches},
    })
    want = golden("config_c4.txt").get("greedy2", {})
    if args.model == "ic" and want.get("blockers"):
        k = min(len(B), len(want["blockers"]))
        out["verified"] = {"vs_oracle": [int(x) for x in B[:k]] == want["blockers"][:k],
                           "rounds": k, "source": "tests/golden/config_c4.txt"}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-samples", type=int, default=256,
                    help="rmat22: samples the CPU oracle times (an eighth of it under LT, whose "
                         "samples reach about 3x more vertices)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["all", "rmat22", "batched", "served"], default="all",
                    help="all: the rmat22 line with the batched and served forms as sub-objects")
    ap.add_argument("--model", choices=["ic", "lt"], default="ic",
                    help="rmat22: propagation model (lt: WC weights as linear-threshold weights)")
    ap.add_argument("--batched-steps", type=int, default=3, help="batched: timed calls")
    ap.add_argument("--queries", type=int, default=2000, help="served: queries of the mix")
    ap.add_argument("--plain-queries", type=int, default=40,
                    help="served: queries timed one plain call at a time")
    ap.add_argument("--poisson-queries", type=int, default=300,
                    help="served: prefix of the mix run under Poisson arrivals for latency")
    ap.add_argument("--hbm-gib", type=float, default=16.0, help="served: query-state budget")
    ap.add_argument("--max-active", type=int, default=256, help="served: admitted at once")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--quad-limit", type=int, default=0)
    ap.add_argument("--pick-div", type=int, default=0)
    ap.add_argument("--pack-per-cu", type=int, default=0,
                    help="batched/served: packed-kernel workgroups per CU (-1: that kernel off)")
    ap.add_argument("--graph", type=int, choices=[0, 1], default=1,
                    help="batched workload: 1 (default) runs each call's rounds as one HIP graph, "
                         "captured once per launch structure and replayed; 0 launches directly")
    ap.add_argument("--tune", action="store_true",
                    help="batched workload: tune the launch shape if no cached entry exists")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(samples would shard across GPUs with one integer reduction of the counts "
              "per round)", file=sys.stderr)
        return 2
    if args.workload == "batched":
        b = bench_batched(args, with_cpu=not args.no_cpu)
        out = line(b.pop("value"), b.pop("unit"), b.pop("steps"), max(1, args.warmup),
                   b.pop("ms_per_step"), b.pop("config"))
        out.update(b)
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "served":
        sv = bench_served(args)
        out = line(sv.pop("value"), sv.pop("unit"), sv.pop("steps"), 1, sv.pop("ms_per_step"),
                   sv.pop("config"))
        out.update(sv)
        print(json.dumps(out), flush=True)
        return 0
    insts = cpu_b = None
    if args.workload == "all":
        # the batched instances' oracle run forks before anything touches the GPU
        from paper_2302_13529_amd import graphgen as gg
        insts = gg.batched_instances()
        if not args.no_cpu:
            cpu_b = batched_cpu_baseline(insts)
    out = bench_headline(args)
    if args.workload == "all":
        out["batched"] = bench_batched(args, with_cpu=False, insts=insts, cpu=cpu_b)
        out["served"] = bench_served(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

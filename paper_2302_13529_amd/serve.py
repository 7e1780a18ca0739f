"""Serving driver: a request loop over ``binding.Server`` with Poisson arrivals.

Queries arrive at seeded exponential gaps; the loop submits every query whose arrival time
has passed, runs one server step (one greedy round of every admitted query, admission by
device-memory footprint, retirement of finished queries), and records each query's
completion time. Latency is completion minus arrival. The server itself is native (the
``imin_server_*`` calls); this module only paces submissions and keeps the clock.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of `rate` queries/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def run(server: binding.Server, queries, arrivals=None, clock=time.perf_counter):
    """Serve `queries` (dicts with seeds, b, theta, seed, and optionally mode: AdvancedGreedy
    by default). With arrivals None every query is submitted at time 0 (saturation). Returns
    (results, latencies, makespan, steps): results and latencies in query order."""
    n = len(queries)
    arrivals = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    order = np.argsort(arrivals, kind="stable")
    results = [None] * n
    latency = np.zeros(n)
    pending = {}
    nxt = 0
    steps = 0
    t0 = clock()
    while nxt < n or pending:
        now = clock() - t0
        while nxt < n and arrivals[order[nxt]] <= now:
            i = int(order[nxt])
            q = queries[i]
            t = server.submit(q["seeds"], q["b"], q["theta"], q["seed"],
                              q.get("mode", binding.IMIN_AG))
            pending[t] = i
            nxt += 1
        if not pending:
            time.sleep(max(0.0, arrivals[order[nxt]] - now))
            continue
        server.step()
        steps += 1
        done_at = clock() - t0
        for t in server.completed():
            i = pending.pop(t)
            results[i] = server.result(t, max(int(queries[i]["b"]), 1))
            latency[i] = done_at - arrivals[i]
    return results, latency, clock() - t0, steps

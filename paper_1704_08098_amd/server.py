"""Serving front-end: a request loop over the C job server (continuous batching).

Jobs arrive over time (e.g. a Poisson trace from workloads.serving_trace);
the loop submits every job whose arrival time has passed, steps the engine
(admission by HBM footprint, one chunk of sweeps for all resident jobs,
retirement), and stamps each job's completion.  Latency = completion -
arrival on the wall clock; throughput = site updates completed / makespan,
and, over the steps that began with jobs still queued (the engine saturated),
the site updates those steps did / their duration.
The engine is any object with submit/step/completed/result/stats (the C
engine `pgg.ServerEngine`, or a stand-in for host-only tests).
"""
from __future__ import annotations

import time

import numpy as np


def percentile(values, q):
    """q-th percentile (nearest rank, q in [0, 100]) of a non-empty sequence."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        raise ValueError("no values")
    k = int(np.ceil(q / 100.0 * v.size)) - 1
    return float(v[min(max(k, 0), v.size - 1)])


def serve(engine, jobs, clock=time.perf_counter, sleep=time.sleep, keep_results=False):
    """Run a job trace through the engine in real time.

    jobs: dicts with arrival (s, relative to the start), L, r, K, p0, seed,
    sweeps.  Returns a report dict; with keep_results, also the counts and
    final lattice of every job (by trace index).
    """
    order = sorted(range(len(jobs)), key=lambda k: jobs[k]["arrival"])
    nxt = 0
    id_to_job = {}
    submitted_at = {}
    finished_at = {}
    results = {}
    steps = 0
    resident_hist = []
    # saturation: the steps that began with jobs still waiting in the queue
    # (the engine had more work than it admitted), and the site updates they did
    sat_time, sat_updates = 0.0, 0
    t0 = clock()
    while len(finished_at) < len(jobs):
        now = clock() - t0
        while nxt < len(order) and jobs[order[nxt]]["arrival"] <= now:
            j = jobs[order[nxt]]
            jid = engine.submit(j["L"], j["r"], j["sweeps"], K=j.get("K", 0.5), p0=j.get("p0", 0.5),
                                seed=j.get("seed", 1))
            id_to_job[jid] = order[nxt]
            submitted_at[order[nxt]] = now
            nxt += 1
        if len(submitted_at) == len(finished_at):
            # nothing in flight: wait for the next arrival
            sleep(max(0.0, jobs[order[nxt]]["arrival"] - (clock() - t0)))
            continue
        st0 = engine.stats()
        step_t0 = clock()
        n_res = engine.step()
        if st0["queued"] > 0:
            sat_time += clock() - step_t0
            sat_updates += engine.stats()["site_updates"] - st0["site_updates"]
        steps += 1
        resident_hist.append(n_res)
        done_t = clock() - t0
        for jid in engine.completed():
            k = id_to_job[jid]
            finished_at[k] = done_t
            counts, lat = engine.result(jid, want_lattice=keep_results)
            if keep_results:
                results[k] = (counts, lat)
    makespan = clock() - t0
    lat_s = [finished_at[k] - jobs[k]["arrival"] for k in range(len(jobs))]
    updates = sum(float(j["L"]) ** 2 * j["sweeps"] for j in jobs)
    report = {
        "jobs": len(jobs), "steps": steps, "makespan_s": makespan,
        "latency_p50_s": percentile(lat_s, 50), "latency_p99_s": percentile(lat_s, 99),
        "latency_mean_s": float(np.mean(lat_s)), "site_updates": updates,
        "site_updates_per_s": updates / makespan if makespan > 0 else float("nan"),
        "mean_resident": float(np.mean(resident_hist)) if resident_hist else 0.0,
        "saturated_s": sat_time,
        "site_updates_per_s_saturated": sat_updates / sat_time if sat_time > 0 else None,
        "max_resident": int(max(resident_hist)) if resident_hist else 0,
        "engine": engine.stats(),
    }
    if keep_results:
        report["results"] = results
        report["latencies"] = lat_s
    return report


def capacity(pgg, n_jobs=1024, max_resident=256, chunk=16, budget_mib=256, master_seed=11, stream=None):
    """The C server's saturated capacity: n_jobs jobs of the serving
    distribution (workloads.serving_trace) submitted at once, at most
    max_resident on the device; the report of serve() on that batch."""
    from . import workloads as wl
    jobs = wl.serving_trace(n_jobs, 1.0, master_seed=master_seed)
    for j in jobs:
        j["arrival"] = 0.0
    engine = pgg.ServerEngine(budget_mib << 20, max_L=2048, max_resident=max_resident, chunk=chunk, stream=stream)
    try:
        rep = serve(engine, jobs)
    finally:
        engine.close()
    rep.pop("engine", None)
    return rep


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="the job server's saturated capacity on the serving distribution")
    ap.add_argument("--jobs", type=int, default=1024)
    ap.add_argument("--max-resident", type=int, default=256)
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--budget-mib", type=int, default=256)
    ap.add_argument("--seed", type=int, default=11, help="master seed of the job trace")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    from . import pgg
    pgg.load()
    print("server capacity: %d jobs, at most %d resident, chunk %d" % (args.jobs, args.max_resident, args.chunk),
          file=sys.stderr, flush=True)
    rep = capacity(pgg, args.jobs, args.max_resident, args.chunk, args.budget_mib, args.seed)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()

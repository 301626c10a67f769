#!/usr/bin/env python3
"""Benchmark of the spatial public goods game sweep on one MI355X.

A step is one Monte Carlo step (one sweep of the 16 colour classes) of the
L x L lattice.  Default workload: L = 4096 (16.8 M sites), r = 3.7443 (the
critical point of Sec. V), K = 0.5, i.i.d. 50/50 start, seed 1; W untimed
sweeps, then K timed sweeps (t = W .. W+K-1), inputs resident in HBM.

Prints one JSON line:
  value       whole-job site updates/s (L^2 * K / wall time of the K sweeps)
  roofline    the dominant kernel (the paired segment sweep) against the HBM
              roof at the algorithmic bytes of the state (read + write once
              per sweep), from its event-timed average launch duration, with
              its measured traffic and its counter-measured VALU use
  windows     the early (timed) window and the late one (t = 10^4), each with
              the fraction of updates that draw random numbers
  dense       the data-independent rate with every site drawing its random
              numbers (no skipping of no-op updates)
  late        the same lattice later in its decay (sweeps 10^4 .. 10^4+K-1)
  batched     256 replicas of uneven L, r, seed in one graph-replayed ensemble
              (the tuner's settings) vs the same replicas one lattice at a time
  serving     a Poisson trace of simulation jobs through the job server:
              p50/p99 latency and aggregate site updates/s
  cpu_baseline  the oracle, single-threaded, on a bounded sample
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

from paper_1704_08098_amd import workloads as wl  # noqa: E402

METRIC = "site updates/s at L=4096 (% HBM roofline); batched replica updates/s vs plain"

# MI355X peaks (published): HBM3E 8 TB/s; 256 CUs at 2.4 GHz, 64 VALU lanes
# per CU per cycle (4 SIMDs x 16 lanes) for full-rate 32-bit operations.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.3 T full-rate lane-ops/s

# VALU issue of the dominant kernel is read from committed SQ counter
# summaries (rocprofv3 --pmc), like the traffic: per dispatch, the VALU
# instructions issued and the lane-cycles they kept busy; the summary records
# the hash of the kernel's sources, and a changed kernel reads as null.
COUNTER_PROFILES = {"segment": os.path.join(ROOT, "profiles", "k_ens_segment_L4096_sq_counters.txt"),
                    "segment_pair": os.path.join(ROOT, "profiles", "k_ens_pair_L4096_sq_counters.txt")}
N_SIMDS = 256 * 4
GPU_CLOCK_HZ = 2.4e9
TRAFFIC_PROFILES = {"segment": os.path.join(ROOT, "profiles", "k_ens_segment_L4096_traffic.txt"),
                    "segment_pair": os.path.join(ROOT, "profiles", "k_ens_pair_L4096_traffic.txt")}
KERNEL_SOURCES = ("paper_1704_08098_amd/csrc/pgg_segment.hpp", "paper_1704_08098_amd/csrc/pgg_fullrow.hpp",
                  "paper_1704_08098_amd/csrc/pgg_ens_kernels.hip", "paper_1704_08098_amd/csrc/pgg_device.hpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, L, tile, group):
    """Bytes per launch from the committed counter summary, or None."""
    path = TRAFFIC_PROFILES.get(kernel)
    if path is None or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if (kv["source_hash"] != kernel_source_hash() or int(kv["L"]) != L or int(kv["tile"]) != tile
                or int(kv["group"]) != group):
            return None
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _summary_fields(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "|" in line:
                k, v = line.split("|", 1)
            elif ":" in line:
                k, v = line.split(":", 1)
            else:
                continue
            kv[k.strip()] = v.strip()
    return kv


def measured_valu(kernel, L, tile, group, launch_us):
    """VALU use of one launch from the committed SQ counter summary: the
    fraction of the SIMDs' issue cycles that issued VALU instructions and the
    fraction of all VALU lanes kept busy, over the launch duration given
    (the live HIP-event average).  None when the summary is missing or was
    taken with other kernel sources or another launch configuration."""
    path = COUNTER_PROFILES.get(kernel)
    if path is None or not os.path.exists(path):
        return None
    kv = _summary_fields(path)
    try:
        if (kv["source_hash"] != kernel_source_hash() or int(kv["L"]) != L or int(kv["tile"]) != tile
                or int(kv["group"]) != group):
            return None
        insts = float(kv["SQ_INSTS_VALU"])
        lane_cycles = float(kv["SQ_THREAD_CYCLES_VALU"])
    except (KeyError, ValueError):
        return None
    cycles = launch_us * 1e-6 * GPU_CLOCK_HZ
    return {"source": os.path.relpath(path, ROOT), "valu_insts_per_launch": insts,
            "active_lanes_per_inst": lane_cycles / insts,
            "issue_frac": insts * 4.0 / (N_SIMDS * cycles),
            "lane_frac": lane_cycles / (N_SIMDS * 16.0 * cycles),
            "definition": "issue_frac = SQ_INSTS_VALU x 4 cycles (wave64 on a 16-lane SIMD) / (1024 SIMDs x "
                          "launch cycles at 2.4 GHz); lane_frac = SQ_THREAD_CYCLES_VALU / (1024 SIMDs x 16 "
                          "lanes x launch cycles): the kernel's share of the chip's full-rate VALU lane-ops"}


# Algorithmic HBM bytes per site update: the state is read and written once
# per sweep; bit-packed = 2 bits, int8 = 2 bytes.
BYTES_PER_UPDATE = {"bits": 0.25, "int8": 2.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sim(pgg, L, r, seed, kernel, layout, stream, tile=0, group=0):
    """The lattice of the timed passes; kernel "tiled" is the double-tiling
    schedule (its own kernel), every other name a kernel of the 16-colour
    sweep."""
    if kernel == "tiled":
        return pgg.Sim(L, r, wl.K_PAPER, 0.5, seed, layout, "auto", stream=stream, schedule="tiled")
    return pgg.Sim(L, r, wl.K_PAPER, 0.5, seed, layout, kernel, stream=stream, tile=tile, group=group)


def time_sweeps(pgg, torch, L, r, seed, kernel, layout, warmup, steps, stream, tile=0, group=0):
    """Wall time of `steps` sweeps after `warmup`, and the HIP-event time of
    the same region recorded on the stream the sweep kernels run on."""
    sim = make_sim(pgg, L, r, seed, kernel, layout, stream, tile, group)
    sim.sweep(warmup, want_counts=False)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.sweep(steps, want_counts=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    nc = sim.coop_count()
    sim.close()
    return dt, nc, ev_ms


def kernel_pass(pgg, torch, L, r, seed, kernel, layout, warmup, steps, stream, tile=0, group=0):
    """Same trajectory with every sweep-kernel launch bracketed by events."""
    sim = make_sim(pgg, L, r, seed, kernel, layout, stream, tile, group)
    sim.sweep(warmup, want_counts=False)
    sim.set_kernel_timing(True)
    sim.sweep(steps, want_counts=False)
    launches, ms, drawn = sim.kernel_timing()
    span_n, span_us = sim.kernel_span()
    sim.close()
    return launches, ms, drawn, (span_us / span_n if span_n else None)


# The batched pass's settings when it is not autotuned: what
# pgg_ensemble_autotune chose for this workload (whole rows for every size,
# chunk 32, 4 waves per workgroup, two concurrent groups, the L <= 256
# replicas resident on 4 waves).
ENSEMBLE_TUNE = dict(chunk=32, waves_per_group=4, branches=2, resident_max_L=256, resident_waves=4)


def ensemble_pass(pgg, torch, sweeps, chunk, plain_per_size, stream, autotune):
    """Batched ensemble (all replicas, one graph replay per chunk) vs the same
    replicas run one lattice at a time (a sample of each size, scaled).  The
    settings are ENSEMBLE_TUNE, or with autotune (and chunk 0) those of
    pgg_ensemble_autotune (untimed, before the timed run)."""
    reps = wl.ensemble_replicas(sweeps=sweeps)
    total = float(sum(rp["L"] ** 2 for rp in reps)) * sweeps
    tune = dict(ENSEMBLE_TUNE, chunk=chunk) if chunk else dict(ENSEMBLE_TUNE)
    chunk = tune["chunk"]
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        tune, ms = pgg.ensemble_autotune(reps, probe_sweeps=8, stream=stream)
        tuned = {"tiles_by_L": {int(rp["L"]): int(w) for rp, w in zip(reps, tune["tiles"])},
                 **{k: tune[k] for k in pgg.TUNE_KEYS}, "probe_ms_per_sweep": ms,
                 "tuning_s": time.perf_counter() - t0}
        chunk = tune["chunk"]
    ens = pgg.Ensemble(reps, stream=stream, **tune)
    ens.sweep(min(chunk, sweeps), want_counts=False)  # first replay builds the graph
    torch.cuda.synchronize()
    ens.close()
    ens = pgg.Ensemble(reps, stream=stream, **tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.sweep(sweeps, want_counts=False)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    nc = ens.coop_counts()
    by_size = {}
    for k, rp in enumerate(reps):
        by_size.setdefault(rp["L"], []).append(k)
    # The plain baseline times a sample of each size alone and checks that
    # each ends exactly where its replica in the batched run ended: the same
    # cooperator count and the same lattice.
    t_plain = 0.0
    checked, mismatched = 0, []
    for L, ks in sorted(by_size.items()):
        sample = ks[::max(1, len(ks) // plain_per_size)][:plain_per_size]
        ts = []
        for k in sample:
            rp = reps[k]
            sim = pgg.Sim(rp["L"], rp["r"], rp["K"], rp["p0"], rp["seed"], "bits", "auto", stream=stream)
            sim.sweep(2, want_counts=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.sweep(sweeps - 2, want_counts=False)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * sweeps / (sweeps - 2))
            same = sim.coop_count() == int(nc[k]) and bool((sim.read_lattice() == ens.read_lattice(k)).all())
            checked += 1
            if not same:
                mismatched.append(k)
            sim.close()
        t_plain += sum(ts) / len(ts) * len(ks)
    ens.close()
    identical = not mismatched
    return {"metric": "replica-site updates/s", "value": total / t_batched, "plain_value": total / t_plain,
            "ratio_vs_plain": t_plain / t_batched if identical else None,
            "identical_to_plain": identical, "plain_checked": checked, "plain_mismatched": mismatched, "replicas": len(reps), "sweeps": sweeps,
            "sizes": sorted(by_size), "chunk": chunk, "settings": {k: tune[k] for k in pgg.TUNE_KEYS},
            "autotuned": tuned, "batched_s": t_batched, "plain_s_estimated": t_plain,
            "plain": "each replica alone (pgg_init/pgg_sweep, automatic kernel), %d per size timed, "
                     "scaled to the %d replicas of each size; each sampled replica's final count and lattice "
                     "compared with its batched run" % (plain_per_size, len(reps) // len(by_size)),
            "mean_final_density": float(sum(int(v) / reps[k]["L"] ** 2 for k, v in enumerate(nc)) / len(reps))}


def late_window(pgg, torch, L, r, seed, kernel, layout, t_start, steps, stream, tile=0, group=0):
    """The same lattice later in its decay: sweeps t_start .. t_start+steps-1
    timed; then the same sweeps again from the lattice saved at t_start, in
    timing mode, for the fraction of updates that draw random numbers and
    the launches' own spans."""
    sim = make_sim(pgg, L, r, seed, kernel, layout, stream, tile, group)
    sim.sweep(t_start, want_counts=False)
    start = sim.read_lattice()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(steps, want_counts=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rho = sim.density()
    sim.write_lattice(start, t_start)
    sim.set_kernel_timing(True)
    sim.sweep(steps, want_counts=False)
    launches, _, drawn = sim.kernel_timing()
    span_n, span_us = sim.kernel_span()
    same = sim.density() == rho
    sim.close()
    return {"t_start": t_start, "steps": steps, "value": float(L) * L * steps / dt, "unit": "site updates/s",
            "ms_per_step": 1e3 * dt / steps, "density_at_end": rho,
            "drawn_fraction": drawn / (float(L) * L * steps),
            "kernel_span_us": span_us / span_n if span_n else None,
            "replay_matches": bool(same)}


def decay_batch_pass(pgg, torch, warmup, steps, stream):
    """The decay runs (L = 4096, r_c and r_c +- 0.005, three seeds each) as
    one ensemble: sweeps warmup .. warmup + steps - 1 of all nine lattices,
    timed like the single-lattice pass."""
    cfg = wl.DECAY
    reps = [dict(L=cfg["L"], r=r, K=cfg["K"], p0=cfg["p0"], seed=s) for r in cfg["r_values"] for s in cfg["seeds"]]
    ens = pgg.Ensemble(reps, chunk=64, stream=stream)
    ens.sweep(warmup, want_counts=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.sweep(steps, want_counts=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ens.close()
    total = len(reps) * float(cfg["L"]) ** 2 * steps
    return {"replicas": len(reps), "L": cfg["L"], "r_values": list(cfg["r_values"]), "seeds": list(cfg["seeds"]),
            "sweeps_timed": "%d..%d" % (warmup, warmup + steps - 1), "value": total / dt,
            "unit": "replica-site updates/s", "ms_per_sweep_of_all": 1e3 * dt / steps}


# The paper's own timing of its graphics-card code (Sec. V prose, Fig. 5 workload):
# 10^6 Monte Carlo steps of the double tiling at L = 4096, r = 3.98, K = 0.5 in
# "less than an hour and a half" on a GeForce GTX 1080, i.e. at least
# 4096^2 * 10^6 / 5400 s site updates/s; the serial CPU code took nearly a month.
PAPER_GPU_UPDATES_PER_S = 4096.0 ** 2 * 1e6 / 5400.0
PAPER_CPU_UPDATES_PER_S = 4096.0 ** 2 * 1e6 / (30 * 86400.0)


def paper_workload_pass(pgg, torch, warmup, steps, stream):
    """The paper's benchmark workload with the paper's own dynamics: the
    double tiling at L = 4096, r = 3.98, K = 0.5 from a 50/50 start."""
    L, r = 4096, 3.98
    sim = pgg.Sim(L, r, wl.K_PAPER, 0.5, 1, "bits", "auto", stream=stream, schedule="tiled")
    sim.sweep(warmup, want_counts=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(steps, want_counts=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rho = sim.density()
    sim.close()
    value = float(L) * L * steps / dt
    return {"schedule": "tiled (Sec. IV double tiling)", "L": L, "r": r, "steps": steps,
            "value": value, "unit": "site updates/s", "ms_per_step": 1e3 * dt / steps, "density_at_end": rho,
            "paper_gtx1080_updates_per_s": PAPER_GPU_UPDATES_PER_S,
            "paper_xeon_updates_per_s": PAPER_CPU_UPDATES_PER_S,
            "ratio_vs_paper_gpu": value / PAPER_GPU_UPDATES_PER_S,
            "note": "context, not a target: the paper's numbers are derived from its prose (10^6 steps at "
                    "L = 4096 in under 1.5 h on a GTX 1080, nearly a month on a 2.8 GHz Xeon) and were "
                    "measured on other hardware"}


def pairwise_pass(pgg, torch, warmup, steps, stream, L=4096, b=1.05, K=0.1):
    """The pairwise prisoner's dilemma (the game Sec. VI names next; temptation
    b, noise K) on one L x L lattice: its 8-colour sweep, timed like the
    single-lattice pass over sweeps warmup .. warmup + steps - 1 (the caller
    keeps them before the lattice dies out)."""
    sim = pgg.Sim(L, b, K, 0.5, 1, "bits", stream=stream, game="pd")
    sim.sweep(warmup, want_counts=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(steps, want_counts=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rho = sim.density()
    sim.close()
    return {"game": "pairwise prisoner's dilemma (R = 1, T = b, S = P = 0)", "L": L, "b": b, "K": K,
            "sweeps_timed": "%d..%d" % (warmup, warmup + steps - 1), "value": float(L) * L * steps / dt,
            "unit": "site updates/s", "ms_per_step": 1e3 * dt / steps, "density_at_end": rho}


def serving_pass(pgg, n_jobs, stream, budget_mib=256, chunk=16, max_resident=256):
    """Poisson arrivals of simulation jobs through the C job server at 70 %
    of its capacity.  The capacity is measured first: 4 x max_resident jobs
    of the same distribution submitted at once, at most max_resident of them
    on the device, and the rate over the steps that began with jobs still
    queued (the server saturated, before the batch drains)."""
    from paper_1704_08098_amd import server

    def run(jobs):
        engine = pgg.ServerEngine(budget_mib << 20, max_L=2048, max_resident=max_resident, chunk=chunk,
                                  stream=stream)
        try:
            rep = server.serve(engine, jobs)
        finally:
            engine.close()
        rep.pop("engine", None)
        return rep

    calib_jobs = 4 * max_resident
    cal = server.capacity(pgg, calib_jobs, max_resident, chunk, budget_mib, master_seed=11, stream=stream)
    capacity = cal["site_updates_per_s_saturated"]
    probe = wl.serving_trace(n_jobs, 1.0)
    mean_work = sum(float(j["L"]) ** 2 * j["sweeps"] for j in probe) / n_jobs
    rate = 0.7 * capacity / mean_work
    rep = run(wl.serving_trace(n_jobs, rate))
    rep.update({"arrival_rate_per_s": rate, "offered_load": 0.7, "capacity_site_updates_per_s": capacity,
                "capacity_basis": "%d jobs of the same distribution submitted at once, at most %d resident: the "
                                  "rate over the %.2f s of steps that began with jobs still queued (the whole "
                                  "batch, drain included: %.3g)" % (calib_jobs, max_resident, cal["saturated_s"],
                                                                    cal["site_updates_per_s"]),
                "hbm_budget_MiB": budget_mib, "chunk": chunk, "max_resident": max_resident,
                "trace": "Poisson arrivals; L log-uniform in [64, 2048] (multiples of 4), r ~ U[3.5, 5.6], "
                         "MCS ~ U{1000..10000}, p0 ~ U[0.1, 0.9], seed 7"})
    return rep


def scan_pass(pgg, torch, sweeps, stream):
    """The r scan near the transition (21 values of r in [3.70, 3.80], L =
    1024, one seed each) as one ensemble: the stationary cooperator density
    per r (mean over the last half of the sweeps, Eq. (4)) and the rate."""
    from paper_1704_08098_amd import observables as ob
    cfg = dict(wl.SCAN, sweeps=sweeps, average_last=max(1, min(wl.SCAN["average_last"], sweeps // 2)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, rho, _ = ob.r_scan(pgg, cfg, stream=stream)
    dt = time.perf_counter() - t0
    n_rep = len(cfg["r_values"])
    return {"L": cfg["L"], "sweeps": sweeps, "average_last": cfg["average_last"], "r": [float(v) for v in r],
            "stationary_density": [float(v) for v in rho], "seconds": dt,
            "replica_site_updates_per_s": n_rep * float(cfg["L"]) ** 2 * sweeps / dt,
            "note": "one batched ensemble; wall time includes the per-block count copies"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(L, r, seed, n_sweeps, repeats=3):
    """The oracle, single-threaded: the median of `repeats` runs of n_sweeps
    sweeps of the benchmark lattice from its initial state (the headline
    workload's own rate), and of the small configuration in full (L = 100,
    r = 3.8, 1000 sweeps, seed 1)."""
    import oracle
    oracle.build(force=False)
    s, _ = oracle.init(L, 0.5, seed)
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.sweep(s, r, wl.K_PAPER, seed, 0, n_sweeps)
        ts.append(time.perf_counter() - t0)
    dt = sorted(ts)[len(ts) // 2]
    small = wl.SMALL
    ts_small = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.run(small["L"], small["r"], small["K"], small["p0"], small["seeds"][0], small["sweeps"])
        ts_small.append(time.perf_counter() - t0)
    dts = sorted(ts_small)[len(ts_small) // 2]
    return {"value": L * L * n_sweeps / dt, "unit": "site updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cores": os.cpu_count(),
            "sample": "median of %d runs of %d sweep(s) of the L=%d, r=%g lattice from its i.i.d. 50/50 start "
                      "(16-colour oracle, single thread, %.1f s each)" % (repeats, n_sweeps, L, r, dt),
            "runs_s": ts,
            "small_config": {"value": small["L"] ** 2 * small["sweeps"] / dts, "unit": "site updates/s",
                             "workload": "L=%d, r=%g, %d sweeps, seed %d, init included (in full)" % (
                                 small["L"], small["r"], small["sweeps"], small["seeds"][0]),
                             "median_s": dts, "runs_s": ts_small}}


def _oracle_replica(args):
    import oracle
    L, r, seed, n = args
    s, _ = oracle.init(L, 0.5, seed)
    oracle.sweep(s, r, wl.K_PAPER, seed, 0, n)
    return L * L * n


def cpu_ensemble_baseline(n_sweeps=3, max_procs=16):
    """Ensemble context: the oracle on the host's cores, one replica of the
    batched ensemble's L = 1024 size per process (a bounded sample), as an
    aggregate replica-site update rate."""
    from concurrent.futures import ProcessPoolExecutor
    import oracle
    oracle.build(force=False)
    procs = max(1, min(max_procs, os.cpu_count() or 1))
    reps = [rp for rp in wl.ensemble_replicas() if rp["L"] == 1024][:procs]
    args = [(rp["L"], rp["r"], rp["seed"], n_sweeps) for rp in reps]
    with ProcessPoolExecutor(max_workers=procs) as ex:
        list(ex.map(_oracle_replica, [(64, 3.8, 1, 1)] * procs))  # start the workers untimed
        t0 = time.perf_counter()
        total = sum(ex.map(_oracle_replica, args))
        dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "replica-site updates/s", "cores": procs, "kind": "oracle",
            "sample": "%d L=1024 replicas of the batched ensemble, %d sweep(s) each, one process per core "
                      "(%.1f s)" % (len(args), n_sweeps, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=20, help="untimed sweeps before them")
    ap.add_argument("--L", type=int, default=wl.DECAY["L"])
    ap.add_argument("--r", type=float, default=wl.R_CRITICAL)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--kernel", default="segment_pair",
                    choices=["segment", "segment_pair", "resident", "strip", "rowband_staged", "rowband_compact",
                             "rowband", "colour", "tiled"],
                    help="sweep kernel of the 16-colour schedule, or 'tiled': the double-tiling schedule of "
                         "Sec. IV (a different dynamics)")
    ap.add_argument("--layout", default="auto", choices=["auto", "int8", "bits"],
                    help="lattice storage (auto: int8 for the colour kernel, else bits); the segment kernels "
                         "run an int8 lattice through a bit-packed working copy")
    ap.add_argument("--tile", type=int, default=0, help="segment width / strip height / rows per band (0 = auto)")
    ap.add_argument("--group", type=int, default=0, help="segment kernel: waves per workgroup (0 = 4)")
    ap.add_argument("--dense-steps", type=int, default=200)
    ap.add_argument("--cpu-sweeps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ensemble-sweeps", type=int, default=5000, help="0 skips the ensemble pass")
    ap.add_argument("--ensemble-chunk", type=int, default=0, help="sweeps per graph replay of the batched pass "
                    "(0 = that of ENSEMBLE_TUNE)")
    ap.add_argument("--plain-per-size", type=int, default=4)
    ap.add_argument("--late-start", type=int, default=10_000, help="first sweep of the late window (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=300, help="jobs in the serving pass (0 skips it)")
    ap.add_argument("--serve-chunk", type=int, default=16, help="sweeps per server step")
    ap.add_argument("--serve-resident", type=int, default=256, help="most jobs on the device at once")
    ap.add_argument("--no-paper-workload", dest="paper_workload", action="store_false",
                    help="skip the paper's own workload (double tiling, L = 4096, r = 3.98)")
    ap.add_argument("--no-pairwise", dest="pairwise", action="store_false",
                    help="skip the pairwise prisoner's dilemma pass (L = 4096, b = 1.05, K = 0.1)")
    ap.add_argument("--no-decay-batch", dest="decay_batch", action="store_false",
                    help="skip the nine L = 4096 decay lattices run as one ensemble")
    ap.add_argument("--scan-sweeps", type=int, default=10_000,
                    help="sweeps of the L = 1024 r scan run as one ensemble (0 skips it)")
    ap.add_argument("--autotune", action="store_true", help="ensemble pass with the settings of "
                    "pgg_ensemble_autotune instead of ENSEMBLE_TUNE")
    ap.add_argument("--source-hash", action="store_true", help="print the segment kernel's source hash and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the sweep of one lattice is not split across "
              "GPUs here; got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_08098_amd import pgg
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    pgg.load()
    layout = args.layout if args.layout != "auto" else ("int8" if args.kernel == "colour" else "bits")
    stream = torch.cuda.Stream()
    L, r, seed = args.L, args.r, args.seed

    if args.copy_probe:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    log("timed pass: L=%d r=%g kernel=%s warmup=%d steps=%d" % (L, r, args.kernel, args.warmup, args.steps))
    dt, nc_end, region_ms = time_sweeps(pgg, torch, L, r, seed, args.kernel, layout, args.warmup, args.steps,
                                        stream, args.tile, args.group)
    updates = float(L) * L * args.steps
    value = updates / dt

    dense = None
    if args.kernel in ("segment", "segment_pair", "strip", "rowband_compact", "rowband_staged") and args.dense_steps > 0:
        log("dense pass: %d sweeps" % args.dense_steps)
        ddt, _, _ = time_sweeps(pgg, torch, L, r, seed, "rowband", "bits", args.warmup,
                                args.dense_steps, stream)
        dense = {"value": float(L) * L * args.dense_steps / ddt, "unit": "site updates/s",
                 "kernel": "rowband (every site draws)", "steps": args.dense_steps,
                 "ms_per_step": 1e3 * ddt / args.dense_steps}

    log("kernel-timing pass")
    launches, kms, drawn, span_us = kernel_pass(pgg, torch, L, r, seed, args.kernel, layout, args.warmup,
                                                args.steps, stream, args.tile, args.group)
    # Average launch duration: the event-timed region of the timed pass over
    # its launches (same trajectory, same launches as the kernel-timing pass).
    # It includes the gaps between launches and the per-chunk bookkeeping
    # kernels, so it bounds the kernel's own duration from above.  The
    # kernel-timing pass also reports each launch's own span (device wall
    # clock, first workgroup start to last workgroup end).
    avg_ms = region_ms / max(launches, 1)
    sites_per_launch = updates / max(launches, 1)  # the strip kernel: one launch per timed call
    if args.kernel in ("colour", "tiled"):
        drawn = updates
    # the segment and resident kernels sweep a bit-packed lattice whatever the layout
    hbm_bytes = BYTES_PER_UPDATE["bits" if args.kernel in ("segment", "segment_pair", "resident") else layout]
    alg_bytes_per_launch = hbm_bytes * sites_per_launch
    achieved_gbs = alg_bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernel_name = {"segment": "k_ens_segment", "segment_pair": "k_ens_pair", "strip": "k_strip",
                   "rowband_staged": "k_rowband_staged", "rowband_compact": "k_rowband_bits<true>",
                   "rowband": "k_rowband_bits<false>", "colour": "k_colour_int8", "tiled": "k_tiled_part",
                   "resident": "k_resident"}[args.kernel]
    # the work split the sweep actually ran (the library's choice when
    # --tile is 0): the committed counter summaries are matched on it
    if args.kernel == "tiled":
        split = 0  # the double tiling has no work split to choose
    else:
        _, split = pgg.pgg_plan(pgg.make_params(L, r, 0.5, 0.5, seed, layout, args.kernel, args.tile, args.group))
    traffic = measured_traffic(args.kernel, L, split, args.group)
    roofline = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_over_algorithmic": traffic / alg_bytes_per_launch if traffic else None,
                "kernel": kernel_name,
                "algorithmic_bytes_per_launch": alg_bytes_per_launch,
                "bytes_per_update": hbm_bytes,
                "sites_per_launch": sites_per_launch,
                "avg_launch_us": avg_ms * 1e3, "launches": launches,
                "avg_launch_source": "HIP events around the timed region on the sweep stream / launches",
                "timing_pass_event_us_per_launch": kms / max(launches, 1) * 1e3,
                "kernel_span_us": span_us,
                "drawn_fraction": drawn / updates,
                "frac_int8_equivalent": achieved_gbs * 2.0 / hbm_bytes / HBM_PEAK_GBS,
                "valu": measured_valu(args.kernel, L, split, args.group, avg_ms * 1e3),
                "note": "the state is read and written once per sweep (2 bits per site update on the bit-packed "
                        "lattice); the path is bound by integer VALU issue (one Philox4x32-10 per drawn update), "
                        "not by HBM -- 'valu' gives the counter-measured share of the VALU lanes"}
    windows = {"early": {"sweeps": "%d..%d" % (args.warmup, args.warmup + args.steps - 1), "value": value,
                         "ms_per_step": 1e3 * dt / args.steps, "drawn_fraction": drawn / updates}}

    batched = None
    if args.ensemble_sweeps > 0:
        log("ensemble pass: %d sweeps" % args.ensemble_sweeps)
        batched = ensemble_pass(pgg, torch, args.ensemble_sweeps, args.ensemble_chunk, args.plain_per_size, stream,
                                args.autotune)

    paper_workload = None
    if args.paper_workload:
        log("paper workload: double tiling, L=4096, r=3.98")
        paper_workload = paper_workload_pass(pgg, torch, args.warmup, args.steps, stream)

    pairwise = None
    if args.pairwise:
        log("pairwise prisoner's dilemma: L=4096")
        # sweeps 5..24: at b = 1.05 the lattice has reached the all-D
        # absorbing state by sweep 1020, after which no site draws
        pairwise = pairwise_pass(pgg, torch, 5, 20, stream)

    decay_batch = None
    if args.decay_batch:
        log("decay batch: 9 lattices of L=%d as one ensemble" % wl.DECAY["L"])
        decay_batch = decay_batch_pass(pgg, torch, args.warmup, args.steps, stream)

    late = None
    if args.late_start > 0:
        log("late window: sweeps %d..%d" % (args.late_start, args.late_start + args.steps - 1))
        late = late_window(pgg, torch, L, r, seed, args.kernel, layout, args.late_start, args.steps, stream,
                           args.tile, args.group)
        windows["late"] = {"sweeps": "%d..%d" % (args.late_start, args.late_start + args.steps - 1),
                           "value": late["value"], "ms_per_step": late["ms_per_step"],
                           "drawn_fraction": late["drawn_fraction"]}

    serving = None
    if args.serve_jobs > 0:
        log("serving pass: capacity batch, then %d jobs" % args.serve_jobs)
        serving = serving_pass(pgg, args.serve_jobs, stream, chunk=args.serve_chunk, max_resident=args.serve_resident)

    scan = None
    if args.scan_sweeps > 0:
        log("r scan: 21 replicas of L=%d, %d sweeps" % (wl.SCAN["L"], args.scan_sweeps))
        scan = scan_pass(pgg, torch, args.scan_sweeps, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle, %d sweep(s) at L=%d" % (args.cpu_sweeps, L))
        cpu = cpu_baseline(L, r, seed, args.cpu_sweeps)
        if batched is not None:
            log("cpu ensemble baseline: oracle on the host cores")
            batched["cpu_baseline_all_cores"] = cpu_ensemble_baseline()

    line = {
        "metric": METRIC, "value": value, "unit": "site updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "single %dx%d periodic lattice, r=%g, K=0.5, i.i.d. 50/50 start "
                               "(seed %d), sweeps %d..%d timed" % (L, L, r, seed, args.warmup,
                                                                 args.warmup + args.steps - 1),
                   "L": L, "r": r, "K": wl.K_PAPER, "p0": 0.5, "seed": seed, "layout": layout,
                   "kernel": args.kernel, "tile": args.tile, "work_split": split, "group": args.group,
                   "parallelism": "single GPU"},
        "roofline": roofline, "windows": windows, "dense": dense, "late": late, "batched": batched, "serving": serving,
        "scan": scan, "decay_batch": decay_batch, "paper_workload": paper_workload, "pairwise": pairwise,
        "cpu_baseline": cpu,
        "final_density": nc_end / float(L * L),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

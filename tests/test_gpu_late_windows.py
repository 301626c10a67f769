"""GPU: segmented parity of the long runs -- late windows the stored
trajectories do not reach, checked against the oracle from GPU states.

A run of the HIP path is stopped at sweep t, its lattice read out, and the
oracle advances that lattice; the GPU's next sweeps must equal the oracle's
bit for bit.  A window of n sweeps is cut into segments that the oracle runs
in parallel host processes, each starting from the GPU lattice at the
segment's start: since every segment starts from a lattice already shown
equal to the previous segment's oracle result, the chain covers every sweep
of the window.  The run that is compared end to end is the one in the
launch configuration the benchmark times; a second run of the same
trajectory supplies the lattices at the segment boundaries.
"""
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from paper_1704_08098_amd import workloads as wl

pytestmark = pytest.mark.gpu

MAX_PROCS = 10  # oracle processes at once (the host's share of cores)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pgg(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.set_device(0)
    from paper_1704_08098_amd import pgg as mod
    mod.load()
    return mod


def _oracle_segment(args):
    """Oracle A: n sweeps of lattice s from sweep index t0 -> (lattice, counts)."""
    import oracle
    s, r, K, seed, t0, n = args
    return oracle.sweep(s, r, K, seed, t0, n)


def _check_chain(starts, ends_counts, final_lattice, r, K, seed):
    """starts: [(t_k, GPU lattice at t_k)] for consecutive segments; the
    GPU's counts over the whole window and its lattice at the window's end.
    Runs the oracle segments in parallel and compares."""
    tasks = []
    for k, (t, s) in enumerate(starts):
        t_next = starts[k + 1][0] if k + 1 < len(starts) else starts[0][0] + len(ends_counts)
        tasks.append((s, r, K, seed, t, t_next - t))
    with ProcessPoolExecutor(max_workers=min(MAX_PROCS, len(tasks))) as ex:
        res = list(ex.map(_oracle_segment, tasks))
    got_counts = np.concatenate([c for _, c in res])
    bad = np.flatnonzero(got_counts != ends_counts)
    assert bad.size == 0, "first differing sweep t = %d" % (starts[0][0] + 1 + bad[0])
    for k in range(len(res) - 1):
        assert np.array_equal(res[k][0], starts[k + 1][1]), "segment %d ends elsewhere than the GPU" % k
    assert np.array_equal(res[-1][0], final_lattice), "last segment ends elsewhere than the GPU"


def test_benchmark_lattice_late_window(pgg):
    """The benchmark lattice (L = 4096, r = r_c, seed 1) as bench.py's late
    window runs it -- the paired kernel on a side stream, one call of 10^4
    sweeps, then one of 20 -- equals the oracle over sweeps 10^4 .. 10^4+19."""
    import torch
    L, r, K, p0, seed, t0, n, seg = 4096, wl.R_CRITICAL, wl.K_PAPER, 0.5, 1, 10_000, 20, 5
    stream = torch.cuda.Stream()
    say("late window L", L, "t", t0, "..", t0 + n, "(bench configuration)")
    with pgg.Sim(L, r, K, p0, seed, "bits", "segment_pair", stream=stream) as sim:
        sim.sweep(t0, want_counts=False)
        start = sim.read_lattice()
        counts = sim.sweep(n)
        final = sim.read_lattice()
    say("late window: segment boundaries from a second run")
    starts = [(t0, start)]
    with pgg.Sim(L, r, K, p0, seed, "bits", "segment_pair", stream=stream) as sim:
        sim.sweep(t0 + seg, want_counts=False)
        for t in range(t0 + seg, t0 + n, seg):
            starts.append((t, sim.read_lattice()))
            sim.sweep(seg, want_counts=False)
        assert np.array_equal(sim.read_lattice(), final)
    assert np.array_equal(starts[0][1], start)
    say("late window: oracle over", len(starts), "segments")
    _check_chain(starts, counts, final, r, K, seed)


def test_decay_run_windows_up_to_1e5_sweeps(pgg):
    """A decay run (L = 4096, r = r_c + 0.005, seed 3) through 10^5 sweeps, the
    length of the decay runs: windows of 5 sweeps from t = 10^4, 5 x 10^4 and
    10^5 - 5 equal the oracle from the GPU lattice at each window's start."""
    import torch
    L, r, K, p0, seed = 4096, wl.DECAY["r_values"][2], wl.K_PAPER, 0.5, 3
    marks, w = (10_000, 50_000, 99_995), 5
    stream = torch.cuda.Stream()
    tasks, gpu = [], []
    with pgg.Sim(L, r, K, p0, seed, "bits", "auto", stream=stream) as sim:
        for m in marks:
            say("decay run L", L, "r", r, "to t", m)
            sim.sweep(m - sim.t, want_counts=False)
            s = sim.read_lattice()
            c = sim.sweep(w)
            gpu.append((c, sim.read_lattice()))
            tasks.append((s, r, K, seed, m, w))
        assert sim.t == 100_000
    say("decay run: oracle windows")
    with ProcessPoolExecutor(max_workers=len(tasks)) as ex:
        res = list(ex.map(_oracle_segment, tasks))
    for m, (ref_s, ref_c), (c, s) in zip(marks, res, gpu):
        assert np.array_equal(c, ref_c), "counts differ in the window from t = %d" % m
        assert np.array_equal(s, ref_s), "lattice differs after the window from t = %d" % m


def test_scan_last_500_sweeps(pgg):
    """The L = 1024 r scan as one 21-replica ensemble (chunks of 64, as the
    scan runs) through 10^4 sweeps: for r = 3.745 (near this dynamics' own
    transition) and r = 3.8, the last 500 sweeps equal the oracle, cut into
    10 segments of 50 from the GPU lattices at t = 9500, 9550, ..."""
    cfg = wl.SCAN
    reps = [dict(L=cfg["L"], r=r, K=cfg["K"], p0=cfg["p0"], seed=s) for r, s in zip(cfg["r_values"], cfg["seeds"])]
    picks = [cfg["r_values"].index(3.745), cfg["r_values"].index(3.8)]
    t_last, seg = cfg["sweeps"] - 500, 50
    starts = {k: [] for k in picks}
    say("scan ensemble, 21 replicas of L", cfg["L"], "to t", t_last)
    with pgg.Ensemble(reps, chunk=64) as ens:
        for _ in range(t_last // 500):
            ens.sweep(500, want_counts=False)
        parts = []
        while ens.t < cfg["sweeps"]:
            for k in picks:
                starts[k].append((ens.t, ens.read_lattice(k)))
            parts.append(ens.sweep(seg))
        counts = np.concatenate(parts, axis=1)
        finals = {k: ens.read_lattice(k) for k in picks}
    for k in picks:
        say("scan replica r", reps[k]["r"], ": oracle over", len(starts[k]), "segments")
        _check_chain(starts[k], counts[k], finals[k], reps[k]["r"], reps[k]["K"], reps[k]["seed"])

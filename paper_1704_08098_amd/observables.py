"""Host-side observables of the cooperator count (Sec. III, Eq. (4)) and the
two experiments that use them (Sec. V).

The device returns N_C(t), the number of cooperators after every sweep t
(integer, exact).  From it:

* the density rho_C(t) = N_C(t) / L^2;
* the stationary density: the time average of rho_C over the last sweeps of
  a run, after a relaxation the paper leaves to the reader (here: the mean
  over sweeps t_max - n + 1 .. t_max, e.g. 5001..10000 of a 10^4-sweep run);
* the density on a logarithmic time grid, for the decay of rho_C at and
  near the critical r of the C+D -> D transition (Fig. 4).

``r_scan`` runs the replicas of an r scan as one batched ensemble and returns
the stationary density per r; ``decay`` runs one lattice and records rho_C on
a log grid.  Both only marshal calls to the C library (``pgg``); all
arithmetic here is the host-side averaging of exact integer counts.
"""
from __future__ import annotations

import numpy as np

from . import workloads as wl


def density_series(counts, L: int) -> np.ndarray:
    """rho_C(t) = N_C(t) / L^2 for an array of counts (any shape)."""
    return np.asarray(counts, dtype=np.float64) / float(L * L)


def stationary_density(counts, L: int, average_last: int) -> float:
    """Mean of N_C(t) / L^2 over the last `average_last` entries of the
    per-sweep counts of one run (Eq. (4) with its time average).  The sum
    is taken in integers, so the result is the exact mean rounded once."""
    c = np.asarray(counts, dtype=np.uint64)
    if c.ndim != 1 or not 0 < average_last <= c.size:
        raise ValueError("need a 1-D count history with at least average_last entries")
    total = int(c[c.size - average_last:].sum(dtype=np.uint64))
    return total / (float(average_last) * float(L) * float(L))


def sample_on_grid(counts, L: int, grid, nc0: int | None = None) -> np.ndarray:
    """rho_C at the sweep indices of `grid` (t >= 1 reads counts[t - 1], the
    count after sweep t; t = 0 needs nc0, the initial count)."""
    c = np.asarray(counts, dtype=np.uint64)
    g = np.asarray(grid, dtype=np.int64)
    if g.size and (g.min() < 0 or g.max() > c.size):
        raise ValueError("grid reaches beyond the count history")
    out = np.empty(g.size, dtype=np.float64)
    for k, t in enumerate(g):
        if t == 0:
            if nc0 is None:
                raise ValueError("t = 0 needs the initial count")
            out[k] = nc0 / float(L * L)
        else:
            out[k] = float(c[t - 1]) / float(L * L)
    return out


def r_scan(pgg, cfg=wl.SCAN, sweeps: int | None = None, average_last: int | None = None,
           chunk: int = 64, stream=None, block: int = 1000, schedule: str = "colour16", progress=None):
    """Stationary density per r: the scan's replicas (one lattice per r, its
    own seed) advanced together as one ensemble (either schedule).  Counts
    are fetched `block` sweeps at a time; progress(sweeps done), if given,
    is called after each block.  Returns (r values, stationary densities,
    counts of shape (replicas, sweeps))."""
    n = int(sweeps if sweeps is not None else cfg["sweeps"])
    last = int(average_last if average_last is not None else min(cfg["average_last"], n))
    reps = [dict(L=cfg["L"], r=r, K=cfg["K"], p0=cfg["p0"], seed=s, schedule=schedule)
            for r, s in zip(cfg["r_values"], cfg["seeds"])]
    parts = []
    with pgg.Ensemble(reps, chunk=chunk, stream=stream) as ens:
        done = 0
        while done < n:
            m = min(block, n - done)
            parts.append(ens.sweep(m))
            done += m
            if progress is not None:
                progress(done)
    counts = np.concatenate(parts, axis=1)
    rho = np.array([stationary_density(counts[k], cfg["L"], last) for k in range(len(reps))])
    return np.array(cfg["r_values"], dtype=np.float64), rho, counts


def r_scan_lattices(pgg, cfg=wl.SCAN, sweeps: int | None = None, average_last: int | None = None,
                    schedule: str = "colour16", workers: int = 4, block: int = 10_000, progress=None):
    """As r_scan, but one lattice per r through pgg_init / pgg_sweep (any
    schedule):
    `workers` host threads each drive their lattices on a stream of their
    own, so up to that many lattices advance on the device at once.
    progress(r, seed), if given, is called as each lattice finishes.
    Returns (r values, stationary densities, counts)."""
    import threading
    import torch
    n = int(sweeps if sweeps is not None else cfg["sweeps"])
    last = int(average_last if average_last is not None else min(cfg["average_last"], n))
    jobs = list(enumerate(zip(cfg["r_values"], cfg["seeds"])))
    counts = np.zeros((len(jobs), n), dtype=np.uint64)
    errors = []
    lock = threading.Lock()

    def worker():
        stream = torch.cuda.Stream()
        while True:
            with lock:
                if not jobs or errors:
                    return
                k, (r, seed) = jobs.pop(0)
            try:
                with pgg.Sim(cfg["L"], r, cfg["K"], cfg["p0"], seed, "bits", "auto", stream=stream,
                             schedule=schedule) as sim:
                    done = 0
                    while done < n:
                        m = min(block, n - done)
                        counts[k, done:done + m] = sim.sweep(m)
                        done += m
                if progress is not None:
                    progress(r, seed)
            except Exception as exc:  # reported after the join
                with lock:
                    errors.append(exc)
                return

    threads = [threading.Thread(target=worker) for _ in range(max(1, workers))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    rho = np.array([stationary_density(counts[k], cfg["L"], last) for k in range(counts.shape[0])])
    return np.array(cfg["r_values"], dtype=np.float64), rho, counts


def decay(pgg, L: int, r: float, seed: int, t_max: int, per_decade: int = 20, K: float = wl.K_PAPER,
          p0: float = 0.5, stream=None, block: int = 10_000, layout: str = "bits", kernel: str = "auto"):
    """rho_C(t) of one lattice from its i.i.d. start on the log grid of
    workloads.log_time_grid (t = 1 .. t_max).  Returns (grid, rho on it)."""
    grid = wl.log_time_grid(t_max, per_decade)
    grid = grid[grid <= t_max]
    parts = []
    with pgg.Sim(L, r, K, p0, seed, layout, kernel, stream=stream) as sim:
        nc0 = sim.coop_count()
        done = 0
        while done < t_max:
            m = min(block, t_max - done)
            parts.append(sim.sweep(m))
            done += m
    counts = np.concatenate(parts)
    return grid, sample_on_grid(counts, L, grid, nc0)

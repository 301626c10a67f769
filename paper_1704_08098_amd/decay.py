"""Decay of the cooperator density at and near the critical point (Sec. V).

At the critical multiplication factor of the C+D -> D transition, the
cooperator density of a large lattice started from a 50/50 state decays as a
power of time, rho_C(t) ~ t^(-delta); slightly above r_c it bends towards a
stationary value, slightly below it falls off faster.  The paper reports the
stationary exponent beta and r_c, not delta, so the decay exponent measured
here is a measurement, not a parity check (for directed percolation in 2 + 1
dimensions delta is about 0.45; the paper does not print it).

The command runs every (r, seed) pair as one batched ensemble, records
rho_C on the logarithmic time grid of Sec. V's decay runs, and fits the
effective exponent -d log rho / d log t over the later decades:

    python -m paper_1704_08098_amd.decay --schedule tiled --r 3.7393 3.7443 3.7493 --seeds 1 2 3

It prints one JSON object (stdout); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import observables as ob
from . import workloads as wl


def local_exponents(grid, rho, t_lo: float, t_hi: float):
    """Least-squares slope of -log rho against log t over the grid points
    with t_lo <= t <= t_hi and rho > 0, and the slopes over each decade in
    that range (None where fewer than 3 points)."""
    g = np.asarray(grid, dtype=np.float64)
    y = np.asarray(rho, dtype=np.float64)

    def slope(lo, hi):
        sel = (g >= lo) & (g <= hi) & (y > 0)
        if np.count_nonzero(sel) < 3:
            return None
        A = np.stack([np.log(g[sel]), np.ones(np.count_nonzero(sel))], axis=1)
        coef, *_ = np.linalg.lstsq(A, np.log(y[sel]), rcond=None)
        return float(-coef[0])

    decades = []
    lo = t_lo
    while lo < t_hi:
        hi = min(lo * 10.0, t_hi)
        decades.append({"t": [lo, hi], "delta": slope(lo, hi)})
        lo = hi
    return slope(t_lo, t_hi), decades


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, default=wl.DECAY["L"])
    ap.add_argument("--r", type=float, nargs="+", default=list(wl.DECAY["r_values"]))
    ap.add_argument("--seeds", type=int, nargs="+", default=list(wl.DECAY["seeds"]))
    ap.add_argument("--sweeps", type=int, default=wl.DECAY["sweeps"])
    ap.add_argument("--schedule", default="colour16", choices=["colour16", "tiled"])
    ap.add_argument("--per-decade", type=int, default=20, help="log grid points per decade")
    ap.add_argument("--fit-from", type=float, default=100.0, help="first t of the exponent fit")
    ap.add_argument("--block", type=int, default=5000, help="sweeps per count read-out")
    args = ap.parse_args(argv)

    import torch
    from . import pgg
    if not torch.cuda.is_available():
        raise SystemExit("the decay runs need a GPU")
    torch.cuda.set_device(0)
    pgg.load()
    reps = [dict(L=args.L, r=r, K=wl.K_PAPER, p0=0.5, seed=s, schedule=args.schedule)
            for r in args.r for s in args.seeds]
    grid = wl.log_time_grid(args.sweeps, args.per_decade)
    grid = grid[(grid >= 1) & (grid <= args.sweeps)]
    rho = np.zeros((len(reps), grid.size))
    print("decay: %d lattices of L = %d (%s), %d sweeps" % (len(reps), args.L, args.schedule, args.sweeps),
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with pgg.Ensemble(reps, chunk=64) as ens:
        nc0 = ens.coop_counts()
        done = 0
        while done < args.sweeps:
            m = min(args.block, args.sweeps - done)
            c = ens.sweep(m)
            sel = (grid > done) & (grid <= done + m)
            rho[:, sel] = c[:, grid[sel] - done - 1].astype(np.float64) / float(args.L) ** 2
            done += m
            print("%d of %d sweeps, %.0f s" % (done, args.sweeps, time.perf_counter() - t0), file=sys.stderr,
                  flush=True)
    dt = time.perf_counter() - t0
    runs = []
    for r in args.r:
        ks = [k for k, rp in enumerate(reps) if rp["r"] == r]
        mean = rho[ks].mean(axis=0)
        delta, decades = local_exponents(grid, mean, args.fit_from, float(args.sweeps))
        runs.append({"r": r, "seeds": [reps[k]["seed"] for k in ks], "rho0": [int(nc0[k]) / float(args.L) ** 2
                                                                           for k in ks],
                     "rho_mean": [float(v) for v in mean], "rho_by_seed": [[float(v) for v in rho[k]] for k in ks],
                     "delta_fit": delta, "delta_by_decade": decades,
                     "rho_final_by_seed": [float(rho[k, -1]) for k in ks]})
    out = {"schedule": args.schedule, "L": args.L, "K": wl.K_PAPER, "sweeps": args.sweeps,
           "grid": [int(t) for t in grid], "fit_from": args.fit_from, "runs": runs, "seconds": dt,
           "replica_site_updates_per_s": len(reps) * float(args.L) ** 2 * args.sweeps / dt,
           "note": "delta = -d log rho / d log t of the seed-averaged density; parity unpinned (the paper "
                   "prints no decay exponent)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Seeded synthetic workloads (parameters only; none of the method's arithmetic).

The paper's runs are themselves synthetic: random initial lattices with each
player a cooperator with probability 1/2 (Sec. III), K = 0.5, lattice sides
from 32 to 4096 (Sec. V).  These generators fix the concrete parameter sets
used by the tests and the benchmark.  Both the oracle side and the GPU side
take their inputs from here.
"""
from __future__ import annotations

import math

import numpy as np

K_PAPER = 0.5
R_CRITICAL = 3.7443  # Sec. V, Fig. 4: r_c of the C+D -> D transition at K = 0.5

# Plain method, small: L = 100, r = 3.8, 1000 sweeps, five seeds.
SMALL = dict(L=100, r=3.8, K=K_PAPER, p0=0.5, seeds=(1, 2, 3, 4, 5), sweeps=1000)

# Single lattice near the transition: 21 values of r in [3.70, 3.80].
SCAN = dict(L=1024, K=K_PAPER, p0=0.5, sweeps=10_000, average_last=5000,
            r_values=tuple(float("%.3f" % (3.70 + 0.005 * i)) for i in range(21)),
            seeds=tuple(100 + i for i in range(21)))

# Large-lattice decay run: L = 4096 at r_c and r_c +- 0.005.
DECAY = dict(L=4096, K=K_PAPER, p0=0.5, sweeps=100_000,
             r_values=(R_CRITICAL - 0.005, R_CRITICAL, R_CRITICAL + 0.005), seeds=(1, 2, 3))

ENSEMBLE_SIZES = (128, 256, 512, 1024)


def log_time_grid(t_max: int, per_decade: int = 20) -> np.ndarray:
    """unique(round(10^(m/per_decade))) <= t_max, for the decay log."""
    m = np.arange(0, int(per_decade * math.log10(max(t_max, 1))) + 1)
    return np.unique(np.round(10.0 ** (m / per_decade)).astype(np.int64))


def ensemble_replicas(master_seed: int = 2017, per_size: int = 64, sizes=ENSEMBLE_SIZES,
                      r_range=(3.6, 3.9), sweeps: int = 5000):
    """Replicas of uneven L, r and seed: per_size replicas of each L."""
    rng = np.random.default_rng(master_seed)
    reps = []
    for L in sizes:
        for _ in range(per_size):
            reps.append(dict(L=int(L), r=float(rng.uniform(*r_range)), K=K_PAPER, p0=0.5,
                             seed=int(rng.integers(1, 2**63 - 1)), sweeps=int(sweeps)))
    return reps


def serving_trace(n_jobs: int, rate_per_s: float, master_seed: int = 7, L_range=(64, 2048),
                  r_range=(3.5, 5.6), mcs_range=(1000, 10_000), p0_range=(0.1, 0.9)):
    """Poisson arrivals of simulation jobs.

    L is log-uniform in L_range rounded to a multiple of 4, r, p0 uniform,
    the number of sweeps uniform on the integers of mcs_range.
    """
    rng = np.random.default_rng(master_seed)
    t = 0.0
    jobs = []
    for q in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        L = int(4 * round(math.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]))) / 4))
        L = max(L_range[0], min(L_range[1], L))
        jobs.append(dict(id=q, arrival=t, L=L, r=float(rng.uniform(*r_range)), K=K_PAPER,
                         p0=float(rng.uniform(*p0_range)),
                         sweeps=int(rng.integers(mcs_range[0], mcs_range[1] + 1)),
                         seed=int(rng.integers(1, 2**63 - 1))))
    return jobs


def random_lattice(L: int, p: float, seed: int) -> np.ndarray:
    """An arbitrary 0/1 lattice (for write_lattice tests), numpy-seeded."""
    rng = np.random.default_rng(seed)
    return (rng.random((L, L)) < p).astype(np.uint8)

"""Write the stored oracle trajectories that the GPU parity tests compare with.

Every value written here comes from the oracle (oracle A: the 16-colour sweep
of the Sec. III elementary step with the Eq. (3) Fermi rule; oracle C: the
double tiling of Sec. IV; counts as in Eq. (4)); nothing else is called.  Run
from the repository root:

    python tests/golden/make_trajectories.py [--jobs 6] [--only decay|scan|tiled]

Outputs (beside this script):

* trajectory_L4096_r3.7443_seed1.txt -- the single-lattice benchmark workload
  (L = 4096, r = 3.7443, K = 0.5, p0 = 0.5, seed 1) through 1020 sweeps:
  N_C(t) for t = 0..1020 and the SHA-256 of the lattice after 20, 520 and
  1020 sweeps.  About two hours of one core.
* rscan_L1024_1000.txt -- the 21 replicas of the L = 1024 r scan through 1000
  sweeps: per replica N_C(1000), the SHA-256 of N_C(1..1000) and of the final
  lattice.  About an hour of one core, spread over --jobs processes.
* tiled_L4096_r3.98_seed1.txt -- the paper's benchmark workload with the
  double tiling of Sec. IV (oracle C): L = 4096, r = 3.98, K = 0.5, p0 = 0.5,
  seed 1 through 1020 steps, in the format of the first file.

Lattice digests are over the L*L bytes (0 or 1, row-major); count digests
over the counts as little-endian uint64.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1704_08098_amd import workloads as wl  # noqa: E402

DECAY_FILE = os.path.join(HERE, "trajectory_L4096_r3.7443_seed1.txt")
TILED_FILE = os.path.join(HERE, "tiled_L4096_r3.98_seed1.txt")
SCAN_FILE = os.path.join(HERE, "rscan_L1024_1000.txt")
DECAY_MARKS = (20, 520, 1020)
SCAN_SWEEPS = 1000


def digest_lattice(s: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(s, dtype=np.uint8).tobytes()).hexdigest()


def digest_counts(c: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(c, dtype="<u8").tobytes()).hexdigest()


def decay_trajectory(tiled=False):
    L, r, K, p0, seed = wl.DECAY["L"], (3.98 if tiled else wl.R_CRITICAL), wl.K_PAPER, 0.5, 1
    step_fn = oracle.sweep_tiled if tiled else oracle.sweep
    s, nc0 = oracle.init(L, p0, seed)
    counts = [nc0]
    marks = {}
    t, t_end, step = 0, DECAY_MARKS[-1], 20
    t_start = time.time()
    while t < t_end:
        n = min(step, t_end - t)
        s, c = step_fn(s, r, K, seed, t, n)
        counts.extend(int(v) for v in c)
        t += n
        if t in DECAY_MARKS:
            marks[t] = digest_lattice(s)
        print("decay: %d / %d sweeps, %.0f s" % (t, t_end, time.time() - t_start), flush=True)
    if tiled:
        head = ["# Oracle trajectory of the double tiling of Sec. IV (oracle C: 4 x 4 domains of",
                "# four types, 16 random sequential steps per domain per part; Fermi rule Eq. (3),",
                "# cooperator count N_C of Eq. (4)) on a %d x %d periodic lattice: r = %r," % (L, L, r),
                "# K = %r, p0 = %r, seed %d -- the paper's benchmark workload (Fig. 5)." % (K, p0, seed)]
    else:
        head = ["# Oracle trajectory of the 16-colour sweep (Sec. III elementary step, Fermi rule",
                "# Eq. (3), cooperator count N_C of Eq. (4)) on a %d x %d periodic lattice:" % (L, L),
                "# r = %r (r_c of Sec. V), K = %r, p0 = %r, seed %d -- the single-lattice" % (r, K, p0, seed),
                "# benchmark workload."]
    lines = head + [
        "# Written by tests/golden/make_trajectories.py, which calls only the oracle.",
        "# 'lattice t hex': SHA-256 of the L*L bytes (0/1, row-major) after t sweeps;",
        "# 'count t N_C': the count after t sweeps (t = 0: the initial state).",
        "L %d" % L, "r %r" % r, "K %r" % K, "p0 %r" % p0, "seed %d" % seed,
    ]
    lines += ["lattice %d %s" % (m, marks[m]) for m in DECAY_MARKS]
    lines += ["count %d %d" % (q, v) for q, v in enumerate(counts)]
    path = TILED_FILE if tiled else DECAY_FILE
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path, flush=True)


def _scan_one(args):
    L, r, K, p0, seed, n = args
    lat, nc0, counts = oracle.run(L, r, K, p0, seed, n)
    return r, seed, int(counts[-1]), digest_counts(counts), digest_lattice(lat)


def scan_replicas(jobs: int):
    cfg = wl.SCAN
    args = [(cfg["L"], r, cfg["K"], cfg["p0"], s, SCAN_SWEEPS) for r, s in zip(cfg["r_values"], cfg["seeds"])]
    rows = []
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        for k, row in enumerate(ex.map(_scan_one, args)):
            rows.append(row)
            print("scan: replica %d of %d done, %.0f s" % (k + 1, len(args), time.time() - t0), flush=True)
    lines = [
        "# Oracle runs of the L = %d r scan (21 values of r in [3.70, 3.80], seeds" % cfg["L"],
        "# 100..120, K = %r, p0 = %r) through %d sweeps of the 16-colour sweep" % (cfg["K"], cfg["p0"], SCAN_SWEEPS),
        "# (Sec. III elementary step, Eq. (3) Fermi rule, Eq. (4) count).  Written by",
        "# tests/golden/make_trajectories.py, which calls only the oracle.",
        "# columns: r seed N_C(%d) sha256(N_C(1..%d) as little-endian uint64)" % (SCAN_SWEEPS, SCAN_SWEEPS),
        "#          sha256(lattice after %d sweeps: L*L bytes 0/1, row-major)" % SCAN_SWEEPS,
        "L %d" % cfg["L"], "sweeps %d" % SCAN_SWEEPS,
    ]
    lines += ["%r %d %d %s %s" % row for row in rows]
    with open(SCAN_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", SCAN_FILE, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", choices=["decay", "scan", "tiled"], default=None)
    args = ap.parse_args()
    oracle.build(force=False)
    if args.only in (None, "scan"):
        scan_replicas(args.jobs)
    if args.only in (None, "decay"):
        decay_trajectory()
    if args.only in (None, "tiled"):
        decay_trajectory(tiled=True)


if __name__ == "__main__":
    main()

"""Write the stored oracle trajectories that the GPU parity tests compare with.

Every value written here comes from the oracle (oracle A: the 16-colour sweep
of the Sec. III elementary step with the Eq. (3) Fermi rule; oracle C: the
double tiling of Sec. IV; counts as in Eq. (4)); nothing else is called.  Run
from the repository root:

    python tests/golden/make_trajectories.py [--jobs 6] [--only decay|scan|tiled|ensemble|serving]

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
* ensemble256_5000.txt -- 32 sampled replicas of the 256-replica batched
  ensemble (8 of each L in {128, 256, 512, 1024}: replicas 0, 8, ..., 56 of
  each size's block of 64) through all 5000 sweeps: per replica N_C at 1000,
  2500 and 5000 sweeps, the SHA-256 of N_C(1..5000) and of the lattice after
  5000 sweeps.  About 2.5 hours of one core, spread over --jobs processes.
* serving_jobs.txt -- 20 jobs of the serving trace (master seed 7: every
  fifth of its first 100 jobs; L from 88 to 1496, up to 9888 sweeps, r in
  [3.5, 5.6], p0 in [0.1, 0.9]) run alone from their own initial state: per
  job N_C(0), N_C after its last sweep, the SHA-256 of N_C(1..n) and of the
  final lattice.  About four hours of one core, spread over --jobs processes.

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
ENSEMBLE_FILE = os.path.join(HERE, "ensemble256_5000.txt")
ENSEMBLE_SWEEPS = 5000
ENSEMBLE_MARKS = (1000, 2500, 5000)
ENSEMBLE_SAMPLE = tuple(64 * b + 8 * m for b in range(4) for m in range(8))  # 8 replicas of each L
SERVING_FILE = os.path.join(HERE, "serving_jobs.txt")
SERVING_TRACE_JOBS = 100
SERVING_SAMPLE = tuple(range(0, SERVING_TRACE_JOBS, 5))


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


def _marked_run(args):
    """Init + n sweeps of oracle A with N_C recorded at the marks."""
    key, L, r, K, p0, seed, n, marks = args
    s, nc0 = oracle.init(L, p0, seed)
    counts = []
    t = 0
    for m in sorted(set(marks) | {n}):
        s, c = oracle.sweep(s, r, K, seed, t, m - t)
        counts.extend(int(v) for v in c)
        t = m
    counts = np.asarray(counts, dtype=np.uint64)
    return key, nc0, counts, digest_counts(counts), digest_lattice(s)


CACHE_DIR = None  # --cache: finished runs are kept there and not repeated


def _cached_run(args):
    """_marked_run, reusing (and saving) a finished run under CACHE_DIR."""
    if CACHE_DIR is None:
        return _marked_run(args)
    key = args[0]
    path = os.path.join(CACHE_DIR, "run_%s.npz" % hashlib.sha256(repr(args).encode()).hexdigest()[:24])
    if os.path.exists(path):
        z = np.load(path)
        return key, int(z["nc0"]), z["counts"], str(z["dc"]), str(z["dl"])
    res = _marked_run(args)
    tmp = path + ".tmp.npz"
    np.savez(tmp, nc0=res[1], counts=res[2], dc=res[3], dl=res[4])
    os.replace(tmp, path)
    return res


def _run_pool(tasks, jobs, label):
    """Run _marked_run over tasks (largest first), yielding results as they end."""
    tasks = sorted(tasks, key=lambda a: -(a[1] ** 2 * a[6]))
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        for k, res in enumerate(ex.map(_cached_run, tasks)):
            print("%s: %d of %d done, %.0f s" % (label, k + 1, len(tasks), time.time() - t0), flush=True)
            yield res


def ensemble_replicas_digests(jobs: int):
    reps = wl.ensemble_replicas(sweeps=ENSEMBLE_SWEEPS)
    tasks = [(k, reps[k]["L"], reps[k]["r"], reps[k]["K"], reps[k]["p0"], reps[k]["seed"], ENSEMBLE_SWEEPS,
              ENSEMBLE_MARKS) for k in ENSEMBLE_SAMPLE]
    rows = {}
    for key, nc0, counts, dc, dl in _run_pool(tasks, jobs, "ensemble"):
        rp = reps[key]
        marks = " ".join("%d" % counts[m - 1] for m in ENSEMBLE_MARKS)
        rows[key] = "%d %d %r %d %d %s %s %s" % (key, rp["L"], rp["r"], rp["seed"], nc0, marks, dc, dl)
    lines = [
        "# Oracle runs of sampled replicas of the batched ensemble (256 replicas, 64 of each",
        "# L in {128, 256, 512, 1024}, r ~ U[3.6, 3.9], K = 0.5, p0 = 0.5, master seed 2017)",
        "# through %d sweeps of the 16-colour sweep (Sec. III elementary step, Eq. (3)" % ENSEMBLE_SWEEPS,
        "# Fermi rule, Eq. (4) count), each run alone from its own initial state.  Written by",
        "# tests/golden/make_trajectories.py, which calls only the oracle.",
        "# columns: replica L r seed N_C(0) N_C(%s) sha256(N_C(1..%d) as little-endian" % (
            ") N_C(".join(str(m) for m in ENSEMBLE_MARKS), ENSEMBLE_SWEEPS),
        "#          uint64) sha256(lattice after %d sweeps: L*L bytes 0/1, row-major)" % ENSEMBLE_SWEEPS,
        "sweeps %d" % ENSEMBLE_SWEEPS,
    ]
    lines += [rows[k] for k in sorted(rows)]
    with open(ENSEMBLE_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", ENSEMBLE_FILE, flush=True)


def serving_job_digests(jobs: int):
    trace = wl.serving_trace(SERVING_TRACE_JOBS, 1.0)
    tasks = [(q, trace[q]["L"], trace[q]["r"], trace[q]["K"], trace[q]["p0"], trace[q]["seed"],
              trace[q]["sweeps"], ()) for q in SERVING_SAMPLE]
    rows = {}
    for key, nc0, counts, dc, dl in _run_pool(tasks, jobs, "serving"):
        j = trace[key]
        rows[key] = "%d %d %r %r %d %d %d %d %s %s" % (key, j["L"], j["r"], j["p0"], j["seed"], j["sweeps"], nc0,
                                                    counts[-1], dc, dl)
    lines = [
        "# Oracle runs of sampled jobs of the serving trace (wl.serving_trace, master seed 7:",
        "# L log-uniform in [64, 2048], r ~ U[3.5, 5.6], sweeps ~ U{1000..10000}, p0 ~ U[0.1, 0.9],",
        "# K = 0.5), each run alone from its own initial state with the 16-colour sweep",
        "# (Sec. III elementary step, Eq. (3) Fermi rule, Eq. (4) count).  Written by",
        "# tests/golden/make_trajectories.py, which calls only the oracle.",
        "# columns: job L r p0 seed sweeps N_C(0) N_C(sweeps) sha256(N_C(1..sweeps) as",
        "#          little-endian uint64) sha256(final lattice: L*L bytes 0/1, row-major)",
        "trace_jobs %d" % SERVING_TRACE_JOBS,
    ]
    lines += [rows[k] for k in sorted(rows)]
    with open(SERVING_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", SERVING_FILE, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", choices=["decay", "scan", "tiled", "ensemble", "serving"], default=None)
    ap.add_argument("--cache", default=None, help="directory that keeps finished ensemble/serving runs, so "
                    "that an interrupted run resumes")
    args = ap.parse_args()
    global CACHE_DIR
    if args.cache:
        os.makedirs(args.cache, exist_ok=True)
        CACHE_DIR = os.path.abspath(args.cache)
    oracle.build(force=False)
    if args.only in (None, "scan"):
        scan_replicas(args.jobs)
    if args.only in (None, "decay"):
        decay_trajectory()
    if args.only in (None, "tiled"):
        decay_trajectory(tiled=True)
    if args.only in (None, "ensemble"):
        ensemble_replicas_digests(args.jobs)
    if args.only in (None, "serving"):
        serving_job_digests(args.jobs)


if __name__ == "__main__":
    main()

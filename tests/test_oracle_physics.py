"""Statistical pins: stationary cooperator density (Eq. (4)) of the oracles.

* Oracle B (random sequential, the paper's own dynamics) must reproduce the
  stationary density the paper prints for the Fig. 5 benchmark point:
  rho_C = 0.5 at r = 3.98, K = 0.5.
* Oracle A (16-colour sweep) is a different schedule of the same elementary
  step.  Its stationary density must agree with oracle B's within three
  combined standard errors plus a stated systematic allowance of 0.02 for the
  schedule (measured difference about +0.009 at L = 128, r = 3.98).
* Oracle C (the double tiling of Sec. IV) runs random sequential steps inside
  each domain; its stationary density must agree with oracle B's within three
  combined standard errors with no schedule allowance, and sit at the
  printed rho_C = 0.5 at r = 3.98 (measured at L = 64: 0.499 +- 0.003
  against 0.504 +- 0.003 for oracle B).
* All must show the absorbing-state transition reported in Sec. V: below
  r ~ 3.74 cooperators die out, above it they survive.
"""
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

L = 64
RELAX, MEASURE = 400, 400
SEEDS = range(1, 9)
SCHEDULE_ALLOWANCE = 0.02


def _rho_b(args):
    import oracle
    r, seed = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.rs_run(s, r, 0.5, 1000 + seed, RELAX + MEASURE)
    return float(c[RELAX:].mean()) / (L * L)


def _rho_a(args):
    import oracle
    r, seed = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.sweep(s, r, 0.5, seed, 0, RELAX + MEASURE)
    return float(c[RELAX:].mean()) / (L * L)


def _rho_c(args):
    import oracle
    r, seed = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.sweep_tiled(s, r, 0.5, seed, 0, RELAX + MEASURE)
    return float(c[RELAX:].mean()) / (L * L)


def _final_c(args):
    import oracle
    r, seed, n = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.sweep_tiled(s, r, 0.5, seed, 0, n)
    return int(c[-1])


def _final_a(args):
    import oracle
    r, seed, n = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.sweep(s, r, 0.5, seed, 0, n)
    return int(c[-1])


def _final_b(args):
    import oracle
    r, seed, n = args
    s, _ = oracle.init(L, 0.5, seed)
    _, c = oracle.rs_run(s, r, 0.5, 50 + seed, n)
    return int(c[-1])


def _mean_sem(v):
    v = np.asarray(v)
    return v.mean(), v.std(ddof=1) / np.sqrt(len(v))


@pytest.fixture(scope="module")
def pool(oracle_lib):
    with ProcessPoolExecutor(max_workers=8) as ex:
        yield ex


def test_random_sequential_density_at_fig5_point(pool):
    m, e = _mean_sem(list(pool.map(_rho_b, [(3.98, s) for s in SEEDS])))
    assert abs(m - 0.5) < max(0.015, 3 * e), (m, e)


@pytest.mark.parametrize("r", [3.98, 4.6])
def test_sweep_schedule_agrees_with_random_sequential(pool, r):
    ma, ea = _mean_sem(list(pool.map(_rho_a, [(r, s) for s in SEEDS])))
    mb, eb = _mean_sem(list(pool.map(_rho_b, [(r, s) for s in SEEDS])))
    assert abs(ma - mb) < 3 * np.hypot(ea, eb) + SCHEDULE_ALLOWANCE, (ma, ea, mb, eb)


@pytest.mark.parametrize("r", [3.98, 4.6])
def test_tiled_schedule_agrees_with_random_sequential(pool, r):
    mc, ec = _mean_sem(list(pool.map(_rho_c, [(r, s) for s in SEEDS])))
    mb, eb = _mean_sem(list(pool.map(_rho_b, [(r, s) for s in SEEDS])))
    assert abs(mc - mb) < 3 * np.hypot(ec, eb), (mc, ec, mb, eb)
    if r == 3.98:
        assert abs(mc - 0.5) < max(0.015, 3 * ec), (mc, ec)


def test_extinction_below_and_survival_above_threshold(pool):
    n = 1000
    for fn in (_final_a, _final_b, _final_c):
        low = list(pool.map(fn, [(3.5, s, n) for s in range(1, 5)]))
        high = list(pool.map(fn, [(4.2, s, n) for s in range(1, 5)]))
        assert all(v == 0 for v in low), low
        assert all(v > 0.4 * L * L for v in high), high


# The full statistical comparison: larger lattices, more seeds, longer runs
# (L = 256, 16 seeds, 5000 sweeps of relaxation then 5000 measured, r in
# {3.9, 4.2, 4.6}): about an hour of eight cores, so it runs only when
# PGG_RUN_SLOW=1 is set (it is marked slow as well).
BIG_L, BIG_RELAX, BIG_MEASURE, BIG_SEEDS = 256, 5000, 5000, range(1, 17)


def _big_rho(args):
    import oracle
    which, r, seed = args
    s, _ = oracle.init(BIG_L, 0.5, seed)
    n = BIG_RELAX + BIG_MEASURE
    if which == "A":
        _, c = oracle.sweep(s, r, 0.5, seed, 0, n)
    elif which == "B":
        _, c = oracle.rs_run(s, r, 0.5, 1000 + seed, n)
    else:
        _, c = oracle.sweep_tiled(s, r, 0.5, seed, 0, n)
    return which, r, float(c[BIG_RELAX:].mean()) / (BIG_L * BIG_L)


@pytest.mark.slow
def test_schedules_against_random_sequential_at_scale(oracle_lib):
    import os
    if os.environ.get("PGG_RUN_SLOW") != "1":
        pytest.skip("set PGG_RUN_SLOW=1 to run the hour-long statistical comparison")
    rs = (3.9, 4.2, 4.6)
    tasks = [(w, r, s) for r in rs for w in "ABC" for s in BIG_SEEDS]
    vals = {}
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        for w, r, rho in ex.map(_big_rho, tasks):
            vals.setdefault((w, r), []).append(rho)
    for r in rs:
        (ma, ea), (mb, eb), (mc, ec) = (_mean_sem(vals[(w, r)]) for w in "ABC")
        print("r = %.2f: A %.5f +- %.5f, B %.5f +- %.5f, C %.5f +- %.5f; A - B = %+.5f (3 sigma %.5f)"
              % (r, ma, ea, mb, eb, mc, ec, ma - mb, 3 * np.hypot(ea, eb)), flush=True)
        assert abs(mc - mb) < 3 * np.hypot(ec, eb), (r, mc, ec, mb, eb)
        assert abs(ma - mb) < 3 * np.hypot(ea, eb) + SCHEDULE_ALLOWANCE, (r, ma, ea, mb, eb)

"""GPU: the batched ensemble equals the replicas run one by one, bit for bit."""
import numpy as np
import pytest

from paper_1704_08098_amd import workloads as wl

pytestmark = pytest.mark.gpu


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


def _solo(pgg, rp, n):
    with pgg.Sim(rp["L"], rp["r"], rp.get("K", 0.5), rp.get("p0", 0.5), rp["seed"], "bits", "segment") as sim:
        c = sim.sweep(n)
        return c, sim.read_lattice()


def test_uneven_replicas_equal_solo_runs(pgg, oracle_lib):
    reps = [dict(L=64, r=3.9, seed=1), dict(L=100, r=4.3, seed=2, p0=0.3), dict(L=128, r=3.75, seed=3),
            dict(L=196, r=5.1, seed=4, K=0.8), dict(L=256, r=3.62, seed=2**40 + 5), dict(L=68, r=4.0, seed=6)]
    n, chunk = 45, 8  # 5 full graph replays and a shorter tail chunk
    say("ensemble of", len(reps), "replicas")
    with pgg.Ensemble(reps, chunk=chunk) as ens:
        got = np.concatenate([ens.sweep(20), ens.sweep(0), ens.sweep(25)], axis=1)
        assert ens.t == n
        nc = ens.coop_counts()
        lats = [ens.read_lattice(k) for k in range(len(reps))]
    for k, rp in enumerate(reps):
        c, lat = _solo(pgg, rp, n)
        assert np.array_equal(got[k], c), k
        assert np.array_equal(lats[k], lat), k
        assert int(nc[k]) == int(c[-1])
    # two replicas against the oracle directly
    for k in (1, 3):
        rp = reps[k]
        ref, _, counts = oracle_lib.run(rp["L"], rp["r"], rp.get("K", 0.5), rp.get("p0", 0.5), rp["seed"], n)
        assert np.array_equal(got[k], counts)
        assert np.array_equal(lats[k], ref)


def test_graph_replays_match_eager_runs(pgg):
    """Every replay of the captured chunk equals the eager single-lattice path."""
    reps = [dict(L=128, r=3.8, seed=11), dict(L=256, r=3.7, seed=12)]
    solo = [_solo(pgg, rp, 60)[0] for rp in reps]
    with pgg.Ensemble(reps, chunk=10) as ens:
        for rep in range(6):
            c = ens.sweep(10)
            for k in range(len(reps)):
                assert np.array_equal(c[k], solo[k][10 * rep:10 * rep + 10]), (rep, k)


@pytest.mark.parametrize("tile", [32, 64, 96, 224])
def test_tiles_do_not_change_results(pgg, tile):
    reps = [dict(L=256, r=3.85, seed=21), dict(L=260, r=4.1, seed=22)]
    ref = [_solo(pgg, rp, 12) for rp in reps]
    with pgg.Ensemble(reps, tiles=[tile, tile], chunk=5) as ens:
        c = ens.sweep(12)
        for k in range(len(reps)):
            assert np.array_equal(c[k], ref[k][0])
            assert np.array_equal(ens.read_lattice(k), ref[k][1])


@pytest.mark.parametrize("wpg", [2, 4, 8])
def test_waves_per_group_do_not_change_results(pgg, wpg):
    """Uneven replicas whose wave counts are not multiples of the group size
    (padding waves idle), each equal to its solo run."""
    reps = [dict(L=100, r=3.85, seed=31), dict(L=132, r=4.2, seed=32), dict(L=64, r=3.7, seed=33)]
    ref = [_solo(pgg, rp, 9) for rp in reps]
    say("waves per group", wpg)
    with pgg.Ensemble(reps, chunk=4, waves_per_group=wpg) as ens:
        c = ens.sweep(9)
        for k in range(len(reps)):
            assert np.array_equal(c[k], ref[k][0]), k
            assert np.array_equal(ens.read_lattice(k), ref[k][1]), k


def test_full_ensemble_sample(pgg):
    """The 256-replica ensemble (L = 128..1024), 40 sweeps: sampled replicas
    equal their solo runs; every count equals a recount of the lattice."""
    reps = wl.ensemble_replicas()
    with pgg.Ensemble(reps, chunk=20) as ens:
        c = ens.sweep(40)
        for k in (0, 70, 130, 200, 255):
            sc, sl = _solo(pgg, reps[k], 40)
            assert np.array_equal(c[k], sc), k
            lat = ens.read_lattice(k)
            assert np.array_equal(lat, sl), k
            assert int(lat.sum()) == int(c[k][-1])


def test_invalid_replicas_are_rejected(pgg):
    for bad in ([dict(L=60, r=3.8, seed=1)], [dict(L=100, r=-1.0, seed=1)], []):
        with pytest.raises(pgg.PggError) as e:
            pgg.Ensemble(bad)
        assert e.value.status == pgg.PGG_E_INVAL
    with pytest.raises(pgg.PggError):
        pgg.Ensemble([dict(L=128, r=3.8, seed=1)], tiles=[48])
    for wpg in (1, 3, 16):
        with pytest.raises(pgg.PggError):
            pgg.Ensemble([dict(L=128, r=3.8, seed=1)], waves_per_group=wpg)


def test_autotune_choices_are_valid_and_do_not_change_results(pgg, oracle_lib):
    """The autotuner times width and chunk choices on trial ensembles (it fails
    itself if any two choices give different counts); the chosen settings are
    valid and reproduce the default ensemble and the oracle."""
    reps = [dict(L=128, r=3.8, seed=11), dict(L=256, r=3.7, seed=12), dict(L=128, r=3.9, seed=13),
            dict(L=256, r=3.65, seed=14), dict(L=96, r=4.0, seed=15)]
    say("autotune over", [rp["L"] for rp in reps])
    tune, ms = pgg.ensemble_autotune(reps, probe_sweeps=4)
    tiles = tune["tiles"]
    assert tune["chunk"] in (8, 16, 32, 64, 128) and tune["waves_per_group"] in (2, 4, 8) and ms > 0.0
    assert tune["branches"] in (1, 2, 4) and tune["resident_max_L"] in (0, 128, 256)
    by_L = {}
    for rp, w in zip(reps, tiles):
        # segments of a multiple of 32 columns up to L - 32, or whole rows (L)
        assert (w % 32 == 0 and 32 <= w <= rp["L"] - 32) or w == rp["L"]
        by_L.setdefault(rp["L"], set()).add(int(w))
    assert all(len(ws) == 1 for ws in by_L.values())
    n = 21
    with pgg.Ensemble(reps, **tune) as a, pgg.Ensemble(reps) as b:
        ca, cb = a.sweep(n), b.sweep(n)
        assert np.array_equal(ca, cb)
        ref, _, counts = oracle_lib.run(256, 3.7, 0.5, 0.5, 12, n)
        assert np.array_equal(ca[1], counts)
        assert np.array_equal(a.read_lattice(1), ref)


def _oracle_run(args):
    import oracle
    L, r, K, p0, seed, n = args
    lat, nc0, counts = oracle.run(L, r, K, p0, seed, n)
    return lat, counts


def test_r_scan_as_one_ensemble_against_oracle(pgg, oracle_lib):
    """The L = 1024 r scan (21 values in [3.70, 3.80], seeds 100..120) run as
    one batched ensemble: every replica's counts after each of 30 sweeps and
    its final lattice equal the oracle's."""
    from concurrent.futures import ProcessPoolExecutor
    cfg, n = wl.SCAN, 30
    reps = [dict(L=cfg["L"], r=r, K=cfg["K"], p0=cfg["p0"], seed=s)
            for r, s in zip(cfg["r_values"], cfg["seeds"])]
    with ProcessPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(_oracle_run, [(rp["L"], rp["r"], rp["K"], rp["p0"], rp["seed"], n) for rp in reps]))
    say("r-scan ensemble of", len(reps))
    with pgg.Ensemble(reps, chunk=16) as ens:
        c = ens.sweep(n)
        for k, (lat, counts) in enumerate(refs):
            assert np.array_equal(c[k], counts), k
            assert np.array_equal(ens.read_lattice(k), lat), k


def test_r_scan_ensemble_against_stored_oracle_runs(pgg):
    """The L = 1024 r scan (21 replicas) as one ensemble through 1000 sweeps,
    with the tuning the benchmark's ensemble pass uses by default (automatic
    widths, chunks of 50): every replica's counts after each sweep and its
    final lattice equal the oracle's (stored digests,
    tests/golden/make_trajectories.py)."""
    import hashlib
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "rscan_L1024_1000.txt")
    rows, n = [], None
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "L":
                assert int(parts[1]) == wl.SCAN["L"]
            elif parts[0] == "sweeps":
                n = int(parts[1])
            else:
                rows.append((float(parts[0]), int(parts[1]), int(parts[2]), parts[3], parts[4]))
    cfg = wl.SCAN
    assert [(r, s) for r, s, *_ in rows] == list(zip(cfg["r_values"], cfg["seeds"]))
    reps = [dict(L=cfg["L"], r=r, K=cfg["K"], p0=cfg["p0"], seed=s) for r, s, *_ in rows]
    say("r-scan ensemble vs stored oracle runs,", len(reps), "replicas,", n, "sweeps")
    with pgg.Ensemble(reps, chunk=50) as ens:
        c = np.concatenate([ens.sweep(1), ens.sweep(n - 1)], axis=1)
        for k, (r, seed, final, counts_sha, lat_sha) in enumerate(rows):
            assert int(c[k, -1]) == final, (k, r)
            assert hashlib.sha256(np.ascontiguousarray(c[k], dtype="<u8").tobytes()).hexdigest() == counts_sha, (k, r)
            assert hashlib.sha256(ens.read_lattice(k).tobytes()).hexdigest() == lat_sha, (k, r)



def test_r_scan_driver_matches_oracle_stationary_densities(pgg, oracle_lib):
    """observables.r_scan (the r scan as one ensemble, counts fetched in
    blocks) on a reduced scan -- L = 128, the 21 values of r, 300 sweeps,
    mean over the last 150 -- gives the oracle's counts and hence exactly the
    oracle's stationary densities."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_1704_08098_amd import observables as ob
    cfg = dict(wl.SCAN, L=128, sweeps=300, average_last=150)
    args = [(cfg["L"], r, cfg["K"], cfg["p0"], s, cfg["sweeps"]) for r, s in zip(cfg["r_values"], cfg["seeds"])]
    with ProcessPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(_oracle_run, args))
    say("r_scan driver, L", cfg["L"])
    r, rho, counts = ob.r_scan(pgg, cfg, block=128)
    for k, (lat, ref_counts) in enumerate(refs):
        assert np.array_equal(counts[k], ref_counts), k
        assert rho[k] == ob.stationary_density(ref_counts, cfg["L"], cfg["average_last"]), k


def test_r_scan_lattices_tiled_matches_oracle_c(pgg, oracle_lib):
    """observables.r_scan_lattices (one lattice per r, four worker threads on
    streams of their own) with the double-tiling schedule: every lattice's
    counts equal oracle C's, whichever thread and stream ran it."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_1704_08098_amd import observables as ob
    cfg = dict(wl.SCAN, L=64, sweeps=150, average_last=50, r_values=(3.74, 3.76, 3.8, 3.9, 4.2),
               seeds=(7, 8, 9, 10, 11))
    args = [(cfg["L"], r, s, cfg["sweeps"]) for r, s in zip(cfg["r_values"], cfg["seeds"])]
    with ProcessPoolExecutor(max_workers=5) as ex:
        refs = list(ex.map(_oracle_tiled, args))
    say("r_scan_lattices tiled, L", cfg["L"])
    r, rho, counts = ob.r_scan_lattices(pgg, cfg, schedule="tiled", workers=4, block=40)
    for k, ref_counts in enumerate(refs):
        assert np.array_equal(counts[k], ref_counts), k


def test_r_scan_lattices_colour16_threads_match_oracle(pgg, oracle_lib):
    """observables.r_scan_lattices with the 16-colour sweep: eight host threads
    create, capture (segment-kernel graphs) and sweep lattices at once, each
    on a stream of its own; every lattice's counts equal the oracle's."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_1704_08098_amd import observables as ob
    cfg = dict(wl.SCAN, L=160, sweeps=300, average_last=100,
               r_values=(3.70, 3.72, 3.74, 3.76, 3.78, 3.80, 3.9, 4.1, 4.4, 5.0),
               seeds=(21, 22, 23, 24, 25, 26, 27, 28, 29, 30))
    args = [(cfg["L"], r, s, cfg["sweeps"]) for r, s in zip(cfg["r_values"], cfg["seeds"])]
    with ProcessPoolExecutor(max_workers=5) as ex:
        refs = list(ex.map(_oracle_colour16, args))
    say("r_scan_lattices colour16, 8 threads, L", cfg["L"])
    r, rho, counts = ob.r_scan_lattices(pgg, cfg, schedule="colour16", workers=8, block=40)
    for k, ref_counts in enumerate(refs):
        assert np.array_equal(counts[k], ref_counts), k


def _oracle_colour16(args):
    import oracle
    L, r, seed, n = args
    return oracle.run(L, r, 0.5, 0.5, seed, n)[2]


def _oracle_tiled(args):
    import oracle
    L, r, seed, n = args
    return oracle.run_tiled(L, r, 0.5, 0.5, seed, n)[2]


def test_tiled_ensemble_equals_oracle_c(pgg, oracle_lib):
    """Replicas of uneven L (multiples of 8, some not of 32), r and seed with
    the double-tiling schedule as one ensemble: every replica's counts after
    each of 30 steps (chunks of 8: graph replays and a short tail) and its
    final lattice equal oracle C's, and a second call continues them."""
    from concurrent.futures import ProcessPoolExecutor
    reps = [dict(L=64, r=3.80, seed=3, schedule="tiled"), dict(L=96, r=4.40, seed=4, schedule="tiled"),
            dict(L=136, r=3.75, seed=5, schedule="tiled"), dict(L=256, r=3.98, seed=6, schedule="tiled"),
            dict(L=520, r=3.745, seed=7, schedule="tiled")]
    n1, n2 = 30, 5
    with ProcessPoolExecutor(max_workers=5) as ex:
        refs = list(ex.map(_oracle_tiled_run, [(rp["L"], rp["r"], rp["seed"], n1 + n2) for rp in reps]))
    say("tiled ensemble of", len(reps))
    with pgg.Ensemble(reps, chunk=8) as ens:
        c = np.concatenate([ens.sweep(n1), ens.sweep(n2)], axis=1)
        for k, (lat, counts) in enumerate(refs):
            assert np.array_equal(c[k], counts), k
            assert np.array_equal(ens.read_lattice(k), lat), k


def _oracle_tiled_run(args):
    import oracle
    L, r, seed, n = args
    lat, _, counts = oracle.run_tiled(L, r, 0.5, 0.5, seed, n)
    return lat, counts


@pytest.mark.parametrize("branches", [2, 3, 4, 16])
def test_concurrent_replica_groups_do_not_change_results(pgg, oracle_lib, branches):
    """Replicas cut into contiguous groups of about equal work that run as
    parallel branches of the chunk's graph: every replica's counts after
    every sweep and its lattice equal the one-branch ensemble's, and two of
    them equal the oracle (chunks of 8 with a short tail, uneven sizes so the
    groups hold different numbers of replicas)."""
    reps = [dict(L=L, r=r, seed=200 + k) for k, (L, r) in
            enumerate([(64, 3.8), (96, 3.9), (128, 3.75), (256, 3.85), (132, 4.1), (512, 3.8), (64, 4.4),
                       (200, 3.95)])]
    n = 21
    say("ensemble with", branches, "branches over", [rp["L"] for rp in reps])
    with pgg.Ensemble(reps, chunk=8, branches=branches) as a, pgg.Ensemble(reps, chunk=8) as b:
        ca, cb = a.sweep(n), b.sweep(n)
        assert np.array_equal(ca, cb)
        for k in range(len(reps)):
            assert np.array_equal(a.read_lattice(k), b.read_lattice(k)), k
        assert np.array_equal(a.coop_counts(), b.coop_counts())
    for k in (0, 5):
        rp = reps[k]
        ref, _, counts = oracle_lib.run(rp["L"], rp["r"], 0.5, 0.5, rp["seed"], n)
        assert np.array_equal(ca[k], counts), k


def test_branches_refused_where_they_do_not_apply(pgg):
    with pytest.raises(pgg.PggError):
        pgg.Ensemble([dict(L=128, r=3.8, seed=1)], branches=17)
    with pytest.raises(pgg.PggError):
        pgg.Ensemble([dict(L=128, r=3.8, seed=1, schedule="tiled"), dict(L=64, r=3.8, seed=2, schedule="tiled")],
                     branches=2)


def test_one_shot_run_equals_the_handle_calls(pgg, oracle_lib):
    """pgg_ensemble_run (autotuned, and with given settings) returns the same
    counts as create / sweep on the same replicas, and the oracle's."""
    reps = [dict(L=L, r=r, seed=300 + k) for k, (L, r) in enumerate([(64, 3.8), (128, 3.9), (100, 4.0), (256, 3.75)])]
    n = 17
    say("one-shot ensemble run over", [rp["L"] for rp in reps])
    with pgg.Ensemble(reps, chunk=8) as ens:
        ref = ens.sweep(n)
    assert np.array_equal(pgg.ensemble_run(reps, n), ref)
    assert np.array_equal(pgg.ensemble_run(reps, n, tune=dict(chunk=4, waves_per_group=2, branches=2)), ref)
    _, _, counts = oracle_lib.run(100, 4.0, 0.5, 0.5, 302, n)
    assert np.array_equal(ref[2], counts)


@pytest.mark.parametrize("res_L,res_waves,branches", [(128, 4, 0), (256, 8, 0), (256, 16, 2), (256, 0, 4),
                                                      (64, 4, 2), (512, 4, 0), (512, 16, 2), (300, 8, 0)])
def test_resident_replicas_do_not_change_results(pgg, oracle_lib, res_L, res_waves, branches):
    """Replicas of side a multiple of 32 up to resident_max_L swept whole in
    LDS (a chunk of sweeps per launch) beside the segment launches of the
    others: counts after every sweep, coop counts and lattices equal the
    plain ensemble's, and a resident and a segment replica equal the oracle
    (chunks of 8 with a short tail; sides that do not fit -- not a multiple
    of 32, or too large -- stay on the segment path; L = 512 takes 104 KB of
    LDS per workgroup)."""
    reps = [dict(L=L, r=r, seed=400 + k) for k, (L, r) in
            enumerate([(64, 3.8), (96, 3.9), (100, 4.0), (128, 3.75), (160, 4.2), (196, 3.85), (224, 3.7),
                       (256, 3.95), (512, 3.8), (68, 4.4)])]
    n = 19
    tune = dict(chunk=8, branches=branches, resident_max_L=res_L, resident_waves=res_waves)
    say("ensemble with resident sides up to", res_L, "waves", res_waves, "branches", branches)
    with pgg.Ensemble(reps, **tune) as a, pgg.Ensemble(reps, chunk=8) as b:
        ca = np.concatenate([a.sweep(11), a.sweep(8)], axis=1)
        cb = b.sweep(n)
        assert np.array_equal(ca, cb)
        for k in range(len(reps)):
            assert np.array_equal(a.read_lattice(k), b.read_lattice(k)), k
        assert np.array_equal(a.coop_counts(), b.coop_counts())
    for k in (0, 2):  # L = 64 is resident for every setting here, L = 100 never
        rp = reps[k]
        ref, _, counts = oracle_lib.run(rp["L"], rp["r"], 0.5, 0.5, rp["seed"], n)
        assert np.array_equal(ca[k], counts), k


def test_resident_settings_refused_where_they_do_not_apply(pgg):
    one = [dict(L=128, r=3.8, seed=1)]
    for bad in (dict(resident_max_L=32), dict(resident_max_L=600), dict(resident_max_L=128, resident_waves=3),
                dict(resident_max_L=128, resident_waves=32)):
        with pytest.raises(pgg.PggError):
            pgg.Ensemble(one, **bad)
    with pytest.raises(pgg.PggError):
        pgg.Ensemble([dict(L=128, r=3.8, seed=1, schedule="tiled")], resident_max_L=128)

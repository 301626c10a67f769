"""GPU parity: the HIP path (through the C ABI) against the oracle.

Bit-exact: lattice state and integer cooperator count after every sweep.
Every GPU step prints what it runs (variant, L, r, seed) before it runs.
"""
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from paper_1704_08098_amd import workloads as wl

pytestmark = pytest.mark.gpu

VARIANTS = [("int8", "colour"), ("bits", "rowband"), ("bits", "rowband_compact"),
            ("bits", "rowband_staged"), ("bits", "strip"), ("bits", "segment"), ("int8", "segment")]
# kernels for lattices of L >= 512, a multiple of 32, beside all the others
LARGE_VARIANTS = VARIANTS + [("bits", "segment_pair"), ("int8", "segment_pair")]


def say(*a):
    print(*a, flush=True)


MIN_L = {"segment": 64}


def open_sim(pgg, L, r, K, p0, seed, layout, kernel, **kw):
    """The Sim, or None after checking that an unsupported size is refused."""
    if L < MIN_L.get(kernel, 4):
        with pytest.raises(pgg.PggError) as e:
            pgg.Sim(L, r, K, p0, seed, layout, kernel, **kw)
        assert e.value.status == pgg.PGG_E_INVAL
        return None
    return pgg.Sim(L, r, K, p0, seed, layout, kernel, **kw)


@pytest.fixture(scope="module")
def pgg(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.set_device(0)
    from paper_1704_08098_amd import pgg as mod
    mod.load()
    return mod


def _oracle_trajectory(args):
    """Lattices after each of n sweeps (oracle, sweep by sweep) and counts."""
    import oracle
    L, r, K, p0, seed, n = args
    s, nc0 = oracle.init(L, p0, seed)
    lats, counts = [], []
    for t in range(n):
        s, c = oracle.sweep(s, r, K, seed, t, 1)
        lats.append(s)
        counts.append(int(c[0]))
    return nc0, np.stack(lats), np.array(counts, dtype=np.uint64)


@pytest.fixture(scope="module")
def small_trajectories(oracle_lib):
    cfg = wl.SMALL
    args = [(cfg["L"], cfg["r"], cfg["K"], cfg["p0"], s, cfg["sweeps"]) for s in cfg["seeds"]]
    with ProcessPoolExecutor(max_workers=len(args)) as ex:
        return dict(zip(cfg["seeds"], ex.map(_oracle_trajectory, args)))


@pytest.mark.parametrize("layout,kernel", VARIANTS)
def test_small_config_every_sweep(pgg, small_trajectories, layout, kernel):
    """L = 100, r = 3.8, 1000 sweeps, five seeds: every sweep, bit for bit."""
    cfg = wl.SMALL
    for seed in cfg["seeds"]:
        nc0, lats, counts = small_trajectories[seed]
        say("small config", layout, kernel, "seed", seed)
        with pgg.Sim(cfg["L"], cfg["r"], cfg["K"], cfg["p0"], seed, layout, kernel) as sim:
            assert sim.coop_count() == nc0
            for t in range(cfg["sweeps"]):
                c = sim.sweep(1)
                assert int(c[0]) == int(counts[t]), (seed, t)
                lat = sim.read_lattice()
                if not np.array_equal(lat, lats[t]):
                    bad = np.argwhere(lat != lats[t])
                    pytest.fail("seed %d sweep %d: %d sites differ, first %s" % (seed, t, len(bad), bad[:5]))
            assert sim.t == cfg["sweeps"]
            assert sim.density() == pytest.approx(int(counts[-1]) / cfg["L"] ** 2, abs=0)


def test_threshold_tables_match_oracle(pgg, oracle_lib):
    rs = sorted({wl.SMALL["r"], *wl.SCAN["r_values"], *wl.DECAY["r_values"], 3.98, 5.0, 0.0, 12.5})
    for r in rs:
        for K in (0.5, 0.05, 3.0):
            say("table r", r, "K", K)
            with pgg.Sim(8, r, K, 0.5, 1, "int8") as sim:
                assert np.array_equal(sim.threshold_table(), oracle_lib.table(r, K)), (r, K)


def test_device_tables_are_the_host_tables(pgg, oracle_lib):
    """The table each handle and ensemble replica holds on the device is the
    host-built one (pgg_fermi_table), which equals the oracle's: random (r, K)
    for single lattices, every replica of the 256-replica ensemble, and the r
    of every job of the serving trace (as replicas of an ensemble)."""
    rng = np.random.default_rng(355)
    for r, K in zip(rng.uniform(0.0, 8.0, 40), np.exp(rng.uniform(np.log(0.02), np.log(10.0), 40))):
        say("table r", r, "K", K)
        with pgg.Sim(64, r, K, 0.5, 1, "bits") as sim:
            T = sim.threshold_table()
        assert np.array_equal(T, oracle_lib.table(r, K)) and np.array_equal(T, pgg.pgg_fermi_table(r, K)), (r, K)
    reps = wl.ensemble_replicas()
    say("tables of the", len(reps), "ensemble replicas")
    with pgg.Ensemble(reps, chunk=8) as ens:
        for k, rp in enumerate(reps):
            assert np.array_equal(ens.threshold_table(k), oracle_lib.table(rp["r"], rp["K"])), k
    jobs = wl.serving_trace(300, 1.0)
    say("tables of the", len(jobs), "serving-trace jobs")
    with pgg.Ensemble([dict(L=64, r=j["r"], K=j["K"], p0=j["p0"], seed=j["seed"]) for j in jobs], chunk=8) as ens:
        for k, j in enumerate(jobs):
            assert np.array_equal(ens.threshold_table(k), oracle_lib.table(j["r"], j["K"])), k


@pytest.mark.parametrize("layout", ["int8", "bits"])
def test_initial_states_match_oracle(pgg, oracle_lib, layout):
    for L in (4, 8, 12, 36, 100, 132, 1024):
        for p0 in (0.0, 0.1, 0.5, 0.9, 1.0):
            seed = 1000 + L
            say("init", layout, "L", L, "p0", p0)
            ref, nc = oracle_lib.init(L, p0, seed)
            with pgg.Sim(L, 3.8, 0.5, p0, seed, layout) as sim:
                assert sim.coop_count() == nc
                assert np.array_equal(sim.read_lattice(), ref)


RAGGED = [(4, 3.8, 0.5, 11), (8, 4.4, 0.5, 12), (12, 3.72, 0.5, 13), (16, 5.0, 0.5, 14),
          (20, 3.9, 1.5, 15), (36, 4.1, 0.5, 16), (60, 3.8, 0.1, 17), (68, 4.6, 0.5, 18),
          (100, 3.75, 0.5, 2**40 + 19), (132, 3.98, 0.5, 20), (196, 4.0, 0.25, 21),
          (260, 3.85, 0.5, 22), (512, 3.8, 0.5, 23)]


@pytest.mark.parametrize("layout,kernel", VARIANTS)
@pytest.mark.parametrize("L,r,K,seed", RAGGED, ids=lambda v: str(v))
def test_ragged_and_tiny_lattices(pgg, oracle_lib, layout, kernel, L, r, K, seed):
    """Sizes that are not multiples of the 32/64-bit words, and the wrap at L = 4..20."""
    n = 24
    say("ragged", layout, kernel, "L", L, "r", r, "K", K, "seed", seed)
    s0, _ = oracle_lib.init(L, 0.5, seed)
    sim = open_sim(pgg, L, r, K, 0.5, seed, layout, kernel)
    if sim is None:
        return
    with sim:
        ref = s0
        for t in range(n):
            ref, c = oracle_lib.sweep(ref, r, K, seed, t, 1)
            got = sim.sweep(1)
            assert int(got[0]) == int(c[0]), t
            assert np.array_equal(sim.read_lattice(), ref), t


@pytest.mark.parametrize("layout,kernel", VARIANTS)
def test_write_lattice_resume_and_chunking(pgg, oracle_lib, layout, kernel):
    L, r, K, seed, t0 = 68, 3.9, 0.5, 77, 123
    lat = wl.random_lattice(L, 0.4, 5)
    ref, counts = oracle_lib.sweep(lat, r, K, seed, t0, 30)
    say("resume", layout, kernel)
    with pgg.Sim(L, r, K, 0.5, seed, layout, kernel) as sim:
        sim.write_lattice(lat, t0)
        assert sim.t == t0 and sim.coop_count() == int(lat.sum())
        got = np.concatenate([sim.sweep(7), sim.sweep(0), sim.sweep(13), sim.sweep(10)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)
        assert sim.t == t0 + 30


@pytest.mark.parametrize("layout,kernel", VARIANTS)
def test_sweep_index_near_2_pow_32(pgg, oracle_lib, layout, kernel):
    L, r, seed = 36, 3.8, 9
    lat, _ = oracle_lib.init(L, 0.5, seed)
    t0 = 2**32 - 3
    ref, counts = oracle_lib.sweep(lat, r, 0.5, seed, t0, 3)
    say("t near 2^32", layout, kernel)
    sim = open_sim(pgg, L, r, 0.5, 0.5, seed, layout, kernel)
    if sim is None:
        return
    with sim:
        sim.write_lattice(lat, t0)
        assert np.array_equal(sim.sweep(3), counts)
        assert np.array_equal(sim.read_lattice(), ref)
        with pytest.raises(pgg.PggError) as e:
            sim.sweep(1)
        assert e.value.status == pgg.PGG_E_INVAL
        assert sim.t == 2**32  # the rejected call changed nothing


@pytest.mark.parametrize("layout,kernel", VARIANTS)
@pytest.mark.parametrize("value", [0, 1])
def test_absorbing_states_stay(pgg, layout, kernel, value):
    say("absorbing", layout, kernel, value)
    with pgg.Sim(128, 3.8, 0.5, float(value), 3, layout, kernel) as sim:
        c = sim.sweep(20)
        assert np.all(c == value * 128 * 128)
        assert np.all(sim.read_lattice() == value)


def test_write_lattice_rejects_bad_bytes(pgg):
    with pgg.Sim(8, 3.8, 0.5, 0.5, 1, "bits") as sim:
        bad = np.zeros((8, 8), dtype=np.uint8)
        bad[3, 3] = 2
        with pytest.raises(pgg.PggError) as e:
            sim.write_lattice(bad, 0)
        assert e.value.status == pgg.PGG_E_INVAL


@pytest.mark.parametrize("L,kernel", [(100, "auto"), (96, "auto"), (160, "resident")])
def test_caller_buffer_and_stream(pgg, oracle_lib, L, kernel):
    import torch
    r, seed, n = 3.8, 4, 40
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    params = pgg.make_params(L, r, 0.5, 0.5, seed, "bits", kernel)
    buf = torch.zeros(pgg.pgg_device_bytes(params), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    say("caller buffer + stream", L, kernel)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, dev_buf=buf, stream=stream) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)
    # the buffer is the caller's and still holds the lattice (rows of 2 ceil(L / 64) words)
    torch.cuda.synchronize()
    row_bytes = 8 * ((L + 63) // 64)
    host = buf.cpu().numpy().reshape(L, row_bytes)
    bits = np.unpackbits(host, axis=1, bitorder="little")[:, :L]
    assert np.array_equal(bits, ref)


@pytest.mark.parametrize("kernel,L", [("auto", 100), ("segment", 260), ("segment_pair", 512), ("auto", 128),
                                      ("resident", 224)])
def test_int8_caller_buffer_on_segment_kernels(pgg, oracle_lib, kernel, L):
    """int8 layout on the segment kernels (a bit-packed working copy inside the
    library): the caller's byte buffer holds the oracle's lattice after every
    call, calls of several lengths in a row, and a lattice written between
    calls is the one the next call starts from."""
    import torch
    r, seed = 3.85, 500 + L
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, 21)
    params = pgg.make_params(L, r, 0.5, 0.5, seed, "int8", kernel)
    buf = torch.full((pgg.pgg_device_bytes(params),), 7, dtype=torch.uint8, device="cuda")
    say("int8 caller buffer", kernel, L)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "int8", kernel, dev_buf=buf) as sim:
        got = np.concatenate([sim.sweep(1), sim.sweep(13), sim.sweep(7)])
        assert np.array_equal(got, counts)
        torch.cuda.synchronize()
        assert np.array_equal(buf.cpu().numpy().reshape(L, L), ref)
        lat = wl.random_lattice(L, 0.3, 8)
        ref2, counts2 = oracle_lib.sweep(lat, r, 0.5, seed, 40, 9)
        sim.write_lattice(lat, 40)
        assert np.array_equal(sim.sweep(9), counts2)
        torch.cuda.synchronize()
        assert np.array_equal(buf.cpu().numpy().reshape(L, L), ref2)
        assert np.array_equal(sim.read_lattice(), ref2)


@pytest.mark.parametrize("layout,kernel", LARGE_VARIANTS)
def test_scan_size_against_oracle(pgg, oracle_lib, layout, kernel):
    """L = 1024 (the r-scan lattice) at r = 3.75: 12 sweeps, bit for bit."""
    L, r, seed, n = 1024, 3.75, 110, 12
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("L=1024", layout, kernel)
    with pgg.Sim(L, r, 0.5, 0.5, seed, layout, kernel) as sim:
        assert sim.coop_count() == nc0
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.fixture(scope="module")
def decay_reference(oracle_lib):
    L, r, seed, n = wl.DECAY["L"], wl.DECAY["r_values"][1], wl.DECAY["seeds"][0], 2
    return oracle_lib.run(L, r, 0.5, 0.5, seed, n)


@pytest.mark.parametrize("layout,kernel", LARGE_VARIANTS)
def test_full_size_L4096_against_oracle(pgg, decay_reference, layout, kernel):
    """L = 4096 at r_c: init and the first two sweeps, bit for bit."""
    L, r, seed = wl.DECAY["L"], wl.DECAY["r_values"][1], wl.DECAY["seeds"][0]
    ref, nc0, counts = decay_reference
    say("L=4096", layout, kernel)
    with pgg.Sim(L, r, 0.5, 0.5, seed, layout, kernel) as sim:
        assert sim.coop_count() == nc0
        assert np.array_equal(sim.sweep(len(counts)), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_kernels_agree_at_benchmark_size(pgg):
    """L = 4096, r = r_c, 400 sweeps: every kernel, identical counts and lattice;
    the running count equals a recount of the lattice (any-size properties)."""
    L, r, seed, n = wl.DECAY["L"], wl.DECAY["r_values"][1], 1, 400
    results = []
    for layout, kernel in LARGE_VARIANTS:
        say("bench size", layout, kernel)
        with pgg.Sim(L, r, 0.5, 0.5, seed, layout, kernel) as sim:
            c = sim.sweep(n)
            lat = sim.read_lattice()
            assert int(lat.sum()) == int(c[-1])
            results.append((c, lat))
    for c, lat in results[1:]:
        assert np.array_equal(c, results[0][0])
        assert np.array_equal(lat, results[0][1])


def test_maximum_size_kernels_agree(pgg):
    """L = 32768 (the largest accepted): the dense and compact row-band kernels
    and the automatic choice (the segment kernel) give identical device
    lattices after two sweeps; counts are recounts."""
    import torch
    L, r, seed = 32768, 3.7443, 5
    bufs, counts = [], []
    for kernel in ("rowband", "rowband_compact", "auto"):
        params = pgg.make_params(L, r, 0.5, 0.5, seed, "bits", kernel)
        buf = torch.empty(pgg.pgg_device_bytes(params), dtype=torch.uint8, device="cuda")
        say("L=32768", kernel)
        with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, dev_buf=buf) as sim:
            counts.append(sim.sweep(2))
        torch.cuda.synchronize()
        bufs.append(buf)
    for b, c in zip(bufs[1:], counts[1:]):
        assert torch.equal(bufs[0], b)
        assert np.array_equal(counts[0], c)
    pop = int(np.bitwise_count(bufs[0].cpu().numpy()).sum(dtype=np.uint64))
    assert pop == int(counts[0][-1])


@pytest.mark.parametrize("kernel,tile", [("strip", 4), ("strip", 5), ("strip", 7), ("strip", 13),
                                         ("strip", 68), ("rowband", 1), ("rowband", 3),
                                         ("rowband_compact", 2), ("rowband_staged", 4),
                                         ("segment", 32)])
def test_tile_do_not_change_results(pgg, oracle_lib, kernel, tile):
    """Strip heights / rows per band, including a single strip (H = L)."""
    L, r, seed, n = 68, 3.85, 31, 16
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("tile", kernel, tile)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, tile=tile) as sim:
        got = np.concatenate([sim.sweep(5), sim.sweep(11)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_strip_abort_path_reports_and_recovers(pgg, oracle_lib):
    """A zero wait bound makes strip workgroups give up on their neighbours:
    every workgroup exits, the call reports PGG_E_DEVICE and the handle is
    poisoned; a fresh handle afterwards computes correctly."""
    L, r, seed = 1024, 3.8, 3
    say("strip abort path")
    sim = pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "strip", tile=4)
    sim.set_strip_wait(0.0)
    with pytest.raises(pgg.PggError) as e:
        sim.sweep(50)  # counts requested: synchronises and checks the flag
    assert e.value.status == pgg.PGG_E_DEVICE
    with pytest.raises(pgg.PggError) as e2:
        sim.sweep(1)
    assert e2.value.status == pgg.PGG_E_STATE
    sim.close()
    ref, nc0, counts = oracle_lib.run(100, r, 0.5, 0.5, seed, 10)
    with pgg.Sim(100, r, 0.5, 0.5, seed, "bits", "strip") as ok:
        assert np.array_equal(ok.sweep(10), counts)
        assert np.array_equal(ok.read_lattice(), ref)


@pytest.mark.parametrize("L,segw", [(64, 32), (100, 32), (100, 64), (132, 96), (196, 64), (260, 224),
                                    (512, 128), (512, 480), (1024, 992),
                                    (68, 68), (100, 100), (196, 196), (260, 260), (500, 500), (1020, 1020),
                                    (1500, 1500), (1500, 768), (2044, 2044)])
def test_segment_widths(pgg, oracle_lib, L, segw):
    """Segment widths from 32 columns to L - 32, including a short last
    segment, and whole periodic rows for L not a multiple of 32 (one row per
    wave, its margins the periodic images of its own sites)."""
    r, seed, n = 3.9, 40 + L, 12
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("segment", L, segw)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment", tile=segw) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.mark.parametrize("kernel,L,segw", [("segment", 4100, 4100), ("segment", 4096, 4064),
                                           ("segment_pair", 4096, 4032)])
def test_rows_wider_than_one_candidate_pass(pgg, oracle_lib, kernel, L, segw):
    """Rows of more than 128 window words (a lane takes two words per pass,
    so these need two passes, the second for the last word or two): a whole
    periodic row of L = 4100, a 4064-column segment with a 32-column last one,
    and 4032-column segments of the paired kernel; two sweeps against the
    oracle."""
    r, seed, n = 3.9, 50 + L + segw, 2
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say(kernel, L, segw)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, tile=segw) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.mark.parametrize("group", [2, 4, 8])
def test_segment_workgroup_shapes(pgg, oracle_lib, group):
    """2, 4 or 8 segment waves per workgroup (the last workgroup padded with
    idle waves): same counts and lattice as the oracle."""
    L, r, seed, n = 196, 3.9, 70 + group, 10
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("segment group", group)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment", tile=64, group=group) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_segment_many_waves_out_of_place(pgg):
    """65 536 waves per launch (L = 4096, 64-column segments): waves start long
    after their neighbours have finished.  The segment update reads rows only
    from buffers that no wave of the same launch writes, so it must equal the
    row-band kernel (whole rows per workgroup) sweep for sweep."""
    L, r, seed, n = 4096, 3.7443, 17, 6
    say("segment 64-column segments at L=4096")
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment", tile=64) as a, \
            pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "rowband_compact") as b:
        for q in range(n):
            assert np.array_equal(a.sweep(1), b.sweep(1)), q
        assert np.array_equal(a.sweep(3), b.sweep(3))
        assert np.array_equal(a.read_lattice(), b.read_lattice())


def test_segment_plain_and_timing_graphs_agree(pgg, oracle_lib):
    """The segment kernel replays captured chunks of 64 sweeps and power-of-two
    tails; timing mode replays graphs of its own (draw counters, launch
    spans).  Calls of ragged lengths (odd, one, several chunks, a chunk and a
    tail) switch between the two on one lattice and must follow the oracle
    sweep for sweep; timing mode reports 4 launches per sweep."""
    L, r, K, p0, seed = 200, 3.8, 0.5, 0.5, 23
    lengths = [1, 63, 64, 65, 130, 3, 2]
    n = sum(lengths)
    ref, nc0, counts = oracle_lib.run(L, r, K, p0, seed, n)
    say("segment graph/eager switching", L, lengths)
    with pgg.Sim(L, r, K, p0, seed, "bits", "segment") as sim:
        got, timing = [], False
        for m in lengths:
            sim.set_kernel_timing(timing)
            got.append(sim.sweep(m))
            timing = not timing
        assert np.array_equal(np.concatenate(got), counts)
        assert np.array_equal(sim.read_lattice(), ref)
        assert sim.t == n
        sim.set_kernel_timing(True)
        sim.sweep(5)
        launches, ms, drawn = sim.kernel_timing()
        span_n, span_us = sim.kernel_span()
        assert launches == 20 and span_n == 20 and ms > 0.0 and span_us > 0.0
        assert 0 < drawn <= 5 * L * L


@pytest.mark.parametrize("L,group", [(64, 4), (96, 4), (128, 2), (160, 8), (256, 4), (512, 4), (1024, 4),
                                     (2048, 4)])
def test_whole_row_waves(pgg, oracle_lib, L, group):
    """Whole rows per wave (tile = L): several rows per wave below L = 1024,
    ragged last waves (L = 96, 160), pad words across the periodic wrap."""
    r, seed, n = 3.85, 90 + L, 9
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("whole rows", L, group)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment", tile=L, group=group) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_whole_rows_and_segments_agree_at_L1024(pgg):
    """L = 1024, 40 sweeps near r_c: whole rows (automatic), 512- and
    992-column segments give identical counts and lattices."""
    L, r, seed, n = 1024, 3.7443, 44, 40
    out = []
    for tile in (0, 512, 992):
        say("L=1024 tile", tile)
        with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment", tile=tile) as sim:
            out.append((sim.sweep(n), sim.read_lattice()))
    for c, lat in out[1:]:
        assert np.array_equal(c, out[0][0])
        assert np.array_equal(lat, out[0][1])


@pytest.mark.parametrize("L,tile", [(512, 0), (512, 448), (544, 96), (640, 576), (1024, 256), (2048, 0)])
def test_segment_pair_against_oracle(pgg, oracle_lib, L, tile):
    """Two residues per launch: bands of 32 rows with their halo rows, 12
    extra margin columns for the first residue; every sweep bit for bit,
    including segments that do not divide L and the last segment's wrap."""
    r, seed, n = 3.8, 300 + L + tile, 10
    s0, _ = oracle_lib.init(L, 0.5, seed)
    say("segment_pair", L, tile)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "segment_pair", tile=tile) as sim:
        ref = s0
        for t in range(n):
            ref, c = oracle_lib.sweep(ref, r, 0.5, seed, t, 1)
            assert int(sim.sweep(1)[0]) == int(c[0]), t
        assert np.array_equal(sim.read_lattice(), ref)
        sim.set_kernel_timing(True)
        sim.sweep(3)
        launches, ms, drawn = sim.kernel_timing()
        assert launches == 6 and sim.kernel_span()[0] == 6


@pytest.mark.parametrize("kernel", ["segment", "resident", "auto"])
def test_long_trajectory_whole_rows(pgg, oracle_lib, kernel):
    """L = 128 (segment: whole rows, 8 per wave; resident: the lattice in one
    workgroup's LDS) through 3000 sweeps near the transition: the count after
    every sweep and the final lattice equal the oracle's (the domains coarsen,
    so late sweeps exercise sparse activity)."""
    L, r, seed, n = 128, 3.9, 4242, 3000
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("long trajectory L=128", kernel, n)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel) as sim:
        got = np.concatenate([sim.sweep(1000), sim.sweep(1), sim.sweep(1999)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)


def _golden_decay():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "trajectory_L4096_r3.7443_seed1.txt")
    params, marks, counts = {}, {}, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            if key == "lattice":
                marks[int(rest[0])] = rest[1]
            elif key == "count":
                counts[int(rest[0])] = int(rest[1])
            else:
                params[key] = float(rest[0]) if key in ("r", "K", "p0") else int(rest[0])
    return params, marks, np.array([counts[t] for t in range(len(counts))], dtype=np.uint64)


def test_benchmark_workload_against_stored_oracle_trajectory(pgg):
    """The single-lattice benchmark workload (L = 4096, r = r_c, seed 1) in
    the kernel and launch configuration the benchmark times (the paired
    segment kernel, graph replays on a side stream, calls of 20 and then
    1000 sweeps): N_C after every one of the 1020 sweeps and the lattice
    after 20, 520 and 1020 sweeps equal the oracle's stored trajectory
    (tests/golden/make_trajectories.py)."""
    import hashlib
    import torch
    params, marks, counts = _golden_decay()
    L, r, K, p0, seed = params["L"], params["r"], params["K"], params["p0"], params["seed"]
    assert (L, r, seed) == (wl.DECAY["L"], wl.R_CRITICAL, 1)
    stream = torch.cuda.Stream()
    say("benchmark workload vs stored oracle trajectory, L", L, "sweeps", len(counts) - 1)

    def digest(sim):
        return hashlib.sha256(sim.read_lattice().tobytes()).hexdigest()

    with pgg.Sim(L, r, K, p0, seed, "bits", "segment_pair", stream=stream) as sim:
        assert sim.coop_count() == int(counts[0])
        got = [sim.sweep(20)]
        assert digest(sim) == marks[20]
        got += [sim.sweep(500)]
        assert digest(sim) == marks[520]
        got += [sim.sweep(500)]
        assert digest(sim) == marks[1020]
        got = np.concatenate(got)
        bad = np.flatnonzero(got != counts[1:])
        assert bad.size == 0, "first differing sweep %d" % (bad[0] + 1 if bad.size else -1)



def test_decay_driver_matches_oracle(pgg, oracle_lib):
    """observables.decay (one lattice, counts fetched in blocks, rho_C on the
    log grid) equals the same grid read off the oracle's counts."""
    from paper_1704_08098_amd import observables as ob
    L, r, seed, n = 256, wl.R_CRITICAL, 3, 500
    ref, nc0, counts = oracle_lib.run(L, r, 0.5, 0.5, seed, n)
    say("decay driver, L", L, "t_max", n)
    grid, rho = ob.decay(pgg, L, r, seed, n, block=128)
    assert np.array_equal(rho, ob.sample_on_grid(counts, L, grid, nc0))


# ---------------------------------------------------------------------------
# The double tiling of Sec. IV (schedule "tiled") against oracle C.

TILED_CASES = [(8, 3.8, 0.5, 31), (16, 4.4, 0.5, 32), (40, 3.9, 0.5, 33), (64, 3.75, 0.1, 34),
               (72, 5.0, 1.5, 2**40 + 35), (96, 3.98, 0.5, 36), (128, 3.85, 0.5, 37)]


@pytest.mark.parametrize("L,r,K,seed", TILED_CASES, ids=lambda v: str(v))
def test_tiled_every_sweep_against_oracle(pgg, oracle_lib, L, r, K, seed):
    """Tiny to mid-size lattices (L % 8 == 0, also not a multiple of 32):
    lattice and count after every Monte Carlo step, bit for bit."""
    n = 20
    say("tiled", L, r, K, seed)
    s0, nc0 = oracle_lib.init(L, 0.5, seed)
    with pgg.Sim(L, r, K, 0.5, seed, "bits", schedule="tiled") as sim:
        assert sim.coop_count() == nc0
        ref = s0
        for t in range(n):
            ref, c = oracle_lib.sweep_tiled(ref, r, K, seed, t, 1)
            assert int(sim.sweep(1)[0]) == int(c[0]), t
            assert np.array_equal(sim.read_lattice(), ref), t


def test_tiled_long_run_against_oracle(pgg, oracle_lib):
    """L = 256 through 400 steps near the transition, calls of uneven length."""
    L, r, seed, n = 256, 3.74, 41, 400
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep_tiled(s0, r, 0.5, seed, 0, n)
    say("tiled long run", L, n)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", schedule="tiled") as sim:
        got = np.concatenate([sim.sweep(1), sim.sweep(150), sim.sweep(249)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_tiled_L4096_against_oracle(pgg, oracle_lib):
    """The benchmark size: two tiled steps of the L = 4096 lattice at r_c."""
    L, r, seed = 4096, wl.R_CRITICAL, 1
    s0, nc0 = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep_tiled(s0, r, 0.5, seed, 0, 2)
    say("tiled L=4096")
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", schedule="tiled") as sim:
        assert sim.coop_count() == nc0
        assert np.array_equal(sim.sweep(2), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_tiled_resume_and_sweep_index_near_2_pow_32(pgg, oracle_lib):
    L, r, K, seed = 48, 3.9, 0.5, 77
    lat = wl.random_lattice(L, 0.4, 6)
    t0 = 2**32 - 5
    ref, counts = oracle_lib.sweep_tiled(lat, r, K, seed, t0, 5)
    say("tiled resume near 2^32")
    with pgg.Sim(L, r, K, 0.5, seed, "bits", schedule="tiled") as sim:
        sim.write_lattice(lat, t0)
        got = np.concatenate([sim.sweep(2), sim.sweep(0), sim.sweep(3)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)
        with pytest.raises(pgg.PggError):
            sim.sweep(1)


@pytest.mark.parametrize("value", [0, 1])
def test_tiled_absorbing_states_stay(pgg, value):
    say("tiled absorbing", value)
    with pgg.Sim(64, 3.8, 0.5, float(value), 3, "bits", schedule="tiled") as sim:
        assert np.all(sim.sweep(10) == value * 64 * 64)
        assert np.all(sim.read_lattice() == value)


@pytest.mark.parametrize("L", [8, 64, 136])
def test_tiled_int8_layout_against_oracle(pgg, oracle_lib, L):
    """The tiled schedule on the int8 layout (a bit-packed working copy):
    every step bit for bit, calls of several lengths, a written lattice."""
    r, seed = 3.9, 60 + L
    s0, nc0 = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep_tiled(s0, r, 0.5, seed, 0, 12)
    say("tiled int8", L)
    with pgg.Sim(L, r, 0.5, 0.5, seed, "int8", schedule="tiled") as sim:
        assert sim.coop_count() == nc0
        got = np.concatenate([sim.sweep(1), sim.sweep(4), sim.sweep(7)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)
        lat = wl.random_lattice(L, 0.6, 3)
        ref2, counts2 = oracle_lib.sweep_tiled(lat, r, 0.5, seed, 30, 5)
        sim.write_lattice(lat, 30)
        assert np.array_equal(sim.sweep(5), counts2)
        assert np.array_equal(sim.read_lattice(), ref2)


def test_tiled_maximum_size_count_is_a_recount(pgg):
    """L = 32768 (the largest accepted; 16.8 M domains per type): two tiled
    steps in a caller buffer; the running count equals a popcount of the
    device lattice, and the lattice changed."""
    import torch
    L, r, seed = 32768, 3.98, 9
    params = pgg.make_params(L, r, 0.5, 0.5, seed, "bits", schedule="tiled")
    buf = torch.empty(pgg.pgg_device_bytes(params), dtype=torch.uint8, device="cuda")
    say("tiled L=32768")
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", dev_buf=buf, schedule="tiled") as sim:
        nc0 = sim.coop_count()
        before = buf.clone()
        c = sim.sweep(2)
    torch.cuda.synchronize()
    pop = int(np.bitwise_count(buf.cpu().numpy()).sum(dtype=np.uint64))
    assert pop == int(c[-1])
    assert not torch.equal(before, buf) and int(c[-1]) != nc0


def test_plan_reports_what_init_runs(pgg):
    """pgg_plan resolves AUTO and the work split as pgg_init does."""
    mk = pgg.make_params
    assert pgg.pgg_plan(mk(4096, 3.7443, kernel="segment_pair")) == ("segment_pair", 2048)
    assert pgg.pgg_plan(mk(4096, 3.7443)) == ("segment_pair", 2048)
    assert pgg.pgg_plan(mk(4096, 3.7443, kernel="segment_pair", tile=1024)) == ("segment_pair", 1024)
    assert pgg.pgg_plan(mk(128, 3.8)) == ("resident", 8)
    assert pgg.pgg_plan(mk(96, 3.8)) == ("resident", 4)
    assert pgg.pgg_plan(mk(100, 3.8)) == ("segment", 100)  # one periodic row per wave
    assert pgg.pgg_plan(mk(2048, 3.8)) == ("segment", 1024)
    assert pgg.pgg_plan(mk(256, 3.8, schedule="tiled")) == ("auto", 0)
    assert pgg.pgg_plan(mk(256, 1.05, game="pd")) == ("auto", 0)

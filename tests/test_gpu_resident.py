"""GPU parity of the resident kernel (one workgroup keeps the lattice in LDS
and runs a whole chunk of sweeps per launch) against the oracle: the
16-colour sweep of the Sec. III elementary step with the Eq. (3) Fermi rule,
lattice and Eq. (4) count after every sweep, bit-exact.

Every GPU step prints what it runs before it runs.
"""
import numpy as np
import pytest

from paper_1704_08098_amd import workloads as wl

pytestmark = pytest.mark.gpu

SIZES = [64, 96, 160, 256]  # multiples of 32 in [64, 256]; 96 and 160 leave rows of the residues on few waves


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


@pytest.mark.parametrize("layout", ["bits", "int8"])
@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("r,K,seed", [(3.8, 0.5, 1), (4.6, 0.1, 7)])
def test_every_sweep_against_oracle(pgg, oracle_lib, layout, L, r, K, seed):
    n = 16
    say("resident every sweep", layout, "L", L, "r", r, "K", K, "seed", seed)
    ref, _ = oracle_lib.init(L, 0.5, seed)
    with pgg.Sim(L, r, K, 0.5, seed, layout, "resident") as sim:
        assert np.array_equal(sim.read_lattice(), ref)
        for t in range(n):
            ref, c = oracle_lib.sweep(ref, r, K, seed, t, 1)
            got = sim.sweep(1)
            assert int(got[0]) == int(c[0]), t
            assert np.array_equal(sim.read_lattice(), ref), t


@pytest.mark.parametrize("group", [4, 8, 16])
@pytest.mark.parametrize("L", [64, 160, 256, 288, 512])
def test_wave_counts(pgg, oracle_lib, L, group):
    """Every workgroup shape (4, 8 or 16 waves, so 1 to 16 rows of a residue
    per wave) gives the oracle's lattice and count after every sweep."""
    r, K, seed, n = 3.76, 0.5, 31, 40
    say("resident waves", group, "L", L)
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep(s0, r, K, seed, 0, n)
    with pgg.Sim(L, r, K, 0.5, seed, "bits", "resident", group=group) as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.mark.parametrize("layout", ["bits", "int8"])
@pytest.mark.parametrize("L", [64, 256])
def test_one_launch_many_sweeps(pgg, oracle_lib, layout, L):
    """Counts after every sweep of a multi-sweep launch, and the final lattice."""
    r, K, seed, n = 3.75, 0.5, 11, 300
    say("resident one call", layout, "L", L, "sweeps", n)
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep(s0, r, K, seed, 0, n)
    with pgg.Sim(L, r, K, 0.5, seed, layout, "resident") as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_calls_longer_than_one_chunk(pgg, oracle_lib):
    """A call of more sweeps than one launch holds (4096) splits into launches."""
    L, r, K, seed, n = 64, 3.9, 0.5, 5, 5000
    say("resident chunks", "L", L, "sweeps", n)
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref, counts = oracle_lib.sweep(s0, r, K, seed, 0, n)
    with pgg.Sim(L, r, K, 0.5, seed, "bits", "resident") as sim:
        assert np.array_equal(sim.sweep(n), counts)
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.mark.parametrize("layout", ["bits", "int8"])
def test_write_lattice_resume_and_chunking(pgg, oracle_lib, layout):
    L, r, K, seed, t0 = 128, 3.9, 0.5, 77, 123
    lat = wl.random_lattice(L, 0.4, 5)
    ref, counts = oracle_lib.sweep(lat, r, K, seed, t0, 30)
    say("resident resume", layout)
    with pgg.Sim(L, r, K, 0.5, seed, layout, "resident") as sim:
        sim.write_lattice(lat, t0)
        assert sim.t == t0 and sim.coop_count() == int(lat.sum())
        got = np.concatenate([sim.sweep(7), sim.sweep(0), sim.sweep(13), sim.sweep(10)])
        assert np.array_equal(got, counts)
        assert np.array_equal(sim.read_lattice(), ref)
        assert sim.t == t0 + 30


def test_sweep_index_near_2_pow_32(pgg, oracle_lib):
    L, r, seed = 96, 3.8, 9
    lat, _ = oracle_lib.init(L, 0.5, seed)
    t0 = 2**32 - 3
    ref, counts = oracle_lib.sweep(lat, r, 0.5, seed, t0, 3)
    say("resident t near 2^32")
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", "resident") as sim:
        sim.write_lattice(lat, t0)
        assert np.array_equal(sim.sweep(3), counts)
        assert np.array_equal(sim.read_lattice(), ref)
        with pytest.raises(pgg.PggError) as e:
            sim.sweep(1)
        assert e.value.status == pgg.PGG_E_INVAL
        assert sim.t == 2**32


@pytest.mark.parametrize("value", [0, 1])
def test_absorbing_states_stay(pgg, value):
    say("resident absorbing", value)
    with pgg.Sim(128, 3.8, 0.5, float(value), 3, "bits", "resident") as sim:
        c = sim.sweep(20)
        assert np.all(c == value * 128 * 128)
        assert np.all(sim.read_lattice() == value)


def test_agrees_with_whole_row_kernel_and_counts_the_same_draws(pgg):
    """Same trajectory as the whole-row segment kernel over a long run, and the
    same number of updates that drew random numbers (both draw exactly for the
    sites with a differing neighbour)."""
    L, r, seed, n = 256, 3.74, 21, 2000
    say("resident vs whole rows", "L", L, "sweeps", n)
    out = {}
    for kernel, tile in (("resident", 0), ("segment", L)):
        with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, tile=tile) as sim:
            sim.set_kernel_timing(True)
            counts = sim.sweep(n)
            launches, ms, drawn = sim.kernel_timing()
            assert launches > 0 and ms > 0
            out[kernel] = (counts, sim.read_lattice(), drawn)
    assert np.array_equal(out["resident"][0], out["segment"][0])
    assert np.array_equal(out["resident"][1], out["segment"][1])
    assert out["resident"][2] == out["segment"][2] > 0


def test_lattices_on_concurrent_streams(pgg, oracle_lib):
    """Eight host threads, each with a stream of its own, run resident and
    whole-row lattices side by side; every lattice matches the oracle."""
    import threading
    import torch
    jobs = [(L, kernel, r, seed) for seed, (L, kernel, r) in enumerate(
        [(64, "resident", 3.8), (128, "resident", 3.76), (256, "resident", 4.2), (96, "resident", 3.9),
         (64, "segment", 3.8), (128, "segment", 3.76), (256, "auto", 4.2), (160, "resident", 3.72)], start=40)]
    n = 200
    refs = {}
    for L, kernel, r, seed in jobs:
        s0, _ = oracle_lib.init(L, 0.5, seed)
        refs[seed] = oracle_lib.sweep(s0, r, 0.5, seed, 0, n)
    got, errors = {}, []

    def work(L, kernel, r, seed):
        try:
            st = torch.cuda.Stream()
            with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", kernel, stream=st) as sim:
                c = np.concatenate([sim.sweep(70), sim.sweep(130)])
                got[seed] = (c, sim.read_lattice())
        except Exception as exc:  # reported after the join
            errors.append(exc)

    say("resident concurrent streams", len(jobs), "lattices")
    threads = [threading.Thread(target=work, args=j) for j in jobs]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for L, kernel, r, seed in jobs:
        ref_lat, ref_counts = refs[seed]
        assert np.array_equal(got[seed][0], ref_counts), (L, kernel)
        assert np.array_equal(got[seed][1], ref_lat), (L, kernel)

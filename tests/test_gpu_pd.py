"""GPU parity of the pairwise prisoner's dilemma (the game Sec. VI names for
the same scheme) against oracle D: lattice and cooperator count after every
sweep, bit for bit, for both storage layouts, lattices from L = 4 (periodic
wrap inside one word) through ragged word tails to L = 4096."""
import numpy as np
import pytest

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


CASES = [(4, 1.5, 0.5, 1, 12), (8, 1.05, 0.1, 2, 12), (12, 1.3, 0.5, 3, 10), (36, 1.05, 0.1, 4, 10),
         (100, 1.5, 0.5, 5, 10), (132, 1.05, 0.1, 6, 8), (260, 1.9, 0.5, 7, 6), (512, 1.05, 0.1, 8, 4)]


@pytest.mark.parametrize("layout", ["bits", "int8"])
@pytest.mark.parametrize("L,b,K,seed,n", CASES)
def test_every_sweep_matches_oracle(pgg, oracle_lib, layout, L, b, K, seed, n):
    say("pairwise game", layout, "L", L, "b", b, "K", K, "seed", seed, "sweeps", n)
    s, nc0 = oracle_lib.init(L, 0.5, seed)
    with pgg.Sim(L, b, K, 0.5, seed, layout, game="pd") as sim:
        assert sim.coop_count() == nc0
        assert np.array_equal(sim.threshold_table().reshape(-1)[:50], oracle_lib.pd_table(b, K).reshape(-1))
        for t in range(n):
            s, c = oracle_lib.pd_sweep(s, b, K, seed, t, 1)
            got = sim.sweep(1)
            assert got[0] == c[0], "count differs after sweep %d" % (t + 1)
            assert np.array_equal(sim.read_lattice(), s), "lattice differs after sweep %d" % (t + 1)


def test_large_lattice_two_sweeps(pgg, oracle_lib):
    L, b, K, seed = 4096, 1.05, 0.1, 11
    say("pairwise game L", L, "2 sweeps")
    ref, nc0, counts = oracle_lib.pd_run(L, b, K, 0.5, seed, 2)
    with pgg.Sim(L, b, K, 0.5, seed, "bits", game="pd") as sim:
        assert sim.coop_count() == nc0
        assert np.array_equal(sim.sweep(2), counts)
        assert np.array_equal(sim.read_lattice(), ref)


def test_chunking_resume_and_sweep_index(pgg, oracle_lib):
    L, b, K, seed = 68, 1.3, 0.5, 21
    say("pairwise game chunking/resume L", L)
    ref, _, counts = oracle_lib.pd_run(L, b, K, 0.5, seed, 15)
    with pgg.Sim(L, b, K, 0.5, seed, "bits", game="pd") as sim:
        got = np.concatenate([sim.sweep(4), sim.sweep(1), sim.sweep(10)])
        assert np.array_equal(got, counts) and sim.t == 15
        assert np.array_equal(sim.read_lattice(), ref)
    # resume from a lattice written at t = 7 (checkpoint / restore)
    s7, _ = oracle_lib.pd_sweep(oracle_lib.init(L, 0.5, seed)[0], b, K, seed, 0, 7)
    with pgg.Sim(L, b, K, 0.5, seed, "bits", game="pd") as sim:
        sim.write_lattice(s7, 7)
        assert np.array_equal(sim.sweep(8), counts[7:])
        assert np.array_equal(sim.read_lattice(), ref)


@pytest.mark.parametrize("value", [0, 1])
def test_absorbing_states(pgg, value):
    L = 64
    say("pairwise game absorbing", value)
    with pgg.Sim(L, 1.5, 0.5, float(value), 3, "bits", game="pd") as sim:
        assert np.all(sim.sweep(5) == value * L * L)
        assert np.all(sim.read_lattice() == value)


def test_refused_where_it_does_not_apply(pgg):
    for kw in (dict(kernel="segment"), dict(schedule="tiled"), dict(tile=32, kernel="segment")):
        with pytest.raises(pgg.PggError) as e:
            pgg.Sim(64, 1.5, 0.5, 0.5, 1, "bits", game="pd", **kw)
        assert e.value.status == pgg.PGG_E_INVAL
    with pytest.raises(pgg.PggError):
        pgg.Ensemble([dict(L=64, r=1.5, K=0.5, p0=0.5, seed=1, game="pd")])

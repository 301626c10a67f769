"""Host-side observables of the cooperator count (Eq. (4)): definitions on
hand-made count histories, and the experiment drivers' marshalling with a
stand-in engine (no GPU)."""
import numpy as np
import pytest

from paper_1704_08098_amd import observables as ob
from paper_1704_08098_amd import workloads as wl


def test_density_series_divides_by_the_site_count():
    assert np.array_equal(ob.density_series([0, 2, 4], 2), [0.0, 0.5, 1.0])


def test_stationary_density_is_the_mean_over_the_last_sweeps():
    counts = np.array([0, 1, 2, 3, 4], dtype=np.uint64)  # L = 2: 4 sites
    assert ob.stationary_density(counts, 2, 2) == (3 + 4) / (2 * 4)
    assert ob.stationary_density(counts, 2, 5) == 10 / 20
    # exact integer sum: 10^4 sweeps of an all-C L = 32768 lattice
    big = np.full(10_000, 32768 * 32768, dtype=np.uint64)
    assert ob.stationary_density(big, 32768, 5000) == 1.0
    with pytest.raises(ValueError):
        ob.stationary_density(counts, 2, 6)
    with pytest.raises(ValueError):
        ob.stationary_density(counts, 2, 0)


def test_sample_on_grid_reads_the_count_after_each_sweep():
    counts = np.array([10, 20, 30, 40], dtype=np.uint64)  # after sweeps 1..4, L = 10
    assert np.array_equal(ob.sample_on_grid(counts, 10, [0, 1, 4], nc0=5), [0.05, 0.1, 0.4])
    with pytest.raises(ValueError):
        ob.sample_on_grid(counts, 10, [5])
    with pytest.raises(ValueError):
        ob.sample_on_grid(counts, 10, [0])


def test_log_time_grid_is_increasing_and_bounded():
    g = wl.log_time_grid(100_000)
    assert g[0] == 1 and g[-1] == 100_000
    assert np.all(np.diff(g) > 0)
    # 20 points per decade once rounding no longer merges them: 10^3 .. 10^5
    assert np.count_nonzero((g >= 1000) & (g <= 100_000)) == 41


class _FakeEnsemble:
    """Replica k's count after sweep t (1-based) is 100 k + t."""

    def __init__(self, reps, chunk=64, stream=None):
        self.reps, self.t = reps, 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False

    def sweep(self, m):
        t = np.arange(self.t + 1, self.t + m + 1, dtype=np.uint64)
        self.t += m
        return np.stack([100 * k + t for k in range(len(self.reps))])


class _FakeSim:
    def __init__(self, L, r, K, p0, seed, layout, kernel, stream=None):
        self.t = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False

    def coop_count(self):
        return 7

    def sweep(self, m):
        t = np.arange(self.t + 1, self.t + m + 1, dtype=np.uint64)
        self.t += m
        return t * 3


class _FakePgg:
    Ensemble = _FakeEnsemble
    Sim = _FakeSim


def test_r_scan_concatenates_blocks_and_averages_per_replica():
    cfg = dict(wl.SCAN, L=10, sweeps=25, average_last=10)
    r, rho, counts = ob.r_scan(_FakePgg, cfg, block=7)
    assert counts.shape == (21, 25)
    assert np.array_equal(counts[3], 300 + np.arange(1, 26))
    # mean of 100 k + t over t = 16..25 is 100 k + 20.5, over 100 sites
    assert np.allclose(rho, (100 * np.arange(21) + 20.5) / 100, rtol=0, atol=1e-15)
    assert np.array_equal(r, cfg["r_values"])


def test_decay_samples_the_log_grid():
    grid, rho = ob.decay(_FakePgg, 10, 3.7, 1, 120, block=50)
    assert np.array_equal(grid, wl.log_time_grid(120)[wl.log_time_grid(120) <= 120])
    assert np.allclose(rho, 3 * grid / 100.0, rtol=0, atol=1e-15)


def test_r_scan_lattices_runs_every_replica_once(monkeypatch):
    """One lattice per r on worker threads: every count row filled from its
    own lattice, whatever thread ran it."""
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "Stream", lambda: None)
    seen = []

    class Sim(_FakeSim):
        def __init__(self, L, r, K, p0, seed, layout, kernel, stream=None, schedule="colour16"):
            super().__init__(L, r, K, p0, seed, layout, kernel, stream)
            seen.append((r, seed, schedule))
            self.base = seed

        def sweep(self, m):
            t = np.arange(self.t + 1, self.t + m + 1, dtype=np.uint64)
            self.t += m
            return t + np.uint64(1000 * self.base)

    class Fake:
        pass

    Fake.Sim = Sim
    cfg = dict(wl.SCAN, L=10, sweeps=30, average_last=10)
    r, rho, counts = ob.r_scan_lattices(Fake, cfg, schedule="tiled", workers=3, block=7)
    assert sorted(seen) == sorted((rv, s, "tiled") for rv, s in zip(cfg["r_values"], cfg["seeds"]))
    for k, s in enumerate(cfg["seeds"]):
        assert np.array_equal(counts[k], 1000 * s + np.arange(1, 31))

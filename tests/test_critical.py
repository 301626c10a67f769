"""Critical-point fit (Sec. V, rho_C ~ (r - r_c)^beta) on synthetic data
with known r_c and beta (no GPU)."""
import numpy as np
import pytest

from paper_1704_08098_amd import critical as cr


def test_power_law_fit_recovers_an_exact_power_law():
    r = np.linspace(3.73, 3.80, 15)
    rho = 0.9 * (r - 3.72) ** 0.584
    beta, icpt, msr, n = cr.fit_power_law(r, rho, 3.72)
    assert beta == pytest.approx(0.584, abs=1e-12)
    assert np.exp(icpt) == pytest.approx(0.9, rel=1e-12)
    assert msr < 1e-24 and n == 15


def test_power_law_fit_needs_three_points_above_r_c():
    assert cr.fit_power_law([3.70, 3.71, 3.75], [0.0, 0.0, 0.1], 3.72) is None


def test_critical_point_fit_finds_r_c_and_beta():
    r_c, beta = 3.7213, 0.58
    r = np.round(np.arange(3.700, 3.8001, 0.0025), 6)
    rho = np.where(r > r_c, 0.85 * np.clip(r - r_c, 0, None) ** beta, 0.0)
    grid = np.arange(r[rho > 0].min() - 0.03, r[rho > 0].min(), 0.0001)
    rc_fit, beta_fit, msr, n = cr.fit_critical_point(r, rho, grid)
    assert rc_fit == pytest.approx(r_c, abs=1.5e-4)
    assert beta_fit == pytest.approx(beta, abs=0.01)


def test_critical_point_fit_with_noise_stays_close():
    rng = np.random.default_rng(3)
    r_c, beta = 3.7213, 0.58
    r = np.round(np.arange(3.700, 3.8001, 0.0025), 6)
    rho = np.where(r > r_c, 0.85 * np.clip(r - r_c, 0, None) ** beta, 0.0)
    rho = rho * np.exp(rng.normal(0, 0.01, rho.size))
    grid = np.arange(r[rho > 0].min() - 0.03, r[rho > 0].min(), 0.0001)
    rc_fit, beta_fit, _, _ = cr.fit_critical_point(r, rho, grid)
    assert abs(rc_fit - r_c) < 1e-3 and abs(beta_fit - beta) < 0.05


def test_stationary_points_flags_decaying_and_extinct_runs():
    L, n, last = 10, 400, 200
    flat = np.full(n, 40, dtype=np.uint64)                        # rho = 0.4 throughout
    decaying = np.linspace(60, 10, n).round().astype(np.uint64)   # still falling
    extinct = np.zeros(n, dtype=np.uint64)
    rho, ok = cr.stationary_points(np.stack([flat, decaying, extinct]), L, last)
    assert ok.tolist() == [True, False, False]
    assert rho[0] == pytest.approx(0.4)

"""Pins for the Fermi acceptance table (Sec. III, Eq. (3))."""
import mpmath
import numpy as np
import pytest

mpmath.mp.dps = 60
TWO32 = 2**32

# r values used by the workloads: L=100 run (3.8), the r scan 3.70..3.80 in
# steps of 0.005, the critical point r_c = 3.7443 and r_c +- 0.005 (Sec. V,
# Fig. 4), the Fig. 5 timing point 3.98, plus the pair-interaction bound r = G.
R_VALUES = sorted({3.8, 3.98, 3.7393, 3.7443, 3.7493, 5.0, 4.37}
                  | {float("%.3f" % (3.70 + 0.005 * i)) for i in range(21)})


def _exact_T(r, K, dsig, ds):
    # Pi_x - Pi_y = (r/5) dSigma - 5 ds with r, K taken as their exact binary64 values.
    dpi = mpmath.mpf(r) * dsig / 5 - 5 * ds
    w = 1 / (1 + mpmath.exp(dpi / mpmath.mpf(K)))
    return min(int(mpmath.floor(w * TWO32 + mpmath.mpf(1) / 2)), TWO32 - 1), w


@pytest.mark.parametrize("r", R_VALUES)
def test_table_is_exactly_rounded(oracle_lib, r):
    T = oracle_lib.table(r, 0.5)
    for dsig in range(-25, 26):
        for ds in (-1, 0, 1):
            exact, _ = _exact_T(r, 0.5, dsig, ds)
            assert int(T[dsig + 25, ds + 1]) == exact, (r, dsig, ds)


def test_table_symmetry_and_midpoint(oracle_lib):
    # W(-z) = 1 - W(z): T(dSigma, ds) + T(-dSigma, -ds) = 2^32 unless clamped.
    for r in (3.8, 3.7443, 4.9):
        T = oracle_lib.table(r, 0.5).astype(np.int64)
        assert T[25, 1] == 2**31  # dSigma = ds = 0: W = 1/2 exactly
        for dsig in range(-25, 26):
            for ds in (-1, 0, 1):
                tot = T[dsig + 25, ds + 1] + T[-dsig + 25, -ds + 1]
                assert tot in (TWO32, TWO32 - 1)


def test_table_monotone(oracle_lib):
    # A larger own-payoff advantage (larger dSigma at r > 0) lowers the chance
    # to copy; becoming a cooperator (ds = -1) is less attractive than staying
    # for equal dSigma, since the cooperator pays the cost in 5 groups.
    T = oracle_lib.table(3.8, 0.5).astype(np.int64)
    for ds in range(3):
        assert np.all(np.diff(T[:, ds]) <= 0)
    assert np.all(T[:, 0] <= T[:, 1]) and np.all(T[:, 1] <= T[:, 2])


def test_lone_cooperator_copying_defector_neighbour(oracle_lib):
    # Hand-worked payoffs (r = 3.8): lone C earns r - 5 = -1.2, its D neighbour
    # 2r/5 = 1.52, so W = 1/(1 + exp(-2.72/0.5)).  Sigma_x = 5, Sigma_y = 2.
    w = 1 / (1 + mpmath.exp(mpmath.mpf("-2.72") / mpmath.mpf("0.5")))
    T = oracle_lib.table(3.8, 0.5)
    assert abs(int(T[3 + 25, 2]) - float(w * TWO32)) < 2.0
    # and the D neighbour copying the lone C: W = 1/(1 + exp(+2.72/0.5)).
    w2 = 1 / (1 + mpmath.exp(mpmath.mpf("2.72") / mpmath.mpf("0.5")))
    assert abs(int(T[-3 + 25, 0]) - float(w2 * TWO32)) < 2.0


def test_small_K_limit(oracle_lib):
    # Sec. III: K -> 0, x copies y iff Pi_y > Pi_x (ties stay at 1/2).
    r = 3.8
    T = oracle_lib.table(r, 1e-3)
    for dsig in range(-25, 26):
        for ds in (-1, 0, 1):
            dpi = r * dsig / 5 - 5 * ds
            v = int(T[dsig + 25, ds + 1])
            if abs(dpi) < 1e-12:
                assert v == 2**31
            elif dpi < 0:
                assert v == TWO32 - 1
            else:
                assert v == 0


def test_large_K_limit(oracle_lib):
    # Sec. III: K -> infinity, payoffs cease to matter (coin flip).  |dPi| <= 30,
    # so |W - 1/2| <= 30/(4K) and 2^32 |W - 1/2| < 1 for K = 1e12.
    T = oracle_lib.table(3.8, 1e12).astype(np.int64)
    assert np.all(np.abs(T - 2**31) <= 1)


@pytest.mark.parametrize("bad", [(3.8, 0.0), (3.8, -1.0), (float("nan"), 0.5),
                                 (3.8, float("inf")), (-1.0, 0.5)])
def test_table_rejects_bad_parameters(oracle_lib, bad):
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.table(*bad)

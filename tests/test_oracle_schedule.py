"""Pins for the oracle's 16-colour sweep: schedule, invariants, brute force."""
import numpy as np
import pytest

import exact_ref


def _colour(i, j):
    return 4 * (i % 4) + (j % 4)


@pytest.mark.parametrize("L", [4, 8, 12, 16, 20, 100])
def test_colouring_is_race_free(L):
    # A site's update reads the strategies of the radius-3 diamond around it
    # (its own two payoff groups rings plus those of the chosen neighbour,
    # Sec. IV, three lines outward).  No other site of the same colour may
    # lie in that read set, with periodic wrap, or concurrent updates race.
    offs = [(a, b) for a in range(-3, 4) for b in range(-3, 4) if 0 < abs(a) + abs(b) <= 3]
    for i in range(L):
        for j in range(L):
            k = _colour(i, j)
            for a, b in offs:
                yi, yj = (i + a) % L, (j + b) % L
                if (yi, yj) != (i, j):
                    assert _colour(yi, yj) != k


def test_order_inside_a_colour_does_not_matter(oracle_lib):
    s0, _ = oracle_lib.init(20, 0.5, 11)
    ref, cref = oracle_lib.sweep(s0, 3.9, 0.5, 11, 0, 30, order=0)
    for order, oseed in ((1, 0), (2, 5), (2, 77)):
        got, c = oracle_lib.sweep(s0, 3.9, 0.5, 11, 0, 30, order=order, order_seed=oseed)
        assert np.array_equal(got, ref)
        assert np.array_equal(c, cref)


@pytest.mark.parametrize("value", [0, 1])
def test_absorbing_states(oracle_lib, value):
    # All-C and all-D admit no change: every neighbour copies an equal
    # strategy (the C+D -> D transition ends in an absorbing state, Sec. V).
    L = 16
    s0 = np.full((L, L), value, dtype=np.uint8)
    for r, K, seed in ((3.8, 0.5, 1), (2.0, 0.1, 2), (6.0, 3.0, 3)):
        s, c = oracle_lib.sweep(s0, r, K, seed, 5, 10)
        assert np.array_equal(s, s0)
        assert np.all(c == value * L * L)


def test_chunking_does_not_matter(oracle_lib):
    s0, _ = oracle_lib.init(24, 0.5, 9)
    whole, cw = oracle_lib.sweep(s0, 3.85, 0.5, 9, 0, 12)
    a, ca = oracle_lib.sweep(s0, 3.85, 0.5, 9, 0, 5)
    b, cb = oracle_lib.sweep(a, 3.85, 0.5, 9, 5, 7)
    assert np.array_equal(whole, b)
    assert np.array_equal(cw, np.concatenate([ca, cb]))


def test_counts_are_recounts(oracle_lib):
    s0, nc0 = oracle_lib.init(32, 0.5, 4)
    assert nc0 == int(s0.sum())
    s, c = oracle_lib.sweep(s0, 3.8, 0.5, 4, 0, 3)
    assert c[-1] == int(s.sum())


def test_init_fractions(oracle_lib):
    L = 64
    assert oracle_lib.init(L, 0.0, 3)[1] == 0
    assert oracle_lib.init(L, 1.0, 3)[1] == L * L
    for p0 in (0.1, 0.5, 0.9):
        n = oracle_lib.init(L, p0, 3)[1]
        sd = (L * L * p0 * (1 - p0)) ** 0.5
        assert abs(n - p0 * L * L) < 5 * sd


@pytest.mark.parametrize("L,r,seed,n", [(4, 3.8, 1, 6), (8, 3.8, 2, 4), (8, 4.4, 0x1234567890, 3),
                                        (12, 3.72, 5, 2), (16, 4.9, 6, 2)])
def test_sweep_matches_exact_brute_force(oracle_lib, rocrand_philox, L, r, seed, n):
    """Oracle A vs a literal, exact-arithmetic re-statement on tiny lattices."""
    K = 0.5
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref = [list(map(int, row)) for row in s0]
    for t in range(n):
        words = rocrand_philox(exact_ref.sweep_counters(L, t, seed))
        exact_ref.sweep(ref, L, r, K, words)
    got, _ = oracle_lib.sweep(s0, r, K, seed, 0, n)
    assert np.array_equal(got, np.array(ref, dtype=np.uint8))
    # a run that changes nothing would pass trivially: require some flips
    assert not np.array_equal(got, s0)


@pytest.mark.parametrize("L", [0, 2, 6, 10, 32772])
def test_rejects_bad_L(oracle_lib, L):
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.init(L, 0.5, 1)


def test_rejects_bad_p0(oracle_lib):
    for p0 in (-0.1, 1.1, float("nan")):
        with pytest.raises(oracle_lib.OracleError):
            oracle_lib.init(8, p0, 1)


# ---------------------------------------------------------------------------
# Oracle C: the double tiling of Sec. IV.

def _domain_type(I, J):
    return 2 * (I % 2) + (J % 2)


@pytest.mark.parametrize("L", [16, 24, 32, 40])
def test_tiling_domains_of_one_type_are_independent(L):
    # A step of a domain writes only the domain and reads at most 3 sites
    # (L1 distance) beyond it (x's groups and those of its neighbour y,
    # Sec. IV "three lines outward").  No other domain of the same type may
    # lie in that read set, with periodic wrap.
    n = L // 4
    offs = [(a, b) for a in range(-3, 4) for b in range(-3, 4) if abs(a) + abs(b) <= 3]
    owner = {}
    for I in range(n):
        for J in range(n):
            for a in range(4):
                for b in range(4):
                    owner[(4 * I + a, 4 * J + b)] = (I, J)
    for I in range(n):
        for J in range(n):
            reads = {((4 * I + a + da) % L, (4 * J + b + db) % L)
                     for a in range(4) for b in range(4) for da, db in offs}
            for site in reads:
                D = owner[site]
                if D != (I, J):
                    assert _domain_type(*D) != _domain_type(I, J), (L, I, J, D)


def test_tiling_types_cover_the_lattice_once_per_step():
    # four parts, one per type; every domain belongs to exactly one type and
    # the types alternate 1,2,1,2 / 3,4,3,4 along rows of domains (Fig. 2)
    n = 6
    types = [[_domain_type(I, J) for J in range(n)] for I in range(n)]
    assert types[0][:4] == [0, 1, 0, 1] and types[1][:4] == [2, 3, 2, 3]
    assert sorted(sum(types, [])) == sorted([0, 1, 2, 3] * (n * n // 4))


def test_tiled_domain_order_does_not_matter(oracle_lib):
    s0, _ = oracle_lib.init(24, 0.5, 12)
    ref, cref = oracle_lib.sweep_tiled(s0, 3.9, 0.5, 12, 0, 25, order=0)
    for order, oseed in ((1, 0), (2, 5), (2, 91)):
        got, c = oracle_lib.sweep_tiled(s0, 3.9, 0.5, 12, 0, 25, order=order, order_seed=oseed)
        assert np.array_equal(got, ref)
        assert np.array_equal(c, cref)


@pytest.mark.parametrize("value", [0, 1])
def test_tiled_absorbing_states(oracle_lib, value):
    L = 16
    s0 = np.full((L, L), value, dtype=np.uint8)
    for r, K, seed in ((3.8, 0.5, 1), (2.0, 0.1, 2), (6.0, 3.0, 3)):
        s, c = oracle_lib.sweep_tiled(s0, r, K, seed, 7, 10)
        assert np.array_equal(s, s0)
        assert np.all(c == value * L * L)


def test_tiled_chunking_does_not_matter(oracle_lib):
    s0, _ = oracle_lib.init(24, 0.5, 19)
    whole, cw = oracle_lib.sweep_tiled(s0, 3.85, 0.5, 19, 0, 12)
    a, ca = oracle_lib.sweep_tiled(s0, 3.85, 0.5, 19, 0, 5)
    b, cb = oracle_lib.sweep_tiled(a, 3.85, 0.5, 19, 5, 7)
    assert np.array_equal(whole, b)
    assert np.array_equal(cw, np.concatenate([ca, cb]))
    assert cw[-1] == int(whole.sum())


def test_tiled_differs_from_the_colour_sweep(oracle_lib):
    # the two schedules are different dynamics from the same state and seed
    s0, _ = oracle_lib.init(16, 0.5, 4)
    a, _ = oracle_lib.sweep(s0, 3.9, 0.5, 4, 0, 3)
    c, _ = oracle_lib.sweep_tiled(s0, 3.9, 0.5, 4, 0, 3)
    assert not np.array_equal(a, c)


@pytest.mark.parametrize("L,r,seed,n", [(8, 3.8, 1, 4), (8, 4.4, 0x1234567890, 3), (16, 3.72, 5, 2),
                                        (16, 4.9, 6, 2)])
def test_tiled_matches_exact_brute_force(oracle_lib, rocrand_philox, L, r, seed, n):
    """Oracle C vs a literal, exact-arithmetic re-statement on tiny lattices."""
    K = 0.5
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref = [list(map(int, row)) for row in s0]
    for t in range(n):
        words = rocrand_philox(exact_ref.tiled_counters(L, t, seed))
        exact_ref.sweep_tiled(ref, L, r, K, words)
    got, _ = oracle_lib.sweep_tiled(s0, r, K, seed, 0, n)
    assert np.array_equal(got, np.array(ref, dtype=np.uint8))
    assert not np.array_equal(got, s0)


@pytest.mark.parametrize("L", [4, 12, 20, 100])
def test_tiled_rejects_L_not_a_multiple_of_8(oracle_lib, L):
    s = np.zeros((L, L), dtype=np.uint8)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.sweep_tiled(s, 3.8, 0.5, 1, 0, 1)

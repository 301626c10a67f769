"""Pins for oracle D, the pairwise prisoner's dilemma that Sec. VI names as
the next game for the same scheme (reading: the weak prisoner's dilemma,
R = 1, T = b, S = P = 0, four pairwise games per player, the Sec. III
imitation with the Fermi rule of Eq. (3), an 8-colour schedule)."""
import itertools
import os

import mpmath
import numpy as np
import pytest

import exact_ref

HERE = os.path.dirname(os.path.abspath(__file__))
TWO32 = 2**32
mpmath.mp.dps = 60

# temptations used below: the classic weak-dilemma range (1, 2], the
# boundary b = 1 (no temptation), and b = 0 (no payoff for defection)
B_VALUES = (0.0, 1.0, 1.01, 1.05, 1.1, 1.3, 1.5, 1.7, 1.9, 2.0, 2.5)
K_VALUES = (0.1, 0.5)


def _sites(spec, L):
    s = np.zeros((L, L), dtype=np.uint8)
    if spec == "-":
        return s
    if spec == "ALL":
        s[:] = 1
        return s
    if spec == "CHECKER":
        for i in range(L):
            for j in range(L):
                s[i, j] = (i + j) % 2 == 0
        return s
    if spec.startswith("ALL-"):
        s[:] = 1
        i, j = map(int, spec[4:].split(","))
        s[i, j] = 0
        return s
    for item in spec.split(";"):
        i, j = map(int, item.split(","))
        s[i, j] = 1
    return s


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "pd_payoffs_b1p5.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append((int(parts[0]), parts[1], int(parts[2]), int(parts[3]), float(parts[4]), int(parts[5]),
                         " ".join(parts[6:])))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[6][:40])
def test_hand_worked_payoffs(oracle_lib, row):
    L, spec, i, j, pay, ncoop, note = row
    s = _sites(spec, L)
    assert oracle_lib.pd_payoff(s, 1.5, i, j) == pay, note
    assert oracle_lib.pd_ncoop(s, i, j) == ncoop, note


def _diamond(r):
    return [(a, b) for a in range(-r, r + 1) for b in range(-r, r + 1) if abs(a) + abs(b) <= r]


def test_integer_form_by_brute_force(oracle_lib):
    # Every state of the 13 sites within distance 2 of x (all that Pi_x and
    # Pi_y read, for any of the 4 neighbours y) on a lattice large enough to
    # avoid wrap: the literal sum of the four games equals n for a
    # cooperator and b * n for a defector, n = cooperating neighbours.
    L, ci, cj = 8, 4, 4
    offs = _diamond(2)
    for b in (1.05, 1.5, 1.9):
        for bits in range(1 << len(offs)):
            s = np.zeros((L, L), dtype=np.uint8)
            for q, (a, c) in enumerate(offs):
                s[ci + a, cj + c] = (bits >> q) & 1
            for (a, c) in [(0, 0), (0, 1), (0, -1), (1, 0), (-1, 0)]:
                i, j = ci + a, cj + c
                n = oracle_lib.pd_ncoop(s, i, j)
                lit = oracle_lib.pd_payoff(s, b, i, j)
                assert lit == (n * 1.0 if s[i, j] else b * n), (b, bits, a, c)


def _exact_T(pix, piy, K):
    w = 1 / (1 + mpmath.exp((pix - piy) / mpmath.mpf(K)))
    return min(int(mpmath.floor(w * TWO32 + mpmath.mpf(1) / 2)), TWO32 - 1)


@pytest.mark.parametrize("b", B_VALUES)
@pytest.mark.parametrize("K", K_VALUES)
def test_table_is_exactly_rounded(oracle_lib, b, K):
    T = oracle_lib.pd_table(b, K)
    bb = mpmath.mpf(b)
    for nx in range(5):
        for ny in range(5):
            # dir 0: x cooperates (earns n_x), y defects (earns b n_y)
            assert int(T[0, nx, ny]) == _exact_T(mpmath.mpf(nx), bb * ny, K), (b, K, nx, ny)
            # dir 1: x defects (earns b n_x), y cooperates (earns n_y)
            assert int(T[1, nx, ny]) == _exact_T(bb * nx, mpmath.mpf(ny), K), (b, K, nx, ny)


def test_table_symmetry_and_limits(oracle_lib):
    # W(-z) = 1 - W(z): a C copying a D with (n_x, n_y) is the mirror of a D
    # copying a C with (n_y, n_x); equal payoffs give W = 1/2 exactly.
    for b in (1.05, 1.5):
        T = oracle_lib.pd_table(b, 0.5).astype(np.int64)
        for nx in range(5):
            for ny in range(5):
                assert T[0, nx, ny] + T[1, ny, nx] in (TWO32, TWO32 - 1)
        assert T[0, 0, 0] == 2**31 and T[1, 0, 0] == 2**31
    # b = 1: a C with n C neighbours and a D with n C neighbours earn the same
    T = oracle_lib.pd_table(1.0, 0.5)
    for n in range(5):
        assert T[0, n, n] == 2**31 and T[1, n, n] == 2**31
    # K -> 0 (tiny K): copy iff the neighbour earns more; ties stay at 1/2
    T = oracle_lib.pd_table(1.5, 1e-3)
    for nx in range(5):
        for ny in range(5):
            d0 = nx - 1.5 * ny
            assert T[0, nx, ny] == (2**31 if d0 == 0 else (TWO32 - 1 if d0 < 0 else 0))


def test_colouring_is_race_free_and_covers_once():
    # A pairwise update of x reads the radius-2 diamond (x, its neighbours,
    # their neighbours): one line less than the public goods game.  No other
    # site of x's class may lie in it (with periodic wrap), and the 8 classes
    # cover every site once, L^2 / 8 each.
    import oracle
    offs = [o for o in _diamond(2) if o != (0, 0)]
    for L in (4, 8, 12, 16, 20):
        cls = np.array([[oracle.pd_class(i, j) for j in range(L)] for i in range(L)])
        for k in range(8):
            assert (cls == k).sum() == L * L // 8
            assert sorted(zip(*np.nonzero(cls == k))) == sorted(exact_ref.pd_sites(L, k))
        for i in range(L):
            for j in range(L):
                for a, c in offs:
                    yi, yj = (i + a) % L, (j + c) % L
                    if (yi, yj) != (i, j):
                        assert cls[yi, yj] != cls[i, j], (L, i, j, a, c)
    # the class of a site repeats with period 4 in both directions and along (2, 2)
    for i, j in itertools.product(range(8), range(8)):
        k = oracle.pd_class(i, j)
        assert oracle.pd_class(i + 4, j) == k and oracle.pd_class(i, j + 4) == k
        assert oracle.pd_class(i + 2, j + 2) == k


def test_class_spacing():
    # Distinct sites of one class are at least 4 apart (L1, with periodic
    # wrap) and some are exactly 4 apart (e.g. (i, j) and (i + 2, j + 2)):
    # the cosets of the sublattice spanned by (2, 2) and (4, 0).  With L a
    # multiple of 4 no colouring with fewer classes keeps every pair 3 apart,
    # as the radius-2 read set requires (a sublattice containing 4 Z^2 has an
    # index dividing 16, and the index-4 ones all hold a vector of length 2).
    import oracle
    for L in (8, 12, 16):
        best = 99
        for i in range(L):
            for j in range(L):
                for a in range(-4, 5):
                    for c in range(-4, 5):
                        if (a, c) == (0, 0):
                            continue
                        yi, yj = (i + a) % L, (j + c) % L
                        if (yi, yj) != (i, j) and oracle.pd_class(yi, yj) == oracle.pd_class(i, j):
                            best = min(best, abs(a) + abs(c))
        assert best == 4, L
    # the index-4 subgroups of (Z/4)^2 each contain an element of wrapped length <= 2
    def wl(v):
        return sum(min(x % 4, 4 - x % 4) for x in v)
    elems = [(x, y) for x in range(4) for y in range(4)]
    for g1, g2 in itertools.combinations(elems, 2):
        sub = {((p * g1[0] + q * g2[0]) % 4, (p * g1[1] + q * g2[1]) % 4) for p in range(4) for q in range(4)}
        if len(sub) == 4:
            assert min(wl(v) for v in sub if v != (0, 0)) <= 2
    for g in elems:
        sub = {((p * g[0]) % 4, (p * g[1]) % 4) for p in range(4)}
        if len(sub) == 4:
            assert min(wl(v) for v in sub if v != (0, 0)) <= 2


def test_order_inside_a_class_does_not_matter(oracle_lib):
    s0, _ = oracle_lib.init(24, 0.5, 5)
    ref, cref = oracle_lib.pd_sweep(s0, 1.05, 0.1, 5, 0, 20, order=0)
    for order, oseed in ((1, 0), (2, 3), (2, 99)):
        got, c = oracle_lib.pd_sweep(s0, 1.05, 0.1, 5, 0, 20, order=order, order_seed=oseed)
        assert np.array_equal(got, ref) and np.array_equal(c, cref)


@pytest.mark.parametrize("value", [0, 1])
def test_absorbing_states(oracle_lib, value):
    s = np.full((16, 16), value, dtype=np.uint8)
    for b in (1.05, 1.5, 2.5):
        got, c = oracle_lib.pd_sweep(s, b, 0.1, 3, 0, 5)
        assert np.array_equal(got, s) and np.all(c == value * 256)


def test_chunking_and_counts(oracle_lib):
    s0, _ = oracle_lib.init(16, 0.5, 9)
    whole, cw = oracle_lib.pd_sweep(s0, 1.3, 0.5, 9, 0, 12)
    a, ca = oracle_lib.pd_sweep(s0, 1.3, 0.5, 9, 0, 5)
    b, cb = oracle_lib.pd_sweep(a, 1.3, 0.5, 9, 5, 7)
    assert np.array_equal(b, whole) and np.array_equal(np.concatenate([ca, cb]), cw)
    assert cw[-1] == whole.sum()


def test_differs_from_the_public_goods_sweep(oracle_lib):
    s0, _ = oracle_lib.init(16, 0.5, 2)
    pd, _ = oracle_lib.pd_sweep(s0, 1.5, 0.5, 2, 0, 3)
    pgg, _ = oracle_lib.sweep(s0, 3.8, 0.5, 2, 0, 3)
    assert not np.array_equal(pd, pgg)


@pytest.mark.parametrize("L,b,K,seed,n", [(8, 1.5, 0.5, 3, 3), (12, 1.05, 0.1, 7, 2), (4, 1.3, 0.5, 1, 3),
                                          (16, 1.9, 0.5, 2**40 + 5, 1)])
def test_sweep_matches_exact_brute_force(oracle_lib, rocrand_philox, L, b, K, seed, n):
    s0, _ = oracle_lib.init(L, 0.5, seed)
    ref = [list(map(int, row)) for row in s0]
    got, counts = oracle_lib.pd_sweep(s0, b, K, seed, 0, n)
    for t in range(n):
        words = rocrand_philox(exact_ref.pd_counters(L, t, seed))
        exact_ref.pd_sweep(ref, L, b, K, words)
        assert counts[t] == sum(map(sum, ref))
    assert np.array_equal(got, np.array(ref, dtype=np.uint8))


def test_rejects_bad_arguments(oracle_lib):
    s = np.zeros((6, 6), dtype=np.uint8)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.pd_sweep(s, 1.5, 0.5, 1, 0, 1)
    s = np.zeros((8, 8), dtype=np.uint8)
    for b, K in ((float("nan"), 0.5), (-1.0, 0.5), (1.5, 0.0)):
        with pytest.raises(oracle_lib.OracleError):
            oracle_lib.pd_sweep(s, b, K, 1, 0, 1)

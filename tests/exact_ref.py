"""Brute-force re-statement of the 16-colour sweep for tiny lattices.

Written from the paper's literal rules, in exact arithmetic, to pin the C
oracle: payoffs are summed group by group (Sec. III, Eq. (1)-(2)) with
Python ``Fraction``s, and the Fermi probability of Eq. (3) is evaluated with
mpmath at 60 significant digits and rounded to the 32-bit threshold exactly.
It never forms the integer sigma, never builds a table and takes its random
words from rocRAND's Philox (passed in), so an indexing, sign or table-layout
mistake in the oracle shows up as a different lattice.

Pure-Python loops: only for L <= 16 and a few sweeps.
"""
from fractions import Fraction

import mpmath

mpmath.mp.dps = 60

_NB = ((0, 0), (0, 1), (0, -1), (1, 0), (-1, 0))  # a site and its 4 neighbours
_DIR = ((0, 1), (0, -1), (1, 0), (-1, 0))          # d = 0 E, 1 W, 2 S, 3 N


def payoff(s, L, r, i, j):
    """Eq. (1)-(2) summed over the 5 groups containing (i, j); exact."""
    r = Fraction(r)
    coop = s[i % L][j % L]
    total = Fraction(0)
    for di, dj in _NB:
        ci, cj = i + di, j + dj
        nc = sum(s[(ci + a) % L][(cj + b) % L] for a, b in _NB)
        total += r * nc / 5 - (1 if coop else 0)
    return total


def threshold(dpi, K):
    """min(2^32 - 1, floor(W * 2^32 + 1/2)), W = 1/(1 + exp(dpi/K)), exact."""
    z = mpmath.mpf(dpi.numerator) / mpmath.mpf(dpi.denominator) / mpmath.mpf(Fraction(K).numerator) \
        * mpmath.mpf(Fraction(K).denominator)
    w = 1 / (1 + mpmath.exp(z))
    t = int(mpmath.floor(w * mpmath.mpf(2) ** 32 + mpmath.mpf(1) / 2))
    return min(t, 2**32 - 1)


def sweep_counters(L, t, seed):
    """Philox rows [c0, c1, c2, c3, k0, k1] for every site of sweep t."""
    rows = []
    for i in range(L):
        for j in range(L):
            k = 4 * (i % 4) + (j % 4)
            rows.append([i * L + j, t, k, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return rows


def sweep(s, L, r, K, words, t=None):
    """One 16-colour sweep in place.  words[x] = Philox output for site x."""
    for k in range(16):
        a, b = divmod(k, 4)
        for i in range(a, L, 4):
            for j in range(b, L, 4):
                w = words[i * L + j]
                d = int(w[0]) >> 30
                u = int(w[1])
                yi, yj = (i + _DIR[d][0]) % L, (j + _DIR[d][1]) % L
                if s[i][j] == s[yi][yj]:
                    continue
                dpi = payoff(s, L, r, i, j) - payoff(s, L, r, yi, yj)
                if u < threshold(dpi, K):
                    s[i][j] = s[yi][yj]
    return s


def _imitate(s, L, r, K, i, j, d, u):
    """Sec. III imitation of y by x = (i, j), exact payoffs and threshold."""
    yi, yj = (i + _DIR[d][0]) % L, (j + _DIR[d][1]) % L
    if s[i][j] == s[yi][yj]:
        return
    dpi = payoff(s, L, r, i, j) - payoff(s, L, r, yi, yj)
    if u < threshold(dpi, K):
        s[i][j] = s[yi][yj]


def tiled_counters(L, t, seed):
    """Philox rows [c0, c1, c2, c3, k0, k1] of one double-tiling step
    (Sec. IV) in execution order: part p = 0..3 (domain type 1 + p, i.e.
    domain row parity p // 2 and column parity p % 2), its domains in raster
    order, 16 elementary steps each; counter (domain index, t, 16 p + m, 2)."""
    n = L // 4
    rows = []
    for p in range(4):
        for I in range(p // 2, n, 2):
            for J in range(p % 2, n, 2):
                for m in range(16):
                    rows.append([I * n + J, t, 16 * p + m, 2, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return rows


def sweep_tiled(s, L, r, K, words):
    """One double-tiling Monte Carlo step in place; words in the order of
    tiled_counters.  The player is word0 >> 28 of the 4 x 4 domain (row-major),
    the direction (word0 >> 26) & 3, the acceptance word word1."""
    n = L // 4
    q = 0
    for p in range(4):
        for I in range(p // 2, n, 2):
            for J in range(p % 2, n, 2):
                for _ in range(16):
                    w = words[q]
                    q += 1
                    idx = int(w[0]) >> 28
                    _imitate(s, L, r, K, 4 * I + idx // 4, 4 * J + idx % 4, (int(w[0]) >> 26) & 3, int(w[1]))
    return s


# ---------------------------------------------------------------------------
# The pairwise prisoner's dilemma (the game Sec. VI names for the same
# scheme; reading: R = 1, T = b, S = P = 0, four games per player).
# ---------------------------------------------------------------------------
def pd_payoff(s, L, b, i, j):
    """Sum of the four pairwise games of (i, j); exact."""
    b = Fraction(b)
    sx = s[i % L][j % L]
    total = Fraction(0)
    for di, dj in _DIR:
        sy = s[(i + di) % L][(j + dj) % L]
        total += (1 if sy else 0) if sx else (b if sy else 0)
    return total


def pd_sites(L, k):
    """The sites of class k of the 8-colour schedule, written out from its
    definition: the coset of the sublattice spanned by (2, 2) and (4, 0)
    that holds (k // 4, k % 4) -- i.e. (i, j) with i = k // 4 (mod 2) and
    j - (k % 4) = 2 ((i - k // 4) / 2) (mod 4)."""
    a, q = divmod(k, 4)
    out = []
    for i in range(L):
        if (i - a) % 2:
            continue
        m = (i - a) // 2
        for j in range(L):
            if (j - q - 2 * m) % 4 == 0:
                out.append((i, j))
    return out


def pd_counters(L, t, seed):
    """Philox rows [c0, c1, c2, c3, k0, k1] of one 8-colour sweep in the
    order pd_sweep visits the sites."""
    rows = []
    for k in range(8):
        for i, j in pd_sites(L, k):
            rows.append([i * L + j, t, k, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return rows


def pd_sweep(s, L, b, K, words):
    """One 8-colour sweep of the pairwise game in place; words in the order
    of pd_counters."""
    q = 0
    for k in range(8):
        for i, j in pd_sites(L, k):
            w = words[q]
            q += 1
            d = int(w[0]) >> 30
            yi, yj = (i + _DIR[d][0]) % L, (j + _DIR[d][1]) % L
            if s[i][j] == s[yi][yj]:
                continue
            dpi = pd_payoff(s, L, b, i, j) - pd_payoff(s, L, b, yi, yj)
            if int(w[1]) < threshold(dpi, K):
                s[i][j] = s[yi][yj]
    return s

"""Pins for the oracle's payoffs (Sec. III, Eq. (1)-(2))."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _parse_sites(spec, L):
    s = np.zeros((L, L), dtype=np.uint8)
    if spec == "-":
        return s
    if spec == "ALL":
        s[:] = 1
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
    with open(os.path.join(HERE, "golden", "payoffs_r3p8.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            L, spec, i, j, pay, sig = parts[:6]
            rows.append((int(L), spec, int(i), int(j), float(pay), int(sig), " ".join(parts[6:])))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[6][:40])
def test_hand_worked_payoffs(oracle_lib, row):
    L, spec, i, j, pay, sig, _ = row
    s = _parse_sites(spec, L)
    assert oracle_lib.payoff(s, 3.8, i, j) == pytest.approx(pay, abs=1e-12)
    assert oracle_lib.sigma(s, i, j) == sig


def test_all_c_payoff_closed_form(oracle_lib):
    # Full cooperation: every group has N_C = 5, Pi_C = 5 (r - 1) (Eq. (1)).
    s = np.ones((12, 12), dtype=np.uint8)
    for r in (1.5, 3.8, 5.0, 7.25):
        assert oracle_lib.payoff(s, r, 5, 7) == pytest.approx(5 * (r - 1), abs=1e-12)


def test_defector_beats_cooperator_below_G(oracle_lib):
    # Sec. III: for r < G a defector always out-earns a cooperator in the same
    # group setting.  Swapping a single player's strategy raises its payoff
    # exactly by 5 - r (it stops paying c = 1 in 5 groups but removes its own
    # contribution r/5 from each), so defection wins iff r < 5.
    rng = np.random.default_rng(7)
    for _ in range(50):
        s = rng.integers(0, 2, size=(10, 10), dtype=np.uint8)
        i, j = rng.integers(0, 10, size=2)
        for r in (3.0, 4.9, 5.0, 6.0):
            sc = s.copy(); sc[i, j] = 1
            sd = s.copy(); sd[i, j] = 0
            gain = oracle_lib.payoff(sd, r, i, j) - oracle_lib.payoff(sc, r, i, j)
            assert gain == pytest.approx(5.0 - r, abs=1e-9)


def test_brute_force_integer_form(helper_bin):
    """All 2^18 states of the two radius-2 diamonds, 4 directions, 3 r."""
    out = subprocess.run([helper_bin("brute18.c")], capture_output=True, text=True,
                         check=True).stdout.split("\n")
    cases, failures = out[0].split()[1], out[0].split()[3]
    assert int(cases) == 4 * 3 * 2**18
    assert int(failures) == 0
    ranges = {int(l.split()[1]): (int(l.split()[3]), int(l.split()[4])) for l in out[1:4]}
    # dSigma realised per ds; the table's [-25, 25] must cover them.
    assert ranges == {-1: (-11, 5), 0: (-8, 8), 1: (-5, 11)}

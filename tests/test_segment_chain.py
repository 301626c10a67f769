"""The segmented-parity check of the long GPU runs, exercised on the host:
a chain of oracle segments accepts a true trajectory and reports a planted
one-site difference at a segment boundary (oracle only)."""
import numpy as np
import pytest

from test_gpu_late_windows import _check_chain


def test_chain_accepts_the_oracle_trajectory_and_catches_a_planted_difference(oracle_lib):
    L, r, K, seed = 32, 3.9, 0.5, 5
    s0, _ = oracle_lib.init(L, 0.5, seed)
    s1, c1 = oracle_lib.sweep(s0, r, K, seed, 0, 3)
    s2, c2 = oracle_lib.sweep(s1, r, K, seed, 3, 3)
    counts = np.concatenate([c1, c2])
    _check_chain([(0, s0), (3, s1)], counts, s2, r, K, seed)
    bad = s1.copy()
    bad[7, 9] ^= 1
    with pytest.raises(AssertionError):
        _check_chain([(0, s0), (3, bad)], counts, s2, r, K, seed)
    wrong = counts.copy()
    wrong[4] += 1
    with pytest.raises(AssertionError):
        _check_chain([(0, s0), (3, s1)], wrong, s2, r, K, seed)

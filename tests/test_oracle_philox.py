"""Pins for the oracle's Philox4x32-10 against rocRAND's independent code."""
import numpy as np


def test_philox_matches_rocrand(oracle_lib, rocrand_philox):
    rng = np.random.default_rng(2024)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    # counters of the shape the sweep uses: (x, t, k, 0) and init (x, 0, 0, 1)
    rows[2] = [12345, 7, 3, 0, 1, 0]
    rows[3] = [99, 0, 0, 1, 0xDEADBEEF, 0x12345678]
    expect = rocrand_philox(rows)
    for row, e in zip(rows, expect):
        got = oracle_lib.philox(row[:4], row[4:])
        assert np.array_equal(got, e), (row, got, e)


def test_init_uses_the_init_stream(oracle_lib, rocrand_philox):
    # Initial strategy of site x is [w0 < 2^31] with counter (x, 0, 0, 1) and
    # key (seed lo, seed hi); p0 = 1/2 (Sec. III, equal probability).
    L, seed = 12, 0x0000000500000003
    s, nc = oracle_lib.init(L, 0.5, seed)
    rows = [[x, 0, 0, 1, seed & 0xFFFFFFFF, seed >> 32] for x in range(L * L)]
    w = rocrand_philox(rows)
    expect = (w[:, 0].astype(np.uint64) < 2**31).astype(np.uint8).reshape(L, L)
    assert np.array_equal(s, expect)
    assert nc == int(expect.sum())

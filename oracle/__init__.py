"""CPU oracle for the spatial public goods game sweep (test infrastructure).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It wraps ``pgg_oracle.c`` (plain C, built
with gcc) through ctypes and shares no code with the HIP library.

What each function follows in the paper (M. Perc, 2017):

* ``payoff``   -- Sec. III, Eq. (1)-(2): group-by-group payoff in binary64.
* ``sigma``    -- Sec. III, Eq. (1)-(2) summed over the five groups (integer).
* ``table``    -- Sec. III, Eq. (3): Fermi probability as 32-bit thresholds.
* ``philox``   -- the counter RNG (Philox4x32-10, Salmon et al. 2011); the
                  paper does not name its generator.
* ``init``     -- Sec. III: i.i.d. initial strategies (fraction p0).
* ``sweep``    -- Sec. III elementary step, swept with the 16-colour schedule
                  (oracle A, the bit-exact contract).
* ``rs_run``   -- Sec. III random-sequential Monte Carlo (oracle B).
* ``sweep_tiled`` -- Sec. IV double tiling: 4 x 4 domains of four types,
                  random sequential steps inside each domain (oracle C).
* ``count``    -- Eq. (4): the cooperator count whose mean over L^2 is rho_C.
* ``pd_payoff``, ``pd_ncoop``, ``pd_table``, ``pd_class``, ``pd_sweep`` --
                  the pairwise prisoner's dilemma that Sec. VI names as the
                  next game for the same scheme (oracle D): four pairwise
                  games per player (R = 1, T = b, S = P = 0, our reading),
                  the Eq. (3) imitation, an 8-colour schedule.

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: hand-worked payoffs, an 18-site brute force, exact rounding with
mpmath, rocRAND's independent Philox, colouring race-freedom, absorbing
states and agreement of oracle A with oracle B and with the paper's printed
stationary density.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pgg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpgg_oracle.so")
_lib = None

N_TABLE = 153  # (dSigma in [-25, 25]) x (ds in {-1, 0, 1})


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libpgg_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.pgg_ref_philox.argtypes = [u32p, u32p, u32p]
    lib.pgg_ref_philox.restype = None
    lib.pgg_ref_group_nc.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_group_nc.restype = ctypes.c_int
    lib.pgg_ref_payoff.argtypes = [u8p, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_payoff.restype = ctypes.c_double
    lib.pgg_ref_sigma.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_sigma.restype = ctypes.c_int
    lib.pgg_ref_table.argtypes = [ctypes.c_double, ctypes.c_double, u32p]
    lib.pgg_ref_table.restype = ctypes.c_int
    lib.pgg_ref_init.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64, u8p, u64p]
    lib.pgg_ref_init.restype = ctypes.c_int
    lib.pgg_ref_count.argtypes = [u8p, ctypes.c_uint32]
    lib.pgg_ref_count.restype = ctypes.c_uint64
    lib.pgg_ref_sweep.argtypes = [u8p, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, u64p,
                                  ctypes.c_int, ctypes.c_uint64]
    lib.pgg_ref_sweep.restype = ctypes.c_int
    lib.pgg_ref_sweep_tiled.argtypes = lib.pgg_ref_sweep.argtypes
    lib.pgg_ref_sweep_tiled.restype = ctypes.c_int
    lib.pgg_ref_rs_run.argtypes = [u8p, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_uint32, u64p]
    lib.pgg_ref_rs_run.restype = ctypes.c_int
    lib.pgg_ref_pd_payoff.argtypes = [u8p, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_pd_payoff.restype = ctypes.c_double
    lib.pgg_ref_pd_ncoop.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_pd_ncoop.restype = ctypes.c_int
    lib.pgg_ref_pd_table.argtypes = [ctypes.c_double, ctypes.c_double, u32p]
    lib.pgg_ref_pd_table.restype = ctypes.c_int
    lib.pgg_ref_pd_class.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.pgg_ref_pd_class.restype = ctypes.c_int
    lib.pgg_ref_pd_sweep.argtypes = lib.pgg_ref_sweep.argtypes
    lib.pgg_ref_pd_sweep.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleError(ValueError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError("%s failed with status %d" % (what, rc))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for counter (4 x u32) and key (2 x u32)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib.pgg_ref_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def _lattice(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.uint8)
    if s.ndim != 2 or s.shape[0] != s.shape[1]:
        raise OracleError("lattice must be a square 2-D array")
    return s


def payoff(s: np.ndarray, r: float, i: int, j: int) -> float:
    """Total payoff of player (i, j), Eq. (1)-(2), binary64."""
    s = _lattice(s)
    return _load().pgg_ref_payoff(_p(s, ctypes.c_uint8), s.shape[0], float(r), int(i), int(j))


def group_nc(s: np.ndarray, i: int, j: int) -> int:
    s = _lattice(s)
    return _load().pgg_ref_group_nc(_p(s, ctypes.c_uint8), s.shape[0], int(i), int(j))


def sigma(s: np.ndarray, i: int, j: int) -> int:
    """Sum of the cooperator counts of the five groups containing (i, j)."""
    s = _lattice(s)
    return _load().pgg_ref_sigma(_p(s, ctypes.c_uint8), s.shape[0], int(i), int(j))


def table(r: float, K: float) -> np.ndarray:
    """Fermi thresholds T[dSigma + 25, ds + 1] (shape 51 x 3, uint32)."""
    t = np.zeros(N_TABLE, dtype=np.uint32)
    _check(_load().pgg_ref_table(float(r), float(K), _p(t, ctypes.c_uint32)), "table")
    return t.reshape(51, 3)


def init(L: int, p0: float, seed: int):
    """Initial lattice (L x L uint8) and its cooperator count."""
    s = np.zeros((L, L), dtype=np.uint8)
    nc = np.zeros(1, dtype=np.uint64)
    _check(_load().pgg_ref_init(int(L), float(p0), int(seed) & (2**64 - 1),
                                _p(s, ctypes.c_uint8), _p(nc, ctypes.c_uint64)), "init")
    return s, int(nc[0])


def count(s: np.ndarray) -> int:
    s = _lattice(s)
    return int(_load().pgg_ref_count(_p(s, ctypes.c_uint8), s.shape[0]))


def sweep(s: np.ndarray, r: float, K: float, seed: int, t0: int, n: int,
          order: int = 0, order_seed: int = 0):
    """Oracle A: n 16-colour sweeps from absolute sweep index t0.

    Returns (new lattice, counts after each sweep).  The input is not
    modified.  ``order`` permutes the visiting order inside each colour class
    (0 raster, 1 reversed, 2 random), which must not change the result.
    """
    s = _lattice(s).copy()
    counts = np.zeros(max(int(n), 1), dtype=np.uint64)
    _check(_load().pgg_ref_sweep(_p(s, ctypes.c_uint8), s.shape[0], float(r), float(K),
                                 int(seed) & (2**64 - 1), int(t0), int(n),
                                 _p(counts, ctypes.c_uint64), int(order),
                                 int(order_seed) & (2**64 - 1)), "sweep")
    return s, counts[:n]


def sweep_tiled(s: np.ndarray, r: float, K: float, seed: int, t0: int, n: int,
                order: int = 0, order_seed: int = 0):
    """Oracle C: n Monte Carlo steps of the double tiling (Sec. IV) from
    absolute sweep index t0; L a multiple of 8.  Returns (new lattice, counts
    after each step).  ``order`` permutes the domains inside each part (0
    raster, 1 reversed, 2 random), which must not change the result."""
    s = _lattice(s).copy()
    counts = np.zeros(max(int(n), 1), dtype=np.uint64)
    _check(_load().pgg_ref_sweep_tiled(_p(s, ctypes.c_uint8), s.shape[0], float(r), float(K),
                                       int(seed) & (2**64 - 1), int(t0), int(n),
                                       _p(counts, ctypes.c_uint64), int(order),
                                       int(order_seed) & (2**64 - 1)), "sweep_tiled")
    return s, counts[:n]


def run_tiled(L: int, r: float, K: float, p0: float, seed: int, n: int):
    """Init + n tiled steps (oracle C): (lattice, N_C(0), counts)."""
    s, nc0 = init(L, p0, seed)
    s, counts = sweep_tiled(s, r, K, seed, 0, n)
    return s, nc0, counts


def rs_run(s: np.ndarray, r: float, K: float, seed: int, n_mcs: int):
    """Oracle B: n_mcs random-sequential Monte Carlo steps (statistical only)."""
    s = _lattice(s).copy()
    counts = np.zeros(max(int(n_mcs), 1), dtype=np.uint64)
    _check(_load().pgg_ref_rs_run(_p(s, ctypes.c_uint8), s.shape[0], float(r), float(K),
                                  int(seed) & (2**64 - 1), int(n_mcs),
                                  _p(counts, ctypes.c_uint64)), "rs_run")
    return s, counts[:n_mcs]


def run(L: int, r: float, K: float, p0: float, seed: int, n: int):
    """Init + n sweeps of oracle A: (lattice after n sweeps, N_C(0), counts)."""
    s, nc0 = init(L, p0, seed)
    s, counts = sweep(s, r, K, seed, 0, n)
    return s, nc0, counts


def pd_payoff(s: np.ndarray, b: float, i: int, j: int) -> float:
    """Oracle D: payoff of (i, j) from its four pairwise games, binary64."""
    s = _lattice(s)
    return _load().pgg_ref_pd_payoff(_p(s, ctypes.c_uint8), s.shape[0], float(b), int(i), int(j))


def pd_ncoop(s: np.ndarray, i: int, j: int) -> int:
    """Oracle D: cooperators among the four nearest neighbours of (i, j)."""
    s = _lattice(s)
    return _load().pgg_ref_pd_ncoop(_p(s, ctypes.c_uint8), s.shape[0], int(i), int(j))


def pd_table(b: float, K: float) -> np.ndarray:
    """Oracle D: Fermi thresholds T[dir, n_x, n_y] (shape 2 x 5 x 5, uint32);
    dir 0: x cooperates and y defects, dir 1: x defects and y cooperates."""
    t = np.zeros(50, dtype=np.uint32)
    _check(_load().pgg_ref_pd_table(float(b), float(K), _p(t, ctypes.c_uint32)), "pd_table")
    return t.reshape(2, 5, 5)


def pd_class(i: int, j: int) -> int:
    """Oracle D: class of (i, j) in the 8-colour schedule."""
    return int(_load().pgg_ref_pd_class(int(i), int(j)))


def pd_sweep(s: np.ndarray, b: float, K: float, seed: int, t0: int, n: int,
             order: int = 0, order_seed: int = 0):
    """Oracle D: n 8-colour sweeps of the pairwise prisoner's dilemma from
    absolute sweep index t0.  Returns (new lattice, counts after each sweep);
    ``order`` permutes the sites inside each class and must not change the
    result."""
    s = _lattice(s).copy()
    counts = np.zeros(max(int(n), 1), dtype=np.uint64)
    _check(_load().pgg_ref_pd_sweep(_p(s, ctypes.c_uint8), s.shape[0], float(b), float(K),
                                    int(seed) & (2**64 - 1), int(t0), int(n),
                                    _p(counts, ctypes.c_uint64), int(order),
                                    int(order_seed) & (2**64 - 1)), "pd_sweep")
    return s, counts[:n]


def pd_run(L: int, b: float, K: float, p0: float, seed: int, n: int):
    """Init (as for oracle A) + n sweeps of oracle D: (lattice, N_C(0), counts)."""
    s, nc0 = init(L, p0, seed)
    s, counts = pd_sweep(s, b, K, seed, 0, n)
    return s, nc0, counts

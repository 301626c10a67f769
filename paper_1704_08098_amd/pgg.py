"""ctypes binding of libpgg.so (declared in include/pgg.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
the library.  There is no fallback: if libpgg.so is missing or no GPU is
visible, the calls raise.

Function names follow the C ABI (``pgg_init``, ``pgg_sweep``,
``pgg_density``, ...); ``Sim`` wraps a handle.  PyTorch is used only to
provide device memory (an optional caller-owned lattice buffer) and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpgg.so")

PGG_OK, PGG_E_INVAL, PGG_E_NOMEM, PGG_E_DEVICE, PGG_E_STATE = 0, -1, -2, -3, -4
LAYOUT_INT8, LAYOUT_BITS = 0, 1
KERNEL_AUTO, KERNEL_COLOUR, KERNEL_ROWBAND, KERNEL_ROWBAND_COMPACT, KERNEL_ROWBAND_STAGED = 0, 1, 2, 3, 4
KERNEL_STRIP, KERNEL_SEGMENT, KERNEL_SEGMENT_PAIR, KERNEL_RESIDENT = 5, 6, 7, 8
SCHEDULE_COLOUR16, SCHEDULE_TILED = 0, 1
LAYOUTS = {"int8": LAYOUT_INT8, "bits": LAYOUT_BITS}
SCHEDULES = {"colour16": SCHEDULE_COLOUR16, "tiled": SCHEDULE_TILED}
GAME_PUBLIC_GOODS, GAME_PAIRWISE_PD = 0, 1
GAMES = {"pgg": GAME_PUBLIC_GOODS, "pd": GAME_PAIRWISE_PD}
KERNELS = {"auto": KERNEL_AUTO, "colour": KERNEL_COLOUR, "rowband": KERNEL_ROWBAND,
           "rowband_compact": KERNEL_ROWBAND_COMPACT, "rowband_staged": KERNEL_ROWBAND_STAGED,
           "strip": KERNEL_STRIP, "segment": KERNEL_SEGMENT, "segment_pair": KERNEL_SEGMENT_PAIR,
           "resident": KERNEL_RESIDENT}

# Every symbol include/pgg.h declares (checked by the CPU test suite).
EXPORTS = ("pgg_device_bytes", "pgg_plan", "pgg_init", "pgg_sweep", "pgg_density", "pgg_coop_count",
           "pgg_sweep_index", "pgg_read_lattice", "pgg_write_lattice", "pgg_threshold_table", "pgg_fermi_table",
           "pgg_pd_table",
           "pgg_set_kernel_timing", "pgg_kernel_timing", "pgg_kernel_span", "pgg_set_strip_wait", "pgg_destroy",
           "pgg_last_error", "pgg_ensemble_create", "pgg_ensemble_sweep", "pgg_ensemble_coop_counts",
           "pgg_ensemble_sweep_index", "pgg_ensemble_read_lattice", "pgg_ensemble_destroy",
           "pgg_ensemble_autotune", "pgg_ensemble_threshold_table", "pgg_ensemble_run",
           "pgg_server_job_bytes", "pgg_server_create", "pgg_server_submit", "pgg_server_step",
           "pgg_server_completed", "pgg_server_job_state", "pgg_server_job_result", "pgg_server_stats",
           "pgg_server_destroy", "pgg_sweep_static_scratch_bytes", "pgg_sweep_static")


class PggParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("r", ctypes.c_double), ("K", ctypes.c_double),
                ("p0", ctypes.c_double), ("seed", ctypes.c_uint64), ("layout", ctypes.c_uint32),
                ("kernel", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32), ("game", ctypes.c_uint32)]


class PggEnsembleTune(ctypes.Structure):
    _fields_ = [("tiles", ctypes.POINTER(ctypes.c_uint32)), ("chunk", ctypes.c_uint32),
                ("waves_per_group", ctypes.c_uint32), ("branches", ctypes.c_uint32),
                ("resident_max_L", ctypes.c_uint32), ("resident_waves", ctypes.c_uint32)]


TUNE_KEYS = ("chunk", "waves_per_group", "branches", "resident_max_L", "resident_waves")


def _tune_struct(tiles=None, chunk=32, waves_per_group=0, branches=0, resident_max_L=0, resident_waves=0):
    """(PggEnsembleTune, the tiles array it points at -- keep it alive)."""
    tl = None
    if tiles is not None:
        tl = np.ascontiguousarray(np.asarray(tiles, dtype=np.uint32))
    t = PggEnsembleTune(tl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if tl is not None else None,
                        int(chunk), int(waves_per_group), int(branches), int(resident_max_L), int(resident_waves))
    return t, tl


class PggServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint32), ("resident", ctypes.c_uint32), ("completed", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64), ("budget", ctypes.c_uint64),
                ("site_updates", ctypes.c_uint64)]


class PggError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("pgg status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load():
    """Load libpgg.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpgg.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, u8p, u32p, u64p = ctypes.c_void_p, P(ctypes.c_uint8), P(ctypes.c_uint32), P(ctypes.c_uint64)
    sig = {
        "pgg_device_bytes": (ctypes.c_size_t, [P(PggParams)]),
        "pgg_plan": (ctypes.c_int, [P(PggParams), P(ctypes.c_uint32), P(ctypes.c_uint32)]),
        "pgg_init": (ctypes.c_int, [P(PggParams), vp, ctypes.c_size_t, vp, P(vp)]),
        "pgg_sweep": (ctypes.c_int, [vp, ctypes.c_uint32, u64p]),
        "pgg_density": (ctypes.c_int, [vp, P(ctypes.c_double)]),
        "pgg_coop_count": (ctypes.c_int, [vp, u64p]),
        "pgg_sweep_index": (ctypes.c_int, [vp, u64p]),
        "pgg_read_lattice": (ctypes.c_int, [vp, u8p]),
        "pgg_write_lattice": (ctypes.c_int, [vp, u8p, ctypes.c_uint64]),
        "pgg_threshold_table": (ctypes.c_int, [vp, u32p]),
        "pgg_fermi_table": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, u32p]),
        "pgg_pd_table": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, u32p]),
        "pgg_set_kernel_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "pgg_kernel_timing": (ctypes.c_int, [vp, u64p, P(ctypes.c_double), u64p]),
        "pgg_kernel_span": (ctypes.c_int, [vp, u64p, P(ctypes.c_double)]),
        "pgg_set_strip_wait": (ctypes.c_int, [vp, ctypes.c_double]),
        "pgg_destroy": (None, [vp]),
        "pgg_last_error": (ctypes.c_char_p, []),
        "pgg_ensemble_create": (ctypes.c_int, [P(PggParams), ctypes.c_uint32, P(PggEnsembleTune), vp, P(vp)]),
        "pgg_ensemble_sweep": (ctypes.c_int, [vp, ctypes.c_uint32, u64p]),
        "pgg_ensemble_coop_counts": (ctypes.c_int, [vp, u64p]),
        "pgg_ensemble_sweep_index": (ctypes.c_int, [vp, u64p]),
        "pgg_ensemble_read_lattice": (ctypes.c_int, [vp, ctypes.c_uint32, u8p]),
        "pgg_ensemble_destroy": (None, [vp]),
        "pgg_ensemble_threshold_table": (ctypes.c_int, [vp, ctypes.c_uint32, u32p]),
        "pgg_ensemble_run": (ctypes.c_int, [P(PggParams), ctypes.c_uint32, ctypes.c_uint32, u64p,
                                            P(PggEnsembleTune), vp]),
        "pgg_ensemble_autotune": (ctypes.c_int, [P(PggParams), ctypes.c_uint32, ctypes.c_uint32, vp, u32p,
                                                 P(PggEnsembleTune), P(ctypes.c_double)]),
        "pgg_server_job_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32]),
        "pgg_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                             vp, P(vp)]),
        "pgg_server_submit": (ctypes.c_int, [vp, P(PggParams), ctypes.c_uint32, u64p]),
        "pgg_server_step": (ctypes.c_int, [vp, u32p]),
        "pgg_server_completed": (ctypes.c_int, [vp, u64p, ctypes.c_uint32, u32p]),
        "pgg_server_job_state": (ctypes.c_int, [vp, ctypes.c_uint64, P(ctypes.c_int), u32p]),
        "pgg_server_job_result": (ctypes.c_int, [vp, ctypes.c_uint64, u64p, u8p]),
        "pgg_server_stats": (ctypes.c_int, [vp, P(PggServerInfo)]),
        "pgg_server_destroy": (None, [vp]),
        "pgg_sweep_static_scratch_bytes": (ctypes.c_size_t, []),
        "pgg_sweep_static": (ctypes.c_int, [P(PggParams), vp, ctypes.c_uint64, ctypes.c_uint32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != PGG_OK:
        raise PggError(status, load().pgg_last_error().decode())


def make_params(L, r, K=0.5, p0=0.5, seed=1, layout="bits", kernel="auto", tile=0, group=0,
                schedule="colour16", game="pgg") -> PggParams:
    """game "pd": the pairwise prisoner's dilemma with temptation b = r."""
    return PggParams(int(L), float(r), float(K), float(p0), int(seed) & (2**64 - 1),
                     LAYOUTS[layout] if isinstance(layout, str) else int(layout),
                     KERNELS[kernel] if isinstance(kernel, str) else int(kernel), int(tile), int(group),
                     SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule),
                     GAMES[game] if isinstance(game, str) else int(game))


def pgg_device_bytes(params: PggParams) -> int:
    return int(load().pgg_device_bytes(ctypes.byref(params)))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def pgg_plan(params: PggParams):
    """The (kernel name, tile) pgg_init would take for these parameters on
    the current device: AUTO resolved, and the work split it runs (segment
    width, rows per band, waves; 0 where there is none).  The tiled schedule
    and the pairwise game report "auto"."""
    k, t = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().pgg_plan(ctypes.byref(params), ctypes.byref(k), ctypes.byref(t)))
    names = {v: n for n, v in KERNELS.items()}
    return names.get(k.value, str(k.value)), int(t.value)


def pgg_init(params: PggParams, dev_buf=None, stream=None):
    """Returns an opaque handle (c_void_p).  dev_buf: torch tensor or None."""
    lib = load()
    h = ctypes.c_void_p()
    ptr, nbytes = None, 0
    if dev_buf is not None:
        ptr, nbytes = dev_buf.data_ptr(), dev_buf.numel() * dev_buf.element_size()
    _check(lib.pgg_init(ctypes.byref(params), ptr, nbytes, _stream_handle(stream), ctypes.byref(h)))
    return h


def pgg_sweep(handle, n: int, want_counts: bool = True):
    """Advance n sweeps; returns N_C after each sweep (uint64) or None."""
    if want_counts:
        out = np.zeros(max(n, 1), dtype=np.uint64)
        _check(load().pgg_sweep(handle, int(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out[:n]
    _check(load().pgg_sweep(handle, int(n), None))
    return None


def pgg_density(handle) -> float:
    v = ctypes.c_double()
    _check(load().pgg_density(handle, ctypes.byref(v)))
    return v.value


def pgg_coop_count(handle) -> int:
    v = ctypes.c_uint64()
    _check(load().pgg_coop_count(handle, ctypes.byref(v)))
    return v.value


def pgg_sweep_index(handle) -> int:
    v = ctypes.c_uint64()
    _check(load().pgg_sweep_index(handle, ctypes.byref(v)))
    return v.value


def pgg_read_lattice(handle, L: int) -> np.ndarray:
    out = np.zeros((L, L), dtype=np.uint8)
    _check(load().pgg_read_lattice(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out


def pgg_write_lattice(handle, lattice: np.ndarray, t: int) -> None:
    a = np.ascontiguousarray(lattice, dtype=np.uint8)
    _check(load().pgg_write_lattice(handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(t)))


def pgg_threshold_table(handle) -> np.ndarray:
    out = np.zeros(153, dtype=np.uint32)
    _check(load().pgg_threshold_table(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return out.reshape(51, 3)


def pgg_fermi_table(r: float, K: float) -> np.ndarray:
    """The Fermi thresholds the library uses for (r, K), built on the host:
    T[dSigma + 25, ds + 1], shape (51, 3) (host only, no device)."""
    out = np.zeros(153, dtype=np.uint32)
    _check(load().pgg_fermi_table(float(r), float(K), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return out.reshape(51, 3)


def pgg_pd_table(b: float, K: float) -> np.ndarray:
    """The thresholds of the pairwise prisoner's dilemma the library uses for
    (b, K), built on the host: T[dir, n_x, n_y], shape (2, 5, 5) (host only)."""
    out = np.zeros(50, dtype=np.uint32)
    _check(load().pgg_pd_table(float(b), float(K), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return out.reshape(2, 5, 5)


def pgg_set_kernel_timing(handle, enable: bool) -> None:
    _check(load().pgg_set_kernel_timing(handle, 1 if enable else 0))


def pgg_kernel_timing(handle):
    """(launches, total_ms, drawn) since timing was last enabled."""
    n, ms, drawn = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint64()
    _check(load().pgg_kernel_timing(handle, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(drawn)))
    return n.value, ms.value, drawn.value


def pgg_set_strip_wait(handle, seconds: float) -> None:
    _check(load().pgg_set_strip_wait(handle, float(seconds)))


def pgg_sweep_static_scratch_bytes() -> int:
    return int(load().pgg_sweep_static_scratch_bytes())


def pgg_sweep_static(params: PggParams, dev_lattice, t0: int, n: int, dev_counts=None, stream=None) -> None:
    """The sweep that allocates nothing: advance the bit-packed lattice in
    the device tensor dev_lattice (pgg_device_bytes(params) bytes) n sweeps
    from sweep index t0; dev_counts: None or a device uint64-sized tensor of
    n entries receiving N_C after each sweep.  Only enqueues work."""
    if dev_lattice.numel() * dev_lattice.element_size() < pgg_device_bytes(params):
        raise ValueError("dev_lattice is smaller than pgg_device_bytes(params)")
    cptr = None
    if dev_counts is not None:
        if dev_counts.numel() * dev_counts.element_size() < 8 * int(n):
            raise ValueError("dev_counts holds fewer than n 64-bit entries")
        cptr = dev_counts.data_ptr()
    _check(load().pgg_sweep_static(ctypes.byref(params), dev_lattice.data_ptr(), int(t0), int(n), cptr,
                                   _stream_handle(stream)))


def pgg_destroy(handle) -> None:
    if handle:
        load().pgg_destroy(handle)


class Sim:
    """One lattice on the GPU.  Mirrors the C calls one to one."""

    def __init__(self, L, r, K=0.5, p0=0.5, seed=1, layout="bits", kernel="auto",
                 dev_buf=None, stream=None, tile=0, group=0, schedule="colour16", game="pgg"):
        self.params = make_params(L, r, K, p0, seed, layout, kernel, tile, group, schedule, game)
        self.L = int(L)
        self._buf = dev_buf  # keep a caller tensor alive as long as the handle
        self.handle = pgg_init(self.params, dev_buf, stream)

    def sweep(self, n, want_counts=True):
        return pgg_sweep(self.handle, n, want_counts)

    def density(self):
        return pgg_density(self.handle)

    def coop_count(self):
        return pgg_coop_count(self.handle)

    @property
    def t(self):
        return pgg_sweep_index(self.handle)

    def read_lattice(self):
        return pgg_read_lattice(self.handle, self.L)

    def write_lattice(self, lattice, t):
        pgg_write_lattice(self.handle, lattice, t)

    def threshold_table(self):
        return pgg_threshold_table(self.handle)

    def set_kernel_timing(self, enable=True):
        pgg_set_kernel_timing(self.handle, enable)

    def kernel_timing(self):
        return pgg_kernel_timing(self.handle)

    def kernel_span(self):
        """(launches, total span in microseconds) of the segment kernel's timed launches."""
        n = ctypes.c_uint64()
        us = ctypes.c_double()
        _check(load().pgg_kernel_span(self.handle, ctypes.byref(n), ctypes.byref(us)))
        return int(n.value), float(us.value)

    def set_strip_wait(self, seconds):
        pgg_set_strip_wait(self.handle, seconds)

    def close(self):
        if self.handle:
            pgg_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _replica_params(replicas):
    arr = (PggParams * len(replicas))()
    for k, rp in enumerate(replicas):
        arr[k] = make_params(rp["L"], rp["r"], rp.get("K", 0.5), rp.get("p0", 0.5),
                             rp.get("seed", 1), "bits", "auto", schedule=rp.get("schedule", "colour16"),
                             game=rp.get("game", "pgg"))
    return arr


def ensemble_autotune(replicas, probe_sweeps=8, stream=None):
    """pgg_ensemble_autotune: (tune, ms) -- tune a dict with the chosen tiles
    (one per replica), chunk, waves_per_group, branches, resident_max_L and
    resident_waves (the keyword arguments of Ensemble), ms the best time per
    sweep."""
    n = len(replicas)
    arr = _replica_params(replicas)
    tiles = np.zeros(n, dtype=np.uint32)
    tune = PggEnsembleTune()
    ms = ctypes.c_double()
    _check(load().pgg_ensemble_autotune(arr, n, int(probe_sweeps), _stream_handle(stream),
                                        tiles.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(tune),
                                        ctypes.byref(ms)))
    out = {k: int(getattr(tune, k)) for k in TUNE_KEYS}
    out["tiles"] = tiles
    return out, float(ms.value)


def ensemble_run(replicas, n_sweeps, tune=None, stream=None):
    """pgg_ensemble_run: counts (n_reps, n_sweeps) of one batched run from the
    initial states.  tune: None (autotune) or a dict with the keyword
    arguments of Ensemble (tiles, chunk, waves_per_group, branches,
    resident_max_L, resident_waves)."""
    n = len(replicas)
    arr = _replica_params(replicas)
    out = np.zeros((n, max(int(n_sweeps), 1)), dtype=np.uint64)
    t, keep = None, None
    if tune is not None:
        t, keep = _tune_struct(**{k: v for k, v in tune.items() if k in TUNE_KEYS + ("tiles",)})
    _check(load().pgg_ensemble_run(arr, n, int(n_sweeps), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   ctypes.byref(t) if t is not None else None, _stream_handle(stream)))
    del keep
    return out[:, :n_sweeps]


class Ensemble:
    """Many replicas advanced together (pgg_ensemble_* calls).

    replicas: sequence of dicts with L, r and optionally K, p0, seed.
    tiles: optional per-replica segment widths (0 = automatic).
    waves_per_group: segment waves per workgroup, 2, 4 or 8 (0 = 4).
    branches: concurrent replica groups (parallel graph branches), 0..16 (0 = two
              for the 16-colour schedule, one for the tiled one).
    resident_max_L: 0, or the largest side swept by the resident kernel.
    resident_waves: waves per resident workgroup, 4, 8 or 16 (0 = 8).
    """

    def __init__(self, replicas, tiles=None, chunk=32, stream=None, waves_per_group=0, branches=0,
                 resident_max_L=0, resident_waves=0):
        lib = load()
        n = len(replicas)
        arr = _replica_params(replicas)
        self.L = [int(rp["L"]) for rp in replicas]
        self.n = n
        tune, self._tiles = _tune_struct(tiles, chunk, waves_per_group, branches, resident_max_L, resident_waves)
        if self._tiles is not None:
            assert self._tiles.shape == (n,)
        h = ctypes.c_void_p()
        _check(lib.pgg_ensemble_create(arr, n, ctypes.byref(tune), _stream_handle(stream), ctypes.byref(h)))
        self.handle = h

    def sweep(self, n_sweeps, want_counts=True):
        """Advance every replica; returns counts (n_reps, n_sweeps) or None."""
        if want_counts:
            out = np.zeros((self.n, max(n_sweeps, 1)), dtype=np.uint64)
            _check(load().pgg_ensemble_sweep(self.handle, int(n_sweeps),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
            return out[:, :n_sweeps]
        _check(load().pgg_ensemble_sweep(self.handle, int(n_sweeps), None))
        return None

    def coop_counts(self):
        out = np.zeros(self.n, dtype=np.uint64)
        _check(load().pgg_ensemble_coop_counts(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out

    @property
    def t(self):
        v = ctypes.c_uint64()
        _check(load().pgg_ensemble_sweep_index(self.handle, ctypes.byref(v)))
        return v.value

    def read_lattice(self, k):
        L = self.L[k]
        out = np.zeros((L, L), dtype=np.uint8)
        _check(load().pgg_ensemble_read_lattice(self.handle, int(k),
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out

    def threshold_table(self, k):
        """The Fermi thresholds replica k uses on the device, shape (51, 3)."""
        out = np.zeros(153, dtype=np.uint32)
        _check(load().pgg_ensemble_threshold_table(self.handle, int(k),
                                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return out.reshape(51, 3)

    def close(self):
        if self.handle:
            load().pgg_ensemble_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerEngine:
    """The C job server (pgg_server_* calls): submit, step, completed, result."""

    def __init__(self, hbm_budget, max_L=2048, max_resident=4096, chunk=16, stream=None):
        h = ctypes.c_void_p()
        _check(load().pgg_server_create(int(hbm_budget), int(max_L), int(max_resident), int(chunk),
                                        _stream_handle(stream), ctypes.byref(h)))
        self.handle = h
        self.chunk = int(chunk)
        self._n = {}

    @staticmethod
    def job_bytes(L, chunk):
        return int(load().pgg_server_job_bytes(int(L), int(chunk)))

    def submit(self, L, r, n_sweeps, K=0.5, p0=0.5, seed=1, tile=0):
        jid = ctypes.c_uint64()
        p = make_params(L, r, K, p0, seed, "bits", "auto", tile)
        _check(load().pgg_server_submit(self.handle, ctypes.byref(p), int(n_sweeps), ctypes.byref(jid)))
        self._n[jid.value] = (int(L), int(n_sweeps))
        return jid.value

    def step(self):
        n = ctypes.c_uint32()
        _check(load().pgg_server_step(self.handle, ctypes.byref(n)))
        return n.value

    def completed(self, cap=4096):
        ids = np.zeros(cap, dtype=np.uint64)
        n = ctypes.c_uint32()
        _check(load().pgg_server_completed(self.handle, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                           cap, ctypes.byref(n)))
        return [int(v) for v in ids[:n.value]]

    def state(self, jid):
        st, done = ctypes.c_int(), ctypes.c_uint32()
        _check(load().pgg_server_job_state(self.handle, int(jid), ctypes.byref(st), ctypes.byref(done)))
        return st.value, done.value

    def result(self, jid, want_lattice=True):
        L, n = self._n.pop(jid)
        counts = np.zeros(n, dtype=np.uint64)
        lat = np.zeros((L, L), dtype=np.uint8) if want_lattice else None
        _check(load().pgg_server_job_result(self.handle, int(jid),
                                            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                            lat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
                                            if lat is not None else None))
        return counts, lat

    def stats(self):
        info = PggServerInfo()
        _check(load().pgg_server_stats(self.handle, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in PggServerInfo._fields_}

    def close(self):
        if self.handle:
            load().pgg_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

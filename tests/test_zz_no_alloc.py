"""GPU: pgg_sweep_static, the sweep that allocates nothing, against the
handle path (pgg_init + pgg_sweep) on the same lattice: counts after every
sweep and the final lattice bit for bit, on two calls in a row -- the second
with a smaller lattice -- so that the shared fixed device array is reused
with a different size.  Also checks the arguments it rejects."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.set_device(0)
    from paper_1704_08098_amd import pgg
    pgg.load()
    return pgg, torch


def _handle_run(pgg, torch, L, r, seed, t_start, n):
    """Handle path: init, t_start sweeps, then the n sweeps compared.
    Returns (lattice tensor copy at t_start, counts of the n sweeps, final
    lattice bytes)."""
    params = pgg.make_params(L, r, 0.5, 0.5, seed, layout="bits")
    nbytes = pgg.pgg_device_bytes(params)
    buf = torch.zeros(nbytes // 4, dtype=torch.int32, device="cuda")
    with pgg.Sim(L, r, 0.5, 0.5, seed, "bits", dev_buf=buf) as sim:
        sim.sweep(t_start, want_counts=False)
        start = buf.clone()
        torch.cuda.synchronize()
        counts = sim.sweep(n)
        final = buf.clone()
        torch.cuda.synchronize()
    return params, start, counts, final


@pytest.mark.parametrize("first,second", [((4096, 3.7443, 1, 30, 70), (1024, 3.8, 5, 3, 9)),
                                          ((256, 3.9, 2, 0, 130), (100, 4.2, 3, 7, 40))])
def test_static_sweep_equals_handle_sweep_twice(env, first, second):
    pgg, torch = env
    stream = torch.cuda.Stream()
    for (L, r, seed, t_start, n) in (first, second):
        say("pgg_sweep_static vs pgg_sweep: L", L, "r", r, "seed", seed, "t", t_start, "+", n)
        params, start, ref_counts, ref_final = _handle_run(pgg, torch, L, r, seed, t_start, n)
        lat = start.clone()
        counts = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        pgg.pgg_sweep_static(params, lat, t_start, n, counts, stream=stream)
        stream.synchronize()
        got = counts.cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, ref_counts), "counts differ (L = %d)" % L
        assert torch.equal(lat, ref_final), "lattice differs (L = %d)" % L
        # the same again without caller counts (the array's own count slot)
        lat2 = start.clone()
        torch.cuda.synchronize()
        pgg.pgg_sweep_static(params, lat2, t_start, n, None, stream=stream)
        stream.synchronize()
        assert torch.equal(lat2, ref_final), "lattice differs without counts (L = %d)" % L


def test_static_sweep_rejects_what_it_cannot_hold(env):
    pgg, torch = env
    import ctypes
    lat = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    lib = pgg.load()
    for L, layout, kernel, schedule in ((4100, "bits", "auto", "colour16"), (60, "bits", "auto", "colour16"),
                                        (256, "int8", "auto", "colour16"), (256, "bits", "segment", "colour16"),
                                        (256, "bits", "auto", "tiled")):
        params = pgg.make_params(L, 3.8, layout=layout, kernel=kernel, schedule=schedule)
        st = lib.pgg_sweep_static(ctypes.byref(params), lat.data_ptr(), 0, 5, None, None)
        assert st == -1, (L, layout, kernel, schedule)
    params = pgg.make_params(256, 3.8)
    assert lib.pgg_sweep_static(ctypes.byref(params), None, 0, 5, None, None) == -1
    assert lib.pgg_sweep_static(ctypes.byref(params), lat.data_ptr(), 2**32 - 3, 5, None, None) == -1
    assert pgg.pgg_sweep_static_scratch_bytes() > 2 * 1024 * 1024

"""GPU: the job server (continuous batching) gives every job the result it
gets alone, bit for bit, while admission keeps device use under the budget."""
import numpy as np
import pytest

from paper_1704_08098_amd import server, workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pgg(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.set_device(0)
    from paper_1704_08098_amd import pgg as mod
    mod.load()
    return mod


def _jobs():
    jobs = wl.serving_trace(14, rate_per_s=400.0, master_seed=11, L_range=(64, 260), mcs_range=(20, 90))
    return jobs


def test_mixed_jobs_equal_their_solo_runs(pgg, oracle_lib):
    jobs = _jobs()
    chunk = 8
    budget = 3 * pgg.ServerEngine.job_bytes(260, chunk)
    say("server with", len(jobs), "jobs, budget", budget)
    with pgg.ServerEngine(budget, max_L=512, max_resident=64, chunk=chunk) as eng:
        rep = server.serve(eng, jobs, keep_results=True)
        st = eng.stats()
    assert st["completed"] == len(jobs)
    assert st["peak_bytes"] <= st["budget"]
    assert rep["max_resident"] >= 2  # work of several jobs overlapped on the device
    for k, j in enumerate(jobs):
        counts, lat = rep["results"][k]
        with pgg.Sim(j["L"], j["r"], j["K"], j["p0"], j["seed"], "bits", "segment") as sim:
            c = sim.sweep(j["sweeps"])
            assert np.array_equal(counts, c), k
            assert np.array_equal(lat, sim.read_lattice()), k
    for k in (0, 5):
        j = jobs[k]
        ref, _, ref_counts = oracle_lib.run(j["L"], j["r"], j["K"], j["p0"], j["seed"], j["sweeps"])
        assert np.array_equal(rep["results"][k][0], ref_counts)
        assert np.array_equal(rep["results"][k][1], ref)


def test_alone_equals_in_the_mix(pgg):
    jobs = _jobs()
    chunk = 8
    k = 3
    with pgg.ServerEngine(pgg.ServerEngine.job_bytes(512, chunk), max_L=512, chunk=chunk) as eng:
        alone = server.serve(eng, [dict(jobs[k], arrival=0.0)], keep_results=True)["results"][0]
    with pgg.ServerEngine(8 * pgg.ServerEngine.job_bytes(260, chunk), max_L=512, chunk=chunk) as eng:
        mix = server.serve(eng, jobs, keep_results=True)["results"][k]
    assert np.array_equal(alone[0], mix[0])
    assert np.array_equal(alone[1], mix[1])


def test_admission_rules(pgg):
    chunk = 4
    b = pgg.ServerEngine.job_bytes(128, chunk)
    assert pgg.ServerEngine.job_bytes(256, chunk) > b
    with pgg.ServerEngine(b, max_L=256, chunk=chunk) as eng:
        with pytest.raises(pgg.PggError):
            eng.submit(256, 3.8, 10)  # larger than the whole budget
        with pytest.raises(pgg.PggError):
            eng.submit(60, 3.8, 10)   # below the smallest L
        with pytest.raises(pgg.PggError):
            eng.submit(512, 3.8, 10)  # above max_L
    with pgg.ServerEngine(2 * b, max_L=256, chunk=chunk) as eng:
        ids = [eng.submit(128, 3.8 + 0.1 * q, 6, seed=q + 1) for q in range(5)]
        assert eng.step() == 2        # only two fit
        assert eng.stats()["queued"] == 3
        done = []
        while len(done) < 5:
            eng.step()
            done += eng.completed()
        assert sorted(done) == sorted(ids)
        assert eng.stats()["peak_bytes"] <= 2 * b

"""GPU: the paper's benchmark workload with the double tiling of Sec. IV
against a stored trajectory of oracle C (tests/golden/make_trajectories.py)."""
import hashlib
import os

import numpy as np
import pytest

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


def _golden(name):
    params, marks, counts = {}, {}, {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            if key == "lattice":
                marks[int(rest[0])] = rest[1]
            elif key == "count":
                counts[int(rest[0])] = int(rest[1])
            else:
                params[key] = float(rest[0]) if key in ("r", "K", "p0") else int(rest[0])
    return params, marks, np.array([counts[t] for t in range(len(counts))], dtype=np.uint64)


def test_paper_workload_tiled_against_stored_oracle_trajectory(pgg):
    """L = 4096, r = 3.98, seed 1, the double tiling, as bench.py's
    paper_workload pass runs it (a side stream, calls of 20, 500 and 500
    steps): N_C after every one of 1020 steps and the lattice after 20, 520
    and 1020 steps equal oracle C's stored trajectory."""
    import torch
    params, marks, counts = _golden("tiled_L4096_r3.98_seed1.txt")
    L, r, K, p0, seed = params["L"], params["r"], params["K"], params["p0"], params["seed"]
    assert (L, r, seed) == (4096, 3.98, 1)
    stream = torch.cuda.Stream()
    say("paper workload, tiled, vs stored oracle C trajectory")

    def digest(sim):
        return hashlib.sha256(sim.read_lattice().tobytes()).hexdigest()

    with pgg.Sim(L, r, K, p0, seed, "bits", "auto", stream=stream, schedule="tiled") as sim:
        assert sim.coop_count() == int(counts[0])
        got = [sim.sweep(20)]
        assert digest(sim) == marks[20]
        got += [sim.sweep(500)]
        assert digest(sim) == marks[520]
        got += [sim.sweep(500)]
        assert digest(sim) == marks[1020]
        got = np.concatenate(got)
        bad = np.flatnonzero(got != counts[1:])
        assert bad.size == 0, "first differing step %d" % (bad[0] + 1 if bad.size else -1)

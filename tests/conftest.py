import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def helper_bin(tmp_path_factory, oracle_lib):
    """Compile a test helper program from tests/csrc on demand."""
    out_dir = tmp_path_factory.mktemp("helpers")
    cache = {}

    def get(name):
        if name in cache:
            return cache[name]
        src = os.path.join(HERE, "csrc", name)
        exe = str(out_dir / os.path.splitext(name)[0])
        if name.endswith(".cpp"):
            hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
            if not os.path.exists(hipcc):
                pytest.skip("hipcc not available")
            cmd = [hipcc, "-O1", "--offload-arch=gfx950", src, "-o", exe]
        else:
            lib = os.path.join(ROOT, "oracle", "libpgg_oracle.so")
            cmd = ["gcc", "-O2", "-std=c99", src, lib, "-Wl,-rpath," + os.path.dirname(lib),
                   "-lm", "-o", exe]
        subprocess.check_call(cmd)
        cache[name] = exe
        return exe

    return get


@pytest.fixture(scope="session")
def rocrand_philox(helper_bin):
    """Philox4x32-10 from rocRAND's own header (an independent implementation).

    Takes an (n, 6) array of [c0, c1, c2, c3, k0, k1] rows, returns (n, 4).
    """
    import numpy as np
    exe = helper_bin("rocrand_philox.cpp")

    def run(rows):
        rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 6)
        text = "\n".join(" ".join("%x" % int(v) for v in row) for row in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        vals = [int(tok, 16) for tok in out.split()]
        return np.array(vals, dtype=np.uint64).reshape(-1, 4).astype(np.uint32)

    return run

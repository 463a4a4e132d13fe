import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    # tuning choices made by the tests (a few sweeps each) go to a file of this run only, never to the
    # user's cache, where a later benchmark would pick them up
    import tempfile
    os.environ["SPIN_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="spin-tune-"), "tune.txt")
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long statistical run")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def rocrand_philox(tmp_path_factory):
    """Callable (counters[n,4], key[2]) -> words[n,4] from rocRAND's own Philox4x32-10."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rocrand") / "rrp")
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")
    subprocess.check_call([hipcc, "-O1", "-w", "-o", exe, src])
    import numpy as np

    def run(counters, key):
        counters = np.asarray(counters, dtype=np.uint64).reshape(-1, 4)
        lines = "".join("%d %d %d %d %d %d\n" % (c[0], c[1], c[2], c[3], key[0], key[1]) for c in counters)
        out = subprocess.run([exe], input=lines.encode(), stdout=subprocess.PIPE, check=True).stdout
        return np.array([[int(v) for v in ln.split()] for ln in out.decode().splitlines()], dtype=np.uint32)

    return run

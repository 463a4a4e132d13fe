"""The persistent launch's autotuner (spin_batch_autotune): plans per lattice
shape chosen by timing, identical bits under every plan, persisted records
read back by a later process."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    return torch


def pool_descs():
    ds = [dict(model=1, L=16, d=3, seed=workloads.seed(0x800), replica=r, coupling_seed=workloads.seed(0x801),
               realisation=r // 4) for r in range(48)]
    ds += [dict(model=0, L=64, d=2, seed=workloads.seed(0x802), replica=r) for r in range(24)]
    return ds


def run_pool(ds, n, beta, every):
    b = spin.Batch(ds)
    recs = b.sweep(n, beta, every)
    spins = [b.spins(i).tobytes() for i in range(len(ds))]
    b.close()
    return [(e.tolist(), m.tolist()) for e, m in recs], spins


def test_autotune_plans_persist_and_keep_bits(oracle_mod):
    ds = pool_descs()
    note("batch autotune: pool of", len(ds), "lattices, untuned run first")
    before = run_pool(ds, 12, 0.7, 4)
    b = spin.Batch(ds)
    tuned = b.autotune(0.7, 5)
    assert tuned == 2
    p16 = spin.batch_plan(3, 1, 16)
    p64 = spin.batch_plan(2, 0, 64)
    note("plans: 3D +-J L=16", p16, " 2D Ising L=64", p64)
    assert p16 is not None and p64 is not None
    for nt, w in (p16, p64):
        assert nt in (256, 512, 576, 1024) and 1 <= w <= 2048 // nt
    assert all(b.t(i) == 0 for i in range(len(ds)))        # the pool's own lattices untouched
    b.close()
    after = run_pool(ds, 12, 0.7, 4)
    assert after == before, "results changed under the tuned plans"
    # the oracle agrees on one lattice of each shape
    for i in (5, 60):
        d = ds[i]
        J = oracle_mod.couplings(d["L"], d["d"], d["coupling_seed"], d["realisation"]) if d["model"] == 1 else None
        ch = oracle_mod.Chain(d["L"], d["d"], d["seed"], d["replica"], J=J)
        Eo, Mo = ch.sweep(12, 0.7, every=4)
        assert after[0][i] == (list(Eo), list(Mo))
        assert after[1][i] == ch.spins.tobytes()
    # persisted: a fresh process reads the plans back from the cache file
    path = os.environ["SPIN_TUNE_CACHE"]
    lines = [ln.split() for ln in open(path) if ln.startswith("batch ")]
    assert any(ln[2:5] == ["3", "1", "16"] for ln in lines) and any(ln[2:5] == ["2", "0", "64"] for ln in lines)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1006_3865_amd import spin\n"
            "print('plan', spin.batch_plan(3, 1, 16), spin.batch_plan(2, 0, 64))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, SPIN_TUNE_CACHE=path))
    assert out.returncode == 0, out.stderr
    assert "plan %r %r" % (p16, p64) in out.stdout

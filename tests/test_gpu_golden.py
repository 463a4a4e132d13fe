"""Full-length runs of the benchmark configurations against stored oracle records.

tests/golden/full_*.json are written by tests/golden/make_full_runs.py, which
runs only the CPU oracle.  Each GPU run here takes the launch configuration
that bench.py times (library's kernel choice, calls of `every` sweeps with
device records for the single lattices; one pool call for the batch) and
must reproduce every (E, M) record and the SHA-256 of the spins at the
stored checkpoints bit for bit.  A record file that has not been generated
skips its test.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(name):
    path = os.path.join(HERE, "full_" + name + ".json")
    if not os.path.exists(path):
        pytest.skip("record %s not generated (tests/golden/make_full_runs.py)" % name)
    with open(path) as f:
        return json.load(f)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    return torch


def run_single(torch, rec):
    L, d, every, sweeps = rec["L"], rec["d"], rec["every"], rec["sweeps"]
    beta = float.fromhex(rec["beta_hex"])
    stream = torch.cuda.Stream()
    lat = spin.Lattice(rec["model"], L, d, rec["seed"], replica=rec["replica"], stream=stream)
    note("golden L", L, "d", d, "beta", beta, "kernel", spin.KERNEL_NAMES[lat.kernel])
    nrec = sweeps // every
    E = torch.zeros(nrec, dtype=torch.int64, device="cuda")
    M = torch.zeros(nrec, dtype=torch.int64, device="cuda")
    hashes = {}
    for k in range(nrec):
        lat.sweep_record_device(every, beta, every, E[k:], M[k:])
        if str(lat.t) in rec["spins_sha256"]:
            hashes[str(lat.t)] = sha(lat.spins())
    lat.synchronize()
    got_E, got_M = E.cpu().numpy(), M.cpu().numpy()
    lat.close()
    np.testing.assert_array_equal(got_E, np.array(rec["E"], dtype=np.int64))
    np.testing.assert_array_equal(got_M, np.array(rec["M"], dtype=np.int64))
    assert hashes == rec["spins_sha256"]


@pytest.mark.parametrize("i", [0, 1, 2])
def test_ising2d_L8192_full_run(gpu, i):
    run_single(gpu, load("ising2d_L8192_b%d" % i))


def test_ising3d_L512_full_run(gpu):
    run_single(gpu, load("ising3d_L512"))


def test_ea3d_batch_subset_full_run(gpu):
    """The stratified subset of the batched 3D +-J workload (2 realisations per L x 16 betas), 5000
    sweeps in one pool call with records every 100, as the batched benchmark runs it."""
    torch = gpu
    recs = []
    for part in range(4):
        data = load("ea3d_subset_%d" % part)
        for lat in data["lattices"]:
            recs.append((data, lat))
    descs = [dict(model=1, L=l["L"], d=3, coupling_seed=data["coupling_seed"], realisation=l["realisation"],
                  seed=data["seed"], replica=l["replica"]) for data, l in recs]
    betas = np.array([float.fromhex(l["beta_hex"]) for _, l in recs])
    sweeps, every = recs[0][0]["sweeps"], recs[0][0]["every"]
    stream = torch.cuda.Stream()
    b = spin.Batch(descs, stream=stream)
    counts = b.record_counts(sweeps, every)
    tot = int(counts.sum())
    E = torch.zeros(tot, dtype=torch.int64, device="cuda")
    M = torch.zeros(tot, dtype=torch.int64, device="cuda")
    b.sweep_device(sweeps, betas, every, E, M)
    b.synchronize()
    E, M = E.cpu().numpy(), M.cpu().numpy()
    o = 0
    for i, (_, l) in enumerate(recs):
        c = int(counts[i])
        np.testing.assert_array_equal(E[o:o + c], np.array(l["E"]), err_msg="E of lattice %d" % i)
        np.testing.assert_array_equal(M[o:o + c], np.array(l["M"]), err_msg="M of lattice %d" % i)
        o += c
        assert sha(b.spins(i)) == l["spins_sha256"]["5000"], "spins of lattice %d" % i
    b.close()

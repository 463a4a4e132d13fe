"""Injected device-allocation failures on the GPU: every constructor and the
calls that allocate on first use return SPIN_ENOMEM when the k-th allocation
fails, hold no device memory afterwards, and an object built once injection
no longer fires computes the same bits as one built without it.
"""
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    spin.use_hip_allocator()
    yield torch
    spin.fault_alloc(-1)


def sweep_lattice(obj):
    E, M = obj.sweep_record(4, 0.5, 2)
    return np.asarray(E).tolist(), np.asarray(M).tolist(), obj.spins().tobytes()


def sweep_batch(obj):
    rec = obj.sweep(3, 0.7, 3)
    return [(np.asarray(e).tolist(), np.asarray(m).tolist()) for e, m in rec], \
        [obj.spins(i).tobytes() for i in obj.members()]


def sweep_msc(obj):
    E, M = obj.sweep_record(4, 1.2, 2)
    return np.asarray(E).tolist(), np.asarray(M).tolist(), obj.spins(5).tobytes()


def sweep_heis(obj):
    obj.sweep(3, 0.7)
    return obj.spins().tobytes()


DESCS = [dict(model=1, L=16, d=3, seed=workloads.seed(0x40), coupling_seed=workloads.seed(0x41), replica=r)
         for r in range(3)] + [dict(model=0, L=512, d=2, seed=workloads.seed(0x42))]

MAKERS = [
    ("2D Ising L=1024", lambda: spin.Lattice(0, 1024, 2, workloads.seed(0x43)), sweep_lattice),
    ("3D +-J L=64", lambda: spin.Lattice(1, 64, 3, workloads.seed(0x44), coupling_seed=workloads.seed(0x45)),
     sweep_lattice),
    ("batch of 3 LDS-sized +-J and one 2D L=512", lambda: spin.Batch(DESCS), sweep_batch),
    ("multi-spin 3D L=32", lambda: spin.Msc(32, 3, workloads.seed(0x46), 0, workloads.seed(0x47)), sweep_msc),
    ("Heisenberg 2D L=64", lambda: spin.Heis(64, 2, workloads.seed(0x48)), sweep_heis),
]


@pytest.mark.parametrize("name,make,run", MAKERS, ids=[m[0] for m in MAKERS])
def test_injected_allocation_failures(name, make, run):
    base = spin.live_allocations()
    ref_obj = make()
    ref = run(ref_obj)
    ref_obj.close()
    assert spin.live_allocations() == base
    fired = 0
    for k in range(64):
        note("fault injection: %s, allocation %d fails" % (name, k))
        spin.fault_alloc(k)
        try:
            obj = make()
        except spin.SpinError as e:
            spin.fault_alloc(-1)
            assert e.code == spin.SPIN_ENOMEM, str(e)
            assert spin.live_allocations() == base, "blocks leaked after a failed constructor"
            fired += 1
            continue
        try:
            got = run(obj)
        except spin.SpinError as e:
            # the failure hit an allocation made on first use by the call itself
            assert e.code == spin.SPIN_ENOMEM, str(e)
            spin.fault_alloc(-1)
            obj.close()
            assert spin.live_allocations() == base
            fired += 1
            continue
        spin.fault_alloc(-1)
        obj.close()
        assert got == ref, "results changed after surviving injection"
        assert spin.live_allocations() == base
        break
    else:
        pytest.fail("injection kept firing for 64 allocations")
    assert fired >= 1

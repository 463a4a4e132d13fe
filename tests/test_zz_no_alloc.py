"""The allocation-free sweep entry point (spin_sweep_record_noalloc) against
spin_sweep_record_device, through the C ABI.

Twin handles (same model, L, d, seed, couplings) are swept with the same n,
beta and record cadence, one through each entry point; records and final
spins must be identical bit for bit.  Each case makes two calls in a row,
the second on a smaller lattice, so that the second call runs on scratch the
first one left filled.  A counting allocator hook checks that the
allocation-free call requests no device memory.
"""
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingAllocator:
    """Allocator hook that counts calls and delegates to torch's caching allocator."""

    def __init__(self, torch):
        self.calls = 0
        self.torch = torch

        def _alloc(nbytes, ctx):
            self.calls += 1
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
            except Exception:
                return None

        def _release(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.hooks = (spin.ALLOC_FN(_alloc), spin.RELEASE_FN(_release))
        spin.load().spin_set_allocator(self.hooks[0], self.hooks[1], None)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    alloc = CountingAllocator(torch)
    yield torch, alloc
    spin.use_hip_allocator()


def twins(model, L, d, seed, cseed=None, kernel=spin.SPIN_KERNEL_AUTO):
    out = []
    for _ in range(2):
        lat = spin.Lattice(model, L, d, seed, coupling_seed=cseed)
        if kernel != spin.SPIN_KERNEL_AUTO:
            lat.set_kernel(kernel)
        out.append(lat)
    return out


# (model, L, d, coupling seed, kernel, n, every, beta): pairs, the second smaller than the first
CASES = [
    ("2D L=8192 streaming, then L=256",
     (0, 8192, 2, None, spin.SPIN_KERNEL_AUTO, 20, 10, workloads.BETA_2D_CRIT),
     (0, 256, 2, None, spin.SPIN_KERNEL_FUSED, 12, 3, 0.6)),
    ("3D L=512 register-column, then 3D +-J L=24 streaming",
     (0, 512, 3, None, spin.SPIN_KERNEL_AUTO, 10, 5, workloads.BETA_3D),
     (1, 24, 3, workloads.seed(0x11), spin.SPIN_KERNEL_STREAM, 6, 2, 1.1)),
    ("2D L=128 LDS-resident, then L=64",
     (0, 128, 2, None, spin.SPIN_KERNEL_AUTO, 30, 1, workloads.BETA_2D_CRIT),
     (0, 64, 2, None, spin.SPIN_KERNEL_AUTO, 10, 1, 0.3)),
    ("3D L=96 tiled per colour with the measure kernel, then 2D L=48 generic",
     (0, 96, 3, None, spin.SPIN_KERNEL_TILED, 8, 2, workloads.BETA_3D),
     (0, 48, 2, None, spin.SPIN_KERNEL_GENERIC, 6, 3, 0.44)),
]


@pytest.mark.parametrize("name,first,second", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_record_device(torch_mod, name, first, second):
    torch, alloc = torch_mod
    seed = workloads.seed(0x31)
    for step, (model, L, d, cseed, kernel, n, every, beta) in enumerate((first, second)):
        note("no-alloc case %s, call %d: model=%d L=%d d=%d n=%d every=%d beta=%r"
             % (name, step + 1, model, L, d, n, every, beta))
        a, b = twins(model, L, d, seed, cseed, kernel)
        nrec = n // every
        Ea = torch.full((nrec,), -7, dtype=torch.int64, device="cuda")
        Ma = torch.full((nrec,), -7, dtype=torch.int64, device="cuda")
        Eb = torch.zeros(nrec, dtype=torch.int64, device="cuda")
        Mb = torch.zeros(nrec, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        before = alloc.calls
        a.sweep_record_noalloc(n, beta, every, Ea, Ma)
        assert alloc.calls == before, "the allocation-free call asked the allocator for memory"
        b.sweep_record_device(n, beta, every, Eb, Mb)
        torch.cuda.synchronize()
        assert torch.equal(Ea, Eb) and torch.equal(Ma, Mb), "records differ between the two entry points"
        assert np.array_equal(a.spins(), b.spins()), "spins differ between the two entry points"
        assert a.t == b.t == n
        a.close()
        b.close()


def test_noalloc_rejects_records_beyond_scratch(torch_mod):
    torch, alloc = torch_mod
    # 3D L=512 on the register-column kernel: 512 counting workgroups (16-row slabs, 32-plane strips),
    # 8 KiB of partials per record
    lat = spin.Lattice(0, 512, 3, workloads.seed(0x32))
    per_record = 512 * 16
    nrec = spin.NOALLOC_SCRATCH_BYTES // per_record + 1
    E = torch.zeros(nrec, dtype=torch.int64, device="cuda")
    M = torch.zeros(nrec, dtype=torch.int64, device="cuda")
    with pytest.raises(spin.SpinError) as ei:
        lat.sweep_record_noalloc(nrec, workloads.BETA_3D, 1, E, M)
    assert ei.value.code == spin.SPIN_EINVAL
    assert "scratch" in str(ei.value)
    assert lat.t == 0
    lat.close()

"""Failure paths of the C ABI that the host can force without a GPU.

Allocation failures are injected with spin_debug_fault_alloc (or the
SPIN_FAULT_ALLOC environment variable).  A host-memory allocator hook stands
in for device memory, so the constructor gets as far as its first allocation
failure (or, with no injection, its first device call, which fails here
because there is no GPU) and the test can check that it returns the right
status and gives back every block it took.
"""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_1006_3865_amd import spin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class HostBlocks:
    """Allocator hook handing out host buffers; tracks what is outstanding."""

    def __init__(self):
        self.held = {}
        self.calls = 0

        def _alloc(n, ctx):
            self.calls += 1
            b = ctypes.create_string_buffer(int(n))
            p = ctypes.addressof(b)
            self.held[p] = b
            return p

        def _release(p, ctx):
            self.held.pop(p)

        self.hooks = (spin.ALLOC_FN(_alloc), spin.RELEASE_FN(_release))

    def install(self):
        spin.load().spin_set_allocator(self.hooks[0], self.hooks[1], None)


@pytest.fixture
def host_blocks():
    spin.load()
    hb = HostBlocks()
    hb.install()
    yield hb
    spin.fault_alloc(-1)
    spin.use_hip_allocator()


def test_injected_failure_of_the_first_allocation(host_blocks):
    base = spin.live_allocations()
    spin.fault_alloc(0)
    with pytest.raises(spin.SpinError) as ei:
        spin.Lattice(spin.SPIN_ISING, 64, 2, 1)
    assert ei.value.code == spin.SPIN_ENOMEM
    assert "allocation" in str(ei.value)
    assert host_blocks.held == {}          # whatever the constructor took went back
    assert spin.live_allocations() == base


@pytest.mark.parametrize("after", [1, 2])
def test_injected_failure_later_releases_earlier_blocks(host_blocks, after):
    base = spin.live_allocations()
    spin.fault_alloc(after)
    with pytest.raises(spin.SpinError) as ei:
        spin.Lattice(spin.SPIN_EA_PMJ, 32, 3, 1, couplings=[1] * (3 * 32 ** 3))
    assert ei.value.code == spin.SPIN_ENOMEM
    assert host_blocks.calls >= after      # blocks before the failure came from the hook ...
    assert host_blocks.held == {}          # ... and went back to it
    assert spin.live_allocations() == base


def test_injection_fires_once(host_blocks):
    spin.fault_alloc(0)
    with pytest.raises(spin.SpinError) as ei:
        spin.Lattice(spin.SPIN_ISING, 16, 2, 1)
    assert ei.value.code == spin.SPIN_ENOMEM
    # off again: the next constructor allocates everything and fails only at its first device
    # call (no GPU here), releasing all it took
    with pytest.raises(spin.SpinError) as ei:
        spin.Lattice(spin.SPIN_ISING, 16, 2, 1)
    assert ei.value.code == spin.SPIN_EDEVICE
    assert host_blocks.calls >= 2
    assert host_blocks.held == {}


def test_fault_alloc_argument_checked():
    spin.load()
    with pytest.raises(spin.SpinError) as ei:
        spin.fault_alloc(-2)
    assert ei.value.code == spin.SPIN_EINVAL


def test_environment_variable_sets_injection():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1006_3865_amd import spin\n"
        "try:\n"
        "    spin.Lattice(0, 64, 2, 1)\n"
        "except spin.SpinError as e:\n"
        "    print('status', e.code)\n" % ROOT)
    env = dict(os.environ, SPIN_FAULT_ALLOC="0")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "status %d" % spin.SPIN_ENOMEM in out.stdout

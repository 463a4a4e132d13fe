"""GPU parity of the multi-spin-coded +-J glass (32 systems per word) against the oracle.

Every one of the 32 systems' spins, and the 32 energies and magnetisations
after every sweep, equal the oracle's multi-spin-coded mode bit for bit, in
2D and 3D, at several inverse temperatures (including 0, inf and 3).
"""
import math
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
    return torch


@pytest.mark.parametrize("L,d,kernel", [
    (8, 2, None), (16, 2, None), (64, 2, None), (8, 3, None), (16, 3, None), (24, 3, None),
    (16, 2, (0, 0, 0, 0)), (24, 3, (0, 0, 0, 0)),                 # one launch per colour
    (40, 2, (1, 0, 7, 512)), (24, 3, (1, 4, 5, 256)), (32, 3, (1, 16, 3, 512)), (16, 3, (1, 8, 16, 256)),
    # rows cut into segments of `width` sites (two neighbouring groups of halo each side)
    (40, 2, (1, 0, 7, 512, 8)), (64, 2, (1, 0, 5, 256, 16)), (24, 3, (1, 4, 5, 256, 8)),
    (32, 3, (1, 16, 3, 512, 16)), (48, 3, (1, 8, 16, 512, 16)), (16, 3, (1, 2, 4, 256, 8)),
])
def test_msc_matches_oracle(oracle_mod, L, d, kernel):
    cs, seed, r0, p0 = workloads.seed(0x60), workloads.seed(0x61), 5, 70
    note("msc", L, d, kernel)
    m = spin.Msc(L, d, cs, r0, seed, p0)
    if kernel is not None:
        m.set_kernel(*kernel)
    ch = oracle_mod.MscChain(L, d, cs, r0, seed, p0)
    for b in (0, 13, 31):
        np.testing.assert_array_equal(m.spins(b), ch.spins[b])
    np.testing.assert_array_equal(np.stack(m.measure()), np.stack(ch.measure()))
    for beta in (0.5, 1.1, 0.0, math.inf, 3.0, workloads.BETA_3D):
        E, M = m.sweep_record(2, beta, 1)
        Eo, Mo = ch.sweep(2, beta, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
    for b in range(32):
        np.testing.assert_array_equal(m.spins(b), ch.spins[b], err_msg="system %d" % b)
    assert m.t == ch.t
    m.close()


def test_msc_system_equals_its_own_lattice_inputs():
    """System b starts from the hot start and couplings a lone lattice of replica p0+b, realisation r0+b has."""
    L, d, cs, seed, r0, p0 = 16, 3, workloads.seed(0x62), workloads.seed(0x63), 9, 3
    m = spin.Msc(L, d, cs, r0, seed, p0)
    for b in (0, 31):
        lone = spin.Lattice(1, L, d, seed, coupling_seed=cs, realisation=r0 + b, replica=p0 + b)
        np.testing.assert_array_equal(m.spins(b), lone.spins())
        E, M = m.measure()
        assert (E[b], M[b]) == lone.measure()
        lone.close()
    m.close()


def test_msc_rejects_bad_shapes():
    for (L, d) in ((12, 2), (4, 3), (16, 4)):
        with pytest.raises(spin.SpinError):
            spin.Msc(L, d, 1, 0, 1)
    m = spin.Msc(24, 3, 1, 0, 1)
    # rows must divide L; threads 256/512; width a multiple of 8 dividing L; no negative sizes
    for k in ((1, 5, 8, 256), (1, 8, 8, 128), (1, 8, 8, 256, 12), (1, 8, 8, 256, 16), (1, -8, 8, 256)):
        with pytest.raises(spin.SpinError):
            m.set_kernel(*k)
    m.set_kernel(1, 8, 8, 256, 8)
    m.close()

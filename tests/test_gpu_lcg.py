"""GPU parity of the LCG draw modes (the RNG-quality experiment) against the oracle.

Spins, E and M after every sweep and every group's generator state after
every call equal the oracle's LCG mode bit for bit, 2D and 3D, for the
array of 32-bit generators and the disjoint sub-sequences of the 32- and
64-bit generators; switching between Philox and an LCG mode in the middle
of a run continues both chains exactly.
"""
import math
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu
MODES = [spin.SPIN_RNG_LCG32_ARRAY, spin.SPIN_RNG_LCG32_DISJOINT, spin.SPIN_RNG_LCG64_DISJOINT]


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


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,d", [(16, 2), (24, 2), (128, 2), (8, 3), (16, 3), (24, 3)])
def test_lcg_matches_oracle(oracle_mod, mode, L, d):
    seed = workloads.seed(0x70 + L + d)
    note("lcg", mode, L, d)
    lat = spin.Lattice(0, L, d, seed, replica=2)
    lat.set_rng(mode)
    ch = oracle_mod.LcgChain(L, d, seed, mode, replica=2)
    np.testing.assert_array_equal(lat.rng_state(), ch.state)
    for beta in (0.44, 0.9, 0.0, math.inf, 3.0, 0.25):
        E, M = lat.sweep_record(2, beta, 1)
        Eo, Mo = ch.sweep(2, beta, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
        np.testing.assert_array_equal(lat.spins(), ch.spins)
        np.testing.assert_array_equal(lat.rng_state(), ch.state)
    lat.close()


def test_switching_between_philox_and_lcg(oracle_mod):
    L, d, seed = 32, 2, workloads.seed(0x7F)
    lat = spin.Lattice(0, L, d, seed)
    ch = oracle_mod.Chain(L, d, seed)
    lat.sweep(3, 0.5)
    ch.sweep(3, 0.5)
    lat.set_rng(spin.SPIN_RNG_LCG64_DISJOINT)
    state = oracle_mod.lcg_init(L, d, spin.SPIN_RNG_LCG64_DISJOINT, seed, 0)
    lat.sweep(4, 0.5)
    oracle_mod.lcg_sweeps(L, d, None, ch.spins, state, spin.SPIN_RNG_LCG64_DISJOINT, 4, 0.5)
    ch.t += 4
    np.testing.assert_array_equal(lat.spins(), ch.spins)
    np.testing.assert_array_equal(lat.rng_state(), state)
    lat.set_rng(spin.SPIN_RNG_PHILOX)
    lat.sweep(3, 0.5)
    ch.sweep(3, 0.5)
    np.testing.assert_array_equal(lat.spins(), ch.spins)
    assert lat.t == ch.t == 10
    lat.close()


def test_lcg_rejects_what_it_cannot_run():
    ea = spin.Lattice(1, 16, 2, 1, coupling_seed=2)
    with pytest.raises(spin.SpinError):
        ea.set_rng(spin.SPIN_RNG_LCG32_ARRAY)          # Ising only
    ea.close()
    odd = spin.Lattice(0, 12, 2, 1)
    with pytest.raises(spin.SpinError):
        odd.set_rng(spin.SPIN_RNG_LCG32_ARRAY)         # L % 8 != 0
    odd.close()
    lat = spin.Lattice(0, 32, 2, 1)
    with pytest.raises(spin.SpinError):
        lat.set_rng(7)                                  # unknown mode
    with pytest.raises(spin.SpinError):
        lat.rng_state()                                 # Philox has no state
    lat.set_schedule(spin.SPIN_SCHEDULE_COARSE, 8, 2)
    with pytest.raises(spin.SpinError):
        lat.set_rng(spin.SPIN_RNG_LCG32_DISJOINT)      # coarse schedule draws from Philox
    lat.set_schedule(spin.SPIN_SCHEDULE_CHECKERBOARD)
    lat.set_rng(spin.SPIN_RNG_LCG32_DISJOINT)
    with pytest.raises(spin.SpinError):
        lat.set_schedule(spin.SPIN_SCHEDULE_COARSE, 8, 2)
    lat.close()

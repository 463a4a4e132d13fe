"""Pins of the oracle's multi-spin-coded +-J glass (32 systems sharing one draw per site and update).

Sec. 4, last paragraph: many disorder realisations at once, combined with
(asynchronous) multi-spin coding.  The mode has its own chain, pinned by:

* each system, on its own, is a Metropolis chain of its realisation driven by
  the shared draws: a brute-force restatement (whole-lattice energy
  differences, rocRAND's own Philox words of the shared counter) reproduces
  every system;
* systems with the same couplings and the same start stay identical;
* beta = 0 negates every spin of every system each sweep; at zero
  temperature no system's energy rises;
* each system samples its own exact Boltzmann distribution (4x4 +-J
  enumeration of all 2^16 states).
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import exact_ising as ex

CSEED, SEED = 0x1006386500000051, 0x1006386500000052


@pytest.mark.parametrize("L,d,beta", [(4, 2, 0.7), (6, 2, 1.3), (4, 3, 0.5), (8, 2, 3.0)])
def test_each_system_matches_bruteforce(oracle_mod, rocrand_philox, L, d, beta):
    r0, p0, t0, n = 3, 40, 2, 2
    ch = oracle_mod.MscChain(L, d, CSEED, r0, SEED, p0)
    start = ch.spins.copy()
    ch.t = t0
    ch.sweep(n, beta)
    N = L ** d
    ctrs, keys = [], []
    for t in range(t0, t0 + n):
        for c in (0, 1):
            for g in range((N + 7) // 8):
                ctrs.append((g, t, p0, 4 + c))
                keys.append((g, t, c))
    w = dict(zip(keys, rocrand_philox(ctrs, (SEED & 0xFFFFFFFF, SEED >> 32))))
    for b in (0, 1, 17, 31):
        ref = start[b].copy()
        J = oracle_mod.couplings(L, d, CSEED, r0 + b)
        for t in range(t0, t0 + n):
            bf.sweep(ref, L, d, J, beta, t, lambda s, tt, c: int(w[(s >> 3, tt, c)][(s >> 1) & 3]))
        np.testing.assert_array_equal(ch.spins[b], ref, err_msg="system %d" % b)


def test_identical_systems_stay_identical(oracle_mod):
    L, d = 8, 3
    J1 = oracle_mod.couplings(L, d, CSEED, 9)
    s1 = oracle_mod.init_spins(L, d, SEED, 2)
    J = np.ascontiguousarray(np.tile(J1, (32, 1)))
    spins = np.ascontiguousarray(np.tile(s1, (32, 1)))
    oracle_mod.msc_sweeps(L, d, J, spins, SEED, 2, 0, 5, 0.9)
    assert (spins == spins[0]).all()
    assert not np.array_equal(spins[0], s1)


def test_infinite_and_zero_temperature(oracle_mod):
    ch = oracle_mod.MscChain(8, 3, CSEED, 0, SEED, 0)
    s0 = ch.spins.copy()
    ch.sweep(1, 0.0)
    np.testing.assert_array_equal(ch.spins, -s0)
    e_prev, _ = ch.measure()
    E, _ = ch.sweep(15, math.inf, every=1)
    for e in E:
        assert (e <= e_prev).all()
        e_prev = e
    assert (E[-1] < E[0]).any()


def _ea_exact_energy(L, J, beta):
    """<E> of a 2D +-J L x L torus by enumerating all 2^(L*L) states."""
    N = L * L
    states = ((np.arange(1 << N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int8) * 2 - 1
    E = np.zeros(1 << N)
    for s in range(N):
        x, y = s % L, s // L
        for dr, nb in ((0, y * L + (x + 1) % L), (1, ((y + 1) % L) * L + x)):
            E -= J[dr * N + s] * states[:, s] * states[:, nb]
    w = np.exp(-beta * (E - E.min()))
    return float((w * E).sum() / w.sum())


def test_systems_sample_their_boltzmann_distribution(oracle_mod):
    L, beta = 4, 0.8
    ch = oracle_mod.MscChain(L, 2, CSEED, 0, SEED, 0)
    ch.sweep(500, beta)
    E, _ = ch.sweep(120000, beta, every=1)
    for b in (0, 5, 31):
        exact = _ea_exact_energy(L, ch.J[b], beta)
        u, du = ex.binned_mean_error(E[:, b])
        assert du < 0.05
        assert abs(u - exact) < 5 * du, (b, u, exact, du)


def test_bad_arguments_rejected(oracle_mod):
    spins = np.zeros(32 * 16, dtype=np.int8)
    J = np.ones(32 * 2 * 16, dtype=np.int8)
    with pytest.raises(ValueError):
        oracle_mod.msc_sweeps(4, 2, J, spins, 1, 0, 0, 1, -1.0)
    with pytest.raises(ValueError):
        oracle_mod.msc_sweeps(4, 2, J, spins, 1, 0, (1 << 32) - 1, 2, 0.5)

"""Pins of the oracle's coarse-tile multi-hit schedule (the paper's own order of updates).

Sec. 3, steps 1-7, and the generalized multi-hit paragraph after them: even
coarse tiles, then odd ones, each tile updating its two fine sub-lattices k
times.  The mode has its own chain (it depends on the tile edge T and on k),
so it is pinned by what fixes it independently of the oracle's code:

* with T = 1 and k = 1 it is the canonical red/black chain (itself pinned in
  test_oracle_pins.py) -- same bits;
* a brute-force restatement (whole-lattice energy differences, rocRAND's own
  Philox draws, the paper's steps spelled out) on tiny lattices;
* beta = 0 accepts every move, so one sweep multiplies the spins by (-1)^k;
* at zero temperature no update raises the energy;
* every single-site update keeps the Boltzmann distribution, so the chain
  samples the exact 4x4 enumeration averages.
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import exact_ising as ex

SEED = 0x1006386500000031


@pytest.mark.parametrize("L,d,ea", [(8, 2, False), (12, 2, True), (6, 3, False), (4, 3, True), (10, 2, False)])
def test_tile_one_single_hit_is_the_canonical_chain(oracle_mod, L, d, ea):
    J = oracle_mod.couplings(L, d, 0x77, 1) if ea else None
    a = oracle_mod.Chain(L, d, SEED, 2, J=J)
    b = oracle_mod.Chain(L, d, SEED, 2, J=J)
    a.sweep(3, 0.5)
    b.coarse_sweep(3, 0.5, 1, 1)
    for beta in (0.3, 0.9, 3.0):
        Ea, Ma = a.sweep(4, beta, every=1)
        Eb, Mb = b.coarse_sweep(4, beta, 1, 1, every=1)
        np.testing.assert_array_equal(Ea, Eb)
        np.testing.assert_array_equal(Ma, Mb)
        np.testing.assert_array_equal(a.spins, b.spins)


@pytest.mark.parametrize("L,d,ea,T,k,beta", [
    (8, 2, False, 2, 2, 0.44), (8, 2, True, 4, 3, 0.8), (4, 2, False, 2, 1, 0.3),
    (12, 2, False, 3, 2, 0.6), (4, 3, True, 2, 2, 0.5), (8, 3, False, 4, 1, 0.25),
])
def test_coarse_sweep_matches_bruteforce(oracle_mod, rocrand_philox, L, d, ea, T, k, beta):
    rng = np.random.default_rng(L * 100 + T * 10 + k)
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d) if ea else None
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=L ** d)
    seed, rep, t0, n = SEED, 3, 5, 2
    got = s0.copy()
    oracle_mod.coarse_sweeps(L, d, J, got, seed, rep, t0, n, beta, T, k)
    N = L ** d
    ctrs, keys = [], []
    for t in range(t0, t0 + n):
        for h in range(k):
            for c in (0, 1):
                for g in range((N + 7) // 8):
                    ctrs.append((g, t * k + h, rep, c))
                    keys.append((g, t * k + h, c))
    w = dict(zip(keys, rocrand_philox(ctrs, (seed & 0xFFFFFFFF, seed >> 32))))
    ref = s0.copy()
    for t in range(t0, t0 + n):
        bf.coarse_sweep(ref, L, d, J, beta, t, T, k, lambda s, hit, c: int(w[(s >> 3, hit, c)][(s >> 1) & 3]))
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_infinite_temperature_flips_k_times(oracle_mod, k):
    for (L, d, T) in ((16, 2, 4), (8, 3, 2)):
        ch = oracle_mod.Chain(L, d, SEED, 0)
        s0 = ch.spins.copy()
        ch.coarse_sweep(1, 0.0, T, k)
        np.testing.assert_array_equal(ch.spins, s0 * (-1) ** k)


def test_zero_temperature_never_raises_energy(oracle_mod):
    for (L, d, ea, T, k) in ((16, 2, False, 4, 2), (16, 2, True, 8, 3), (8, 3, True, 2, 2)):
        J = oracle_mod.couplings(L, d, 0x55, 0) if ea else None
        ch = oracle_mod.Chain(L, d, SEED + L, 1, J=J)
        e_prev = ch.measure()[0]
        E, _ = ch.coarse_sweep(20, math.inf, T, k, every=1)
        for e in E:
            assert e <= e_prev
            e_prev = e
        assert E[-1] < E[0] or E[0] == -d * L ** d


@pytest.mark.parametrize("k", [1, 3])
def test_4x4_coarse_chain_samples_boltzmann(oracle_mod, k):
    beta = float.fromhex("0x1.c34366871d961p-2")  # 0.4406868
    ch = oracle_mod.Chain(4, 2, 0x1006386500000004)
    ch.coarse_sweep(1000, beta, 2, k)
    E, M = ch.coarse_sweep(400000, beta, 2, k, every=1)
    exact = ex.enumeration_averages(4, beta)
    u, du = ex.binned_mean_error(E / 16)
    am, dam = ex.binned_mean_error(np.abs(M) / 16)
    assert du < 3e-3
    assert abs(u - exact["u"]) < 5 * du, (u, exact["u"], du)
    assert abs(am - exact["abs_m"]) < 5 * dam, (am, exact["abs_m"], dam)


def test_bad_tiles_rejected(oracle_mod):
    s = oracle_mod.init_spins(12, 2, 1)
    for (T, k) in ((5, 1), (4, 1), (12, 1), (2, 0)):   # T does not divide L; L/T odd (3); L/T = 1; k < 1
        with pytest.raises(ValueError):
            oracle_mod.coarse_sweeps(12, 2, None, s, 1, 0, 0, 1, 0.5, T, k)

"""Pins of the oracle's LCG mode (the RNG-quality experiment of Sec. 4, first paragraph).

* The 32-bit generator (a = 1664525, c = 1013904223) started from 0 gives the
  sequence printed for it in Numerical Recipes (2nd ed., Sec. 7.1, the
  "quick and dirty" generator): 1013904223, 1196435762, 3519870697, ...
* Skip-ahead by squaring equals stepping one at a time, composes, and the
  generators have full period (2^32 and 2^64: c odd, a = 1 mod 4).
* Initial states: the array mode takes Philox words (pinned to rocRAND);
  in the disjoint modes, group g + 1 starts exactly where group g's block of
  floor(2^P / G) draws ends.
* One sweep equals a brute-force restatement (whole-lattice energy
  differences) driven by per-group streams drawn in increasing x; beta = 0
  flips every spin; at zero temperature the energy never rises.
"""
import math

import numpy as np
import pytest

import bruteforce as bf

SEED = 0x1006386500000071
A32, C32 = 1664525, 1013904223
A64, C64 = 6364136223846793005, 1442695040888963407


def step(mode, x):
    if mode == 3:
        return (A64 * x + C64) % (1 << 64)
    return (A32 * x + C32) % (1 << 32)


def out(mode, x):
    return x >> 32 if mode == 3 else x


def test_numerical_recipes_sequence(oracle_mod):
    x, seq = 0, []
    for _ in range(5):
        x = oracle_mod.lcg_skip(1, x, 1)
        seq.append(x)
    assert seq == [1013904223, 1196435762, 3519870697, 2868466484, 1649599747]


@pytest.mark.parametrize("mode", [1, 3])
def test_skip_equals_stepping(oracle_mod, mode):
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = int(rng.integers(0, 1 << 62)) if mode == 3 else int(rng.integers(0, 1 << 32))
        k = int(rng.integers(0, 3000))
        y = x
        for _ in range(k):
            y = step(mode, y)
        assert oracle_mod.lcg_skip(mode, x, k) == y


@pytest.mark.parametrize("mode", [2, 3])
def test_skip_composes_and_full_period(oracle_mod, mode):
    x = 123456789
    a, b = (1 << 40) + 977, (1 << 37) + 12345
    assert oracle_mod.lcg_skip(mode, oracle_mod.lcg_skip(mode, x, a), b) == oracle_mod.lcg_skip(mode, x, a + b)
    if mode == 3:
        half = oracle_mod.lcg_skip(mode, x, 1 << 63)
        assert half != x and oracle_mod.lcg_skip(mode, half, 1 << 63) == x
    else:
        assert oracle_mod.lcg_skip(mode, x, 1 << 31) != x
        assert oracle_mod.lcg_skip(mode, x, 1 << 32) == x


def test_array_mode_seeds_are_philox_words(oracle_mod, rocrand_philox):
    L, d, rep = 16, 2, 3
    st = oracle_mod.lcg_init(L, d, 1, SEED, rep)
    G = L ** d // 8
    ctr = np.array([[g, 0, rep, 6] for g in range(G)], dtype=np.uint32)
    words = rocrand_philox(ctr, [SEED & 0xFFFFFFFF, SEED >> 32])
    np.testing.assert_array_equal(st, words[:, 0].astype(np.uint64))


@pytest.mark.parametrize("mode,L,d", [(2, 16, 2), (2, 24, 2), (3, 16, 2), (3, 8, 3), (2, 8, 3)])
def test_disjoint_blocks_are_contiguous(oracle_mod, rocrand_philox, mode, L, d):
    G = L ** d // 8
    st = oracle_mod.lcg_init(L, d, mode, SEED, 2)
    w = rocrand_philox(np.array([[0, 0, 2, 7]], dtype=np.uint32), [SEED & 0xFFFFFFFF, SEED >> 32])[0]
    x0 = int(w[0]) | ((int(w[1]) << 32) if mode == 3 else 0)
    assert int(st[0]) == x0
    length = (1 << (64 if mode == 3 else 32)) // G
    for g in range(G - 1):
        assert oracle_mod.lcg_skip(mode, int(st[g]), length) == int(st[g + 1])


@pytest.mark.parametrize("mode,L,d,beta", [(1, 8, 2, 0.44), (2, 8, 2, 0.9), (3, 8, 2, 0.3), (2, 8, 3, 0.25),
                                           (3, 16, 2, 3.0)])
def test_sweep_matches_bruteforce(oracle_mod, mode, L, d, beta):
    ch = oracle_mod.LcgChain(L, d, SEED, mode, replica=1)
    spins = ch.spins.copy()
    state = [int(v) for v in ch.state]

    def draw(s, t, c):
        g = s >> 3
        state[g] = step(mode, state[g])
        return out(mode, state[g])

    for t in range(2):
        bf.sweep(spins, L, d, None, beta, t, draw)
        E, M = ch.sweep(1, beta, every=1)
        np.testing.assert_array_equal(ch.spins, spins)
        assert list(ch.state) == state
        assert (E[0], M[0]) == (bf.energy(spins, L, d), bf.magnetisation(spins))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_invariants(oracle_mod, mode):
    L, d = 16, 2
    ch = oracle_mod.LcgChain(L, d, SEED, mode)
    s0 = ch.spins.copy()
    ch.sweep(1, 0.0)
    np.testing.assert_array_equal(ch.spins, -s0)
    E, _ = ch.sweep(6, math.inf, every=1)
    assert all(E[i + 1] <= E[i] for i in range(len(E) - 1))


def test_bad_arguments(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.lcg_init(12, 2, 1, SEED)         # L % 8 != 0
    with pytest.raises(ValueError):
        oracle_mod.lcg_init(16, 2, 4, SEED)         # unknown mode

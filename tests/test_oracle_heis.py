"""Pins of the oracle's classical Heisenberg mode (continuous spins in single precision).

* Hot start and trial directions follow their Philox words (rocRAND), with
  z = 2u - 1 exact and the other two components on the circle of radius
  sqrt(1 - z^2); every spin stays a unit vector.
* beta = 0 accepts every trial: after one sweep every spin is its trial.
* At zero temperature (beta = inf) the energy never rises.
* One sweep equals a brute-force restatement deciding each site from the
  whole-lattice energy difference in double precision (same draws).
* High temperature: a bond's correlation is the Langevin function
  coth(beta) - 1/beta plus corrections from the smallest loops,
  2 (beta/3)^3 per bond on the square lattice and 4 (beta/3)^3 on the
  cubic lattice at leading order, so u = -(d) <S_i . S_j> per site within
  the statistical error at beta = 0.05.
"""
import math

import numpy as np
import pytest

SEED = 0x1006386500000091


def uniforms(words):
    return (np.asarray(words, dtype=np.uint64) >> 8).astype(np.float64) * 2.0 ** -24


def directions(w0, w1):
    u0, u1 = uniforms(w0), uniforms(w1)
    z = 2 * u0 - 1
    phi = 2 * math.pi * u1
    rho = np.sqrt(1 - z * z)
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def key():
    return [SEED & 0xFFFFFFFF, SEED >> 32]


def test_hot_start_follows_philox(oracle_mod, rocrand_philox):
    L, d, rep = 8, 3, 4
    sp = oracle_mod.heis_init(L, d, SEED, rep)
    N = L ** d
    w = rocrand_philox(np.array([[s, 0, rep, 9] for s in range(N)], dtype=np.uint32), key())
    ref = directions(w[:, 0], w[:, 1])
    np.testing.assert_array_equal(sp[:, 2], ref[:, 2].astype(np.float32))   # z is exact
    np.testing.assert_allclose(sp[:, :3], ref, atol=2e-6)
    assert np.all(sp[:, 3] == 0)
    np.testing.assert_allclose(np.linalg.norm(sp[:, :3].astype(np.float64), axis=1), 1.0, atol=1e-6)


def test_beta_zero_accepts_every_trial(oracle_mod, rocrand_philox):
    L, d, rep, t = 8, 2, 1, 0
    ch = oracle_mod.HeisChain(L, d, SEED, rep)
    ch.sweep(1, 0.0)
    N = L ** d
    col = np.array([((s % L) + (s // L)) & 1 for s in range(N)])
    w = rocrand_philox(np.array([[s, t, rep, 10 + col[s]] for s in range(N)], dtype=np.uint32), key())
    np.testing.assert_allclose(ch.spins[:, :3], directions(w[:, 0], w[:, 1]), atol=2e-6)


def test_zero_temperature_never_raises_energy(oracle_mod):
    ch = oracle_mod.HeisChain(16, 2, SEED)
    E, _ = ch.sweep(8, math.inf, every=1)
    assert all(E[i + 1] <= E[i] + 1e-4 for i in range(len(E) - 1))
    np.testing.assert_allclose(np.linalg.norm(ch.spins[:, :3].astype(np.float64), axis=1), 1.0, atol=1e-6)


def lattice_energy(S, L, d):
    g = S.reshape((L,) * d + (3,)) if d == 2 else S.reshape(L, L, L, 3)
    e = 0.0
    for ax in range(d):
        e -= float((g * np.roll(g, -1, axis=d - 1 - ax)).sum())
    return e


@pytest.mark.parametrize("L,d,beta", [(6, 2, 0.7), (4, 3, 0.4), (8, 2, 2.0)])
def test_sweep_matches_bruteforce(oracle_mod, rocrand_philox, L, d, beta):
    rep = 2
    ch = oracle_mod.HeisChain(L, d, SEED, rep)
    S = ch.spins[:, :3].astype(np.float64).copy()
    N = L ** d
    for t in range(2):
        for c in (0, 1):
            for s in range(N):
                x, y, z = s % L, (s // L) % L, s // (L * L)
                if (x + y + (z if d == 3 else 0)) % 2 != c:
                    continue
                w = rocrand_philox(np.array([[s, t, rep, 10 + c]], dtype=np.uint32), key())[0]
                trial = directions([w[0]], [w[1]])[0]
                e0 = lattice_energy(S, L, d)
                old = S[s].copy()
                S[s] = trial
                dE = lattice_energy(S, L, d) - e0
                u2 = float(uniforms([w[2]])[0])
                p = math.exp(-beta * dE) if beta * dE < 700 else 0.0
                assert abs(u2 - p) > 1e-5, "decision too close to call in double and single precision"
                if not u2 < p:
                    S[s] = old
        ch.sweep(1, beta)
        np.testing.assert_allclose(ch.spins[:, :3], S, atol=2e-5)


@pytest.mark.parametrize("d", [2, 3])
def test_high_temperature_energy(oracle_mod, d):
    beta, L = 0.05, (16 if d == 2 else 8)
    ch = oracle_mod.HeisChain(L, d, SEED + d)
    ch.sweep(50, beta)
    E, _ = ch.sweep(20000, beta, every=1)
    N = L ** d
    e = E / N
    blocks = e.reshape(50, -1).mean(axis=1)
    mean, err = blocks.mean(), blocks.std(ddof=1) / math.sqrt(50)
    langevin = 1 / math.tanh(beta) - 1 / beta
    loops = (2 if d == 2 else 4) * (beta / 3) ** 3
    expect = -d * (langevin + loops)
    assert abs(mean - expect) < 5 * err + 1e-5, (mean, expect, err)

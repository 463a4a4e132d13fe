"""Pins of the oracle's classical Heisenberg mode (continuous spins in single precision).

* Hot start and trial directions follow their Philox words (rocRAND), with
  z = 2u - 1 exact and the other two components on the circle of radius
  sqrt(1 - z^2); every spin stays a unit vector.
* The float direction step equals (rho cos phi, rho sin phi, z) in double
  precision within 3e-7 per component (a few float ulps) over many words.
* The float acceptance step equals u < exp(y) in double precision whenever
  u is 1e-6 (relative) or more away from exp(y), over -87 < y < 0, and
  takes the stated cut-offs at y >= 0 and y <= -87.
* beta = 0 accepts every trial: after one sweep every spin is its trial.
* dE = 0 is accepted at beta = inf (Metropolis, min[1, e^0] = 1): on a
  state whose colour-1 spins cancel around every colour-0 site, each
  colour-0 site takes its trial.
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
    np.testing.assert_allclose(sp[:, :3], ref, atol=3e-7)
    assert np.all(sp[:, 3] == 0)
    np.testing.assert_allclose(np.linalg.norm(sp[:, :3].astype(np.float64), axis=1), 1.0, atol=1e-6)


def test_beta_zero_accepts_every_trial(oracle_mod, rocrand_philox):
    L, d, rep, t = 8, 2, 1, 0
    ch = oracle_mod.HeisChain(L, d, SEED, rep)
    ch.sweep(1, 0.0)
    N = L ** d
    col = np.array([((s % L) + (s // L)) & 1 for s in range(N)])
    w = rocrand_philox(np.array([[s, t, rep, 10 + col[s]] for s in range(N)], dtype=np.uint32), key())
    np.testing.assert_allclose(ch.spins[:, :3], directions(w[:, 0], w[:, 1]), atol=3e-7)


def test_direction_against_double(oracle_mod):
    rng = np.random.default_rng(21)
    words = rng.integers(0, 1 << 32, size=(20000, 2), dtype=np.uint64).tolist()
    # octant and quadrant boundaries of phi, the poles and the equator of z
    edges = [(a << 8, b << 8) for a in (0, 1, 1 << 23, (1 << 24) - 1) for b in
             [k << 21 for k in range(8)] + [(k << 21) - 1 for k in range(1, 9)] + [(k << 21) + 1 for k in range(8)]]
    got = np.array([oracle_mod.heis_direction(a, b) for a, b in words + edges], dtype=np.float64)
    ref = directions([a for a, _ in words + edges], [b for _, b in words + edges])
    np.testing.assert_allclose(got, ref, atol=3e-7, rtol=0)
    np.testing.assert_allclose(np.linalg.norm(got, axis=1), 1.0, atol=4e-7)


def test_accept_against_double_exp(oracle_mod):
    acc = oracle_mod.heis_accept
    for y in np.concatenate([np.linspace(-86.99, -1e-7, 20001),
                             -np.logspace(-7, 0, 200)]).astype(np.float32).tolist():
        e = math.exp(y)
        assert acc(e * (1 - 1e-6), y), y
        assert not acc(e * (1 + 1e-6), y), y
    top = 1 - 2.0 ** -24                      # the largest u
    assert acc(top, 0.0) and acc(top, -0.0) and acc(top, 3.0) and acc(top, math.inf)
    assert not acc(0.0, -87.0) and not acc(0.0, -math.inf) and not acc(0.0, -200.0)
    assert acc(0.0, -86.99)                  # exp(y) > 0 above the cut-off
    assert acc(0.0, -1e-30) and not acc(top, -1e-6)


def cancelling_state(oracle_mod, seed):
    """L = 4 square lattice: colour-1 spins (0, 0, s(x) s(y)) with s = (+, +, -, -), so the four
    neighbours of every colour-0 site add to exactly zero; colour-0 spins from the hot start."""
    L, d = 4, 2
    sp = oracle_mod.heis_init(L, d, seed, 0)
    sgn = [1.0, 1.0, -1.0, -1.0]
    for s in range(L * L):
        x, y = s % L, s // L
        if (x + y) & 1:
            sp[s] = [0.0, 0.0, sgn[x] * sgn[y], 0.0]
    return sp


def test_zero_energy_change_accepted_at_zero_temperature(oracle_mod, rocrand_philox):
    L, d, rep, t = 4, 2, 0, 0
    ch = oracle_mod.HeisChain(L, d, SEED, rep)
    ch.spins = cancelling_state(oracle_mod, SEED)
    ch.sweep(1, math.inf)
    for s in range(L * L):
        x, y = s % L, s // L
        if (x + y) & 1 == 0:
            w = rocrand_philox(np.array([[s, t, rep, 10]], dtype=np.uint32), key())[0]
            np.testing.assert_array_equal(ch.spins[s, :3], oracle_mod.heis_direction(int(w[0]), int(w[1])))


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

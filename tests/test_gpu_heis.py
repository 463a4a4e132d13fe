"""GPU parity of the classical Heisenberg mode (continuous spins, float) against the oracle.

Bar (floating point): every accept decision equal, spin components within
1e-6 (a few ulps: the device's cos, sin and exp may differ from the host
library's by an ulp; every other operation is written to round the same way,
and an accepted spin is a fresh trial, so differences do not accumulate),
E and |M| within 1e-5 per site.  A differing decision would move a spin by
O(1) and fail the component check.
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


@pytest.mark.parametrize("L,d", [(8, 2), (16, 2), (64, 2), (4, 3), (8, 3), (16, 3)])
def test_heis_matches_oracle(oracle_mod, L, d):
    seed = workloads.seed(0x90 + L + d)
    note("heis", L, d)
    h = spin.Heis(L, d, seed, replica=3)
    ch = oracle_mod.HeisChain(L, d, seed, 3)
    np.testing.assert_allclose(h.spins(), ch.spins, atol=1e-6, rtol=0)
    N = L ** d
    for beta in (0.3, 0.7, 0.0, math.inf, 2.0, 1.1):
        E, M = h.sweep_record(2, beta, 1)
        Eo, Mo = ch.sweep(2, beta, every=1)
        np.testing.assert_allclose(h.spins(), ch.spins, atol=1e-6, rtol=0, err_msg="beta %g" % beta)
        np.testing.assert_allclose(E, Eo, atol=1e-5 * N, rtol=0)
        np.testing.assert_allclose(M, Mo, atol=1e-5 * N, rtol=0)
    E, Mv = h.measure()
    Eo, Mvo = ch.measure()
    assert abs(E - Eo) <= 1e-5 * N
    np.testing.assert_allclose(Mv, Mvo, atol=1e-5 * N, rtol=0)
    assert h.t == ch.t == 12
    h.close()


def test_heis_full_size_sampled_sites():
    """2D L = 1024: one sweep verified site by site on a sample, in double precision, from the
    states before and after the sweep (colour-0 sites see the old neighbours, colour-1 sites the
    final colour-0 ones); decisions closer than 1e-5 to the boundary are not judged."""
    from oracle import philox4x32_10
    L, d, seed, rep, beta = 1024, 2, workloads.seed(0x9F), 0, 0.9
    N = L * L
    h = spin.Heis(L, d, seed, rep)
    h.sweep(3, beta)
    t = h.t
    old = h.spins()[:, :3].astype(np.float64)
    h.sweep(1, beta)
    new = h.spins()[:, :3].astype(np.float64)
    h.close()
    rng = np.random.default_rng(3)
    judged = 0
    for s in rng.choice(N, 3000, replace=False).tolist():
        x, y = s % L, s // L
        c = (x + y) & 1
        nb = new if c == 1 else old
        idx = [y * L + (x - 1) % L, y * L + (x + 1) % L, ((y - 1) % L) * L + x, ((y + 1) % L) * L + x]
        hv = nb[idx].sum(axis=0)
        w = philox4x32_10((s, t, rep, 10 + c), (seed & 0xFFFFFFFF, seed >> 32))
        u = [(int(v) >> 8) * 2.0 ** -24 for v in w[:3]]
        z, phi = 2 * u[0] - 1, 2 * math.pi * u[1]
        trial = np.array([math.sqrt(1 - z * z) * math.cos(phi), math.sqrt(1 - z * z) * math.sin(phi), z])
        dE = float(old[s] @ hv - trial @ hv)
        p = math.exp(-beta * dE)
        if abs(u[2] - p) < 1e-5:
            continue
        expect = trial if u[2] < p else old[s]
        np.testing.assert_allclose(new[s], expect, atol=2e-6, err_msg="site %d" % s)
        judged += 1
    assert judged > 2900


def test_heis_rejects_bad_shapes():
    for (L, d) in ((7, 2), (2, 2), (8, 4)):
        with pytest.raises(spin.SpinError):
            spin.Heis(L, d, 1)
    h = spin.Heis(8, 2, 1)
    with pytest.raises(spin.SpinError):
        h.sweep(1, -1.0)
    h.close()

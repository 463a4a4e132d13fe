"""Exact results for the 2D Ising ferromagnet used to pin the oracle.

* ``enumerate_levels(L)``: brute-force enumeration of all 2^(L*L) states of a
  periodic L x L lattice (L <= 4), giving the energy and |M| histogram.
* ``kaufman_u(L, beta)``: internal energy per site of the periodic L x L
  lattice from Kaufman's finite-lattice partition function (the exact
  finite-size results the paper validates against, Sec. 4: Ferdinand and
  Fisher's evaluation of it).
* ``onsager_u(beta)``: the infinite-lattice internal energy.

None of this code touches the oracle; it is an independent statement of
what equilibrium Metropolis sampling must converge to.
"""
import functools
import math

import mpmath
import numpy as np
from scipy.special import ellipk

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


@functools.lru_cache(maxsize=None)
def enumerate_levels(L):
    """Histogram {(E, |M|): count} over all states of the periodic L x L lattice."""
    N = L * L
    assert N <= 16
    states = np.arange(1 << N, dtype=np.int64)
    bits = (states[:, None] >> np.arange(N)[None, :]) & 1
    s = (1 - 2 * bits).reshape(-1, L, L).astype(np.int64)  # s[state, y, x]
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = np.abs(s.sum(axis=(1, 2)))
    hist = {}
    for e, m in zip(E.tolist(), M.tolist()):
        hist[(e, m)] = hist.get((e, m), 0) + 1
    return hist


def enumeration_averages(L, beta):
    """Exact <E>/N, C/N = beta^2 var(E)/N, <|m|>, <m^2> from the enumeration."""
    hist = enumerate_levels(L)
    N = L * L
    mp = mpmath.mp
    mp.dps = 40
    Z = e1 = e2 = am = m2 = mpmath.mpf(0)
    emin = min(e for e, _ in hist)
    for (e, m), c in hist.items():
        w = c * mpmath.exp(-mpmath.mpf(beta) * (e - emin))
        Z += w
        e1 += w * e
        e2 += w * e * e
        am += w * m
        m2 += w * m * m
    e1 /= Z
    e2 /= Z
    return {
        "u": float(e1 / N),
        "c": float(mpmath.mpf(beta) ** 2 * (e2 - e1 * e1) / N),
        "abs_m": float(am / Z / N),
        "m2": float(m2 / Z / N / N),
    }


def _kaufman_lnZ(L, K):
    """ln Z of the periodic L x L Ising model at coupling K (mpmath number)."""
    two_k = 2 * K
    c = mpmath.cosh(two_k) * mpmath.coth(two_k)

    def gamma(l):
        if l == 0:
            return two_k + mpmath.log(mpmath.tanh(K))
        return mpmath.acosh(c - mpmath.cos(mpmath.pi * l / L))

    odd = [gamma(2 * r + 1) for r in range(L)]
    even = [gamma(2 * r) for r in range(L)]
    z1 = mpmath.fprod(2 * mpmath.cosh(L * g / 2) for g in odd)
    z2 = mpmath.fprod(2 * mpmath.sinh(L * g / 2) for g in odd)
    z3 = mpmath.fprod(2 * mpmath.cosh(L * g / 2) for g in even)
    z4 = mpmath.fprod(2 * mpmath.sinh(L * g / 2) for g in even)
    N = L * L
    return mpmath.log(mpmath.mpf(1) / 2) + (mpmath.mpf(N) / 2) * mpmath.log(2 * mpmath.sinh(two_k)) \
        + mpmath.log(z1 + z2 + z3 + z4)


def kaufman_u(L, beta, dps=50):
    """Exact internal energy per site -d lnZ/dK / N of the periodic L x L lattice."""
    with mpmath.workdps(dps):
        K = mpmath.mpf(beta)
        d = mpmath.diff(lambda k: _kaufman_lnZ(L, k), K)
        return float(-d / (L * L))


def kaufman_c(L, beta, dps=50):
    """Exact specific heat per site K^2 d^2 lnZ/dK^2 / N."""
    with mpmath.workdps(dps):
        K = mpmath.mpf(beta)
        d2 = mpmath.diff(lambda k: _kaufman_lnZ(L, k), K, 2)
        return float(K * K * d2 / (L * L))


def onsager_u(beta):
    """Onsager's internal energy per site of the infinite square lattice."""
    t = math.tanh(2 * beta)
    if abs(2 * t * t - 1) < 1e-15:  # beta_c: the elliptic term is 0 * (log divergence) -> 0
        return -1.0 / t
    kappa = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = ellipk(kappa * kappa)
    return -(1.0 / t) * (1 + (2 / math.pi) * (2 * t * t - 1) * K)


def binned_mean_error(x, nbins=50):
    """Mean and standard error from nbins equal blocks (blocks longer than the autocorrelation time)."""
    x = np.asarray(x, dtype=np.float64)
    n = (len(x) // nbins) * nbins
    blocks = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(blocks.mean()), float(blocks.std(ddof=1) / math.sqrt(nbins))

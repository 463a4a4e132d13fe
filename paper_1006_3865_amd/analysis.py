"""Host-side analysis of recorded time series (measurement tooling, not part of the sweep path).

Integrated autocorrelation time with a self-consistent summation window
(Sokal's rule: the smallest window W with W >= c * tau_int(W)), used to turn
attempts/ns into the cost of one statistically independent measurement, as
needed to weigh the multi-hit schedule against its longer autocorrelation
times near the critical point (Sec. 3, multi-hit paragraph).
"""
import numpy as np


def autocorrelation(x):
    """Normalised autocorrelation function rho(t), t = 0 .. n-1, of a 1-D series (FFT, zero padded)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 2:
        raise ValueError("need at least two samples")
    y = x - x.mean()
    var = np.dot(y, y) / n
    if var == 0.0:
        return np.concatenate([[1.0], np.zeros(n - 1)])
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(y, m)
    acf = np.fft.irfft(f * np.conj(f), m)[:n] / (n * var)
    # unbiased lag normalisation: sum over n - t pairs
    return acf * n / (n - np.arange(n))


def tau_int(x, c=6.0):
    """(tau_int, window, error) of a series: tau_int(W) = 1/2 + sum_{t=1}^{W} rho(t), with W the
    first window satisfying W >= c * tau_int(W); error from Sokal's estimate
    tau * sqrt(2 (2W + 1) / n)."""
    rho = autocorrelation(x)
    n = rho.size
    tau = 0.5
    for w in range(1, n):
        tau += rho[w]
        if w >= c * tau:
            return tau, w, tau * np.sqrt(2.0 * (2 * w + 1) / n)
    return tau, n - 1, float("inf")


# ------------------------------------------------ exact finite-lattice 2D Ising (Kaufman)

def _ln_z(L, K, mp):
    """ln Z of the periodic L x L Ising ferromagnet at coupling K (Kaufman's four-term product form)."""
    two_k = 2 * K
    ch = mp.cosh(two_k) / mp.tanh(two_k)
    gam = [two_k + mp.log(mp.tanh(K))] + [mp.acosh(ch - mp.cos(mp.pi * q / L)) for q in range(1, 2 * L)]
    prods = []
    for start in (1, 0):                       # odd, then even indices q = 2r + start
        gs = [gam[q] for q in range(start, 2 * L, 2)]
        prods.append(mp.fprod(2 * mp.cosh(L * g / 2) for g in gs))
        prods.append(mp.fprod(2 * mp.sinh(L * g / 2) for g in gs))
    return mp.log(mp.fsum(prods) / 2) + mp.mpf(L * L) / 2 * mp.log(2 * mp.sinh(two_k))


def exact_u_c(L, beta, dps=40):
    """Internal energy per site u = -(1/N) d lnZ/dK and specific heat per site c = (K^2/N) d^2 lnZ/dK^2
    of the periodic L x L Ising ferromagnet at K = beta (J = 1)."""
    import mpmath
    with mpmath.workdps(dps):
        K = mpmath.mpf(beta)
        f = lambda k: _ln_z(L, k, mpmath)  # noqa: E731
        d1 = mpmath.diff(f, K)
        d2 = mpmath.diff(f, K, 2)
        N = L * L
        return float(-d1 / N), float(K * K * d2 / N)


def energy_stats(E, N, beta, nbins=50):
    """u = <E>/N and c = beta^2 (<E^2> - <E>^2) / N with jackknife errors over nbins equal blocks of the
    series (blocks much longer than the autocorrelation time)."""
    e = np.asarray(E, dtype=np.float64)
    n = (e.size // nbins) * nbins
    blocks = e[:n].reshape(nbins, -1)
    s1, s2 = blocks.sum(axis=1), (blocks * blocks).sum(axis=1)
    m = blocks.shape[1]

    def uc(t1, t2, cnt):
        mean = t1 / cnt
        return mean / N, beta * beta * (t2 / cnt - mean * mean) / N

    u, c = uc(s1.sum(), s2.sum(), n)
    ju, jc = np.empty(nbins), np.empty(nbins)
    for b in range(nbins):
        ju[b], jc[b] = uc(s1.sum() - s1[b], s2.sum() - s2[b], n - m)
    f = (nbins - 1) / nbins
    return u, float(np.sqrt(f * ((ju - ju.mean()) ** 2).sum())), c, float(np.sqrt(f * ((jc - jc.mean()) ** 2).sum()))

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

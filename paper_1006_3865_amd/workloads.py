"""Seeded synthetic inputs of the benchmark configurations.

Shared by the tests, the benchmark and the oracle checks; holds no part of
the Metropolis arithmetic (no RNG of the chain, no table, no update) -- only
sizes, seeds, inverse temperatures and job traces.  The paper measures on
synthetic lattices only (Sec. 4: periodic L x L and L^3 lattices from a
random start), so there is no dataset to stand in for.
"""
import math

import numpy as np

SEED_BASE = 0x1006386500000000


def seed(n):
    return SEED_BASE + n


# Inverse temperatures as exact doubles (hex literals of the decimal values).
BETA_2D_CRIT = float.fromhex("0x1.c34366871d961p-2")   # 0.4406868, just above ln(1+sqrt2)/2
BETA_2D = (float.fromhex("0x1.3333333333333p-2"),       # 0.30
           BETA_2D_CRIT,
           float.fromhex("0x1.3333333333333p-1"))       # 0.60
BETA_3D = float.fromhex("0x1.c5f2bdf81db37p-3")         # 0.2216544

# name -> dict(model, L, d, betas, sweeps, every, seed)
CONFIGS = {
    "ising2d_L64": dict(model=0, L=64, d=2, betas=(BETA_2D_CRIT,), sweeps=1000, every=1, seed=seed(1)),
    "ising2d_L8192": dict(model=0, L=8192, d=2, betas=BETA_2D, sweeps=2000, every=10, seed=seed(2)),
    "ising3d_L512": dict(model=0, L=512, d=3, betas=(BETA_3D,), sweeps=1000, every=10, seed=seed(3)),
}


def ea_betas(n=16, lo=0.5, hi=3.0):
    """Geometric ladder lo*(hi/lo)^(t/(n-1)), t = 0..n-1."""
    return tuple(lo * (hi / lo) ** (t / (n - 1)) for t in range(n))


def ea_batch(realisations=512, sizes=(16, 24, 32, 48, 64), rng_seed=0x12):
    """Batched 3D EA workload: per realisation its L; each runs at the 16 betas.

    Returns a list of dicts (realisation r, L, coupling seed, spin seed,
    replica = 16 r + t, beta) -- 16 * realisations lattices.
    """
    rng = np.random.default_rng(rng_seed)
    Ls = rng.choice(np.asarray(sizes), size=realisations)
    betas = ea_betas()
    out = []
    for r in range(realisations):
        for t, b in enumerate(betas):
            out.append(dict(realisation=r, L=int(Ls[r]), d=3, model=1, coupling_seed=seed(0x11),
                            seed=seed(0x10), replica=16 * r + t, beta=b))
    return out


def serve_trace(jobs=1000, rate_per_s=1.0, rng_seed=0x20):
    """Poisson job stream: model, L (multiple of 8), beta, sweeps, seed, arrival."""
    rng = np.random.default_rng(rng_seed)
    out = []
    t = 0.0
    for j in range(jobs):
        t += rng.exponential(1.0 / rate_per_s)
        kind = int(rng.integers(0, 3))  # 0: 2D Ising, 1: 3D Ising, 2: 3D EA
        if kind == 0:
            L = math.exp(rng.uniform(math.log(32), math.log(4096)))
        else:
            L = math.exp(rng.uniform(math.log(16), math.log(256)))
        L = max(16, int(round(L / 8.0)) * 8)
        sweeps = int(round(math.exp(rng.uniform(math.log(100), math.log(10000)))))
        out.append(dict(job=j, arrival=t, model=1 if kind == 2 else 0, d=2 if kind == 0 else 3, L=L,
                        beta=float(rng.uniform(0.1, 1.0)), sweeps=sweeps, seed=seed(0x1000 + j),
                        coupling_seed=seed(0x2000 + j)))
    return out

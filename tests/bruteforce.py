"""Brute-force restatement of one Metropolis sweep for tiny lattices.

Independent of the oracle: energies are recomputed over the whole lattice
for every proposed flip (so the local-field bookkeeping is never used), the
acceptance probability is min(1, exp(-beta*dE)) of Eq. 2 compared against a
32-bit uniform, and the random words come from a caller-supplied generator
(the tests pass rocRAND's Philox4x32-10).  Only for L^d of a few hundred.
"""
import math

import numpy as np


def grid(spins, L, d):
    return np.asarray(spins, dtype=np.int64).reshape((L,) * d)  # axes (z,) y, x


def energy(spins, L, d, J=None):
    """E = -sum over bonds J s s, Eq. 1; direction 0 is x (last axis)."""
    s = grid(spins, L, d)
    N = L ** d
    e = 0
    for dr in range(d):
        axis = d - 1 - dr
        Jd = np.ones_like(s) if J is None else np.asarray(J[dr * N:(dr + 1) * N], dtype=np.int64).reshape(s.shape)
        e -= int((Jd * s * np.roll(s, -1, axis=axis)).sum())
    return e


def magnetisation(spins):
    return int(np.asarray(spins, dtype=np.int64).sum())


def colour(s, L, d):
    x = s % L
    y = (s // L) % L
    z = s // (L * L) if d == 3 else 0
    return (x + y + z) % 2


def threshold(beta, dE):
    """Exact-rule threshold for a 32-bit uniform: accept iff r < threshold."""
    if dE <= 0:
        return 1 << 32
    return int(math.floor(math.ldexp(math.exp(-(beta * float(dE))), 32)))


def sweep(spins, L, d, J, beta, t, draw, zero_temperature=False):
    """One red/black sweep in place.  draw(s, t, c) -> 32-bit word for site s."""
    N = L ** d
    cur = np.array(spins, dtype=np.int8)
    for c in (0, 1):
        for s in range(N):
            if colour(s, L, d) != c:
                continue
            e0 = energy(cur, L, d, J)
            cur[s] = -cur[s]
            dE = energy(cur, L, d, J) - e0
            cur[s] = -cur[s]
            if zero_temperature:
                accept = dE <= 0
            else:
                accept = draw(s, t, c) < threshold(beta, dE)
            if accept:
                cur[s] = -cur[s]
    spins[:] = cur
    return spins


def coarse_sweep(spins, L, d, J, beta, t, T, k, draw):
    """One sweep of the paper's coarse-tile schedule (Sec. 3, steps 1-7, and k-fold multi-hit), in place:
    tiles of edge T; every tile whose tile coordinates sum to an even number, then every odd one; in each
    tile k times its colour-0 sites, then its colour-1 sites.  draw(s, hit, c) -> 32-bit word, with
    hit = t * k + h for the h-th repetition."""
    B = L // T
    cur = np.array(spins, dtype=np.int8)
    sites_of_tile = {}
    for s in range(L ** d):
        x, y = s % L, (s // L) % L
        z = s // (L * L) if d == 3 else 0
        tile = (x // T, y // T, z // T if d == 3 else 0)
        sites_of_tile.setdefault(tile, []).append(s)
    for q in (0, 1):
        for tile, sites in sorted(sites_of_tile.items()):
            if sum(tile) % 2 != q:
                continue
            for h in range(k):
                for c in (0, 1):
                    for s in sites:
                        if colour(s, L, d) != c:
                            continue
                        e0 = energy(cur, L, d, J)
                        cur[s] = -cur[s]
                        dE = energy(cur, L, d, J) - e0
                        cur[s] = -cur[s]
                        if draw(s, t * k + h, c) < threshold(beta, dE):
                            cur[s] = -cur[s]
    assert B % 2 == 0
    spins[:] = cur
    return spins

"""GPU parity of the batched path: every lattice of a batch against the oracle, bit for bit.

Mixed batches (2D/3D, Ising/+-J, generated and caller couplings, shared
couplings across replicas), per-lattice sweep counts and inverse
temperatures (including 0, inf and 3, which has T = 0 entries), records
after every sweep, and the equality of a lattice swept alone and in a batch.
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


def oracle_chain(oracle_mod, desc):
    J = desc.get("couplings")
    if desc["model"] == 1 and J is None:
        J = oracle_mod.couplings(desc["L"], desc["d"], desc["coupling_seed"], desc.get("realisation", 0))
    return oracle_mod.Chain(desc["L"], desc["d"], desc["seed"], desc.get("replica", 0), J=J)


def check_batch(oracle_mod, descs, schedule, tag):
    """schedule: list of (n per lattice, beta per lattice, every)."""
    note("batch", tag, len(descs), "lattices")
    b = spin.Batch(descs)
    chains = [oracle_chain(oracle_mod, d) for d in descs]
    for i, ch in enumerate(chains):
        np.testing.assert_array_equal(b.spins(i), ch.spins)
    for (n, beta, every) in schedule:
        n = np.broadcast_to(np.asarray(n), (len(descs),))
        beta = np.broadcast_to(np.asarray(beta, dtype=np.float64), (len(descs),))
        recs = b.sweep(n, beta, every)
        for i, ch in enumerate(chains):
            if n[i] > 0:
                Eo, Mo = ch.sweep(int(n[i]), float(beta[i]), every=every)
            elif every:
                e, m = ch.measure()
                Eo, Mo = np.array([e]), np.array([m])
            else:
                Eo = Mo = np.zeros(0, dtype=np.int64)
            if every:
                np.testing.assert_array_equal(recs[i][0], Eo, err_msg="E of lattice %d" % i)
                np.testing.assert_array_equal(recs[i][1], Mo, err_msg="M of lattice %d" % i)
            got = b.spins(i)
            if not np.array_equal(got, ch.spins):
                raise AssertionError("lattice %d (L=%d d=%d model=%d): spins differ at %d sites"
                                     % (i, descs[i]["L"], descs[i]["d"], descs[i]["model"],
                                        int((got != ch.spins).sum())))
            assert b.t(i) == ch.t
    E, M = b.measure()
    for i, ch in enumerate(chains):
        assert (E[i], M[i]) == ch.measure()
    b.close()


def mixed_descs():
    rng = np.random.default_rng(5)
    descs = []
    for L in (8, 16, 24):
        descs.append(dict(model=0, L=L, d=2, seed=workloads.seed(100 + L), replica=L))
    for L in (8, 16):
        descs.append(dict(model=0, L=L, d=3, seed=workloads.seed(200 + L), replica=1))
    for L in (8, 16, 24):
        for rep in (0, 1):  # two replicas share generated couplings
            descs.append(dict(model=1, L=L, d=3, seed=workloads.seed(300 + L), replica=rep,
                              coupling_seed=workloads.seed(0x11), realisation=L))
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=2 * 16 * 16)
    descs.append(dict(model=1, L=16, d=2, seed=workloads.seed(400), replica=3, couplings=J))
    return descs


def test_mixed_batch_matches_oracle(oracle_mod):
    descs = mixed_descs()
    k = len(descs)
    rng = np.random.default_rng(6)
    betas = np.array([0.3, workloads.BETA_2D_CRIT, 0.6, 0.2216544, 0.5, 0.9, 1.5, 3.0, 0.0, math.inf, 0.7,
                      2.0])[:k]
    sched = [
        (rng.integers(1, 6, size=k), betas, 1),
        (rng.integers(0, 4, size=k), betas[::-1].copy(), 1),
        (3, 0.0, 0),
        (4, math.inf, 2),
        (2, 3.0, 1),
    ]
    check_batch(oracle_mod, descs, sched, "mixed")


def test_ea_batch_benchmark_sizes(oracle_mod):
    """The batch workload's lattice sizes, 3D +-J, a few betas of its ladder."""
    ladder = workloads.ea_betas()
    descs, betas = [], []
    for r, L in enumerate((16, 24, 32, 48, 64)):
        for t in (0, 7, 15):
            descs.append(dict(model=1, L=L, d=3, coupling_seed=workloads.seed(0x11), realisation=r,
                              seed=workloads.seed(0x10), replica=16 * r + t))
            betas.append(ladder[t])
    check_batch(oracle_mod, descs, [(2, np.array(betas), 1), (1, np.array(betas), 1)], "ea-sizes")


def test_many_small_lattices(oracle_mod):
    descs = [dict(model=1, L=16, d=3, coupling_seed=workloads.seed(0x11), realisation=r // 4,
                  seed=workloads.seed(0x10), replica=r) for r in range(160)]
    betas = np.array([workloads.ea_betas()[r % 16] for r in range(160)])
    check_batch(oracle_mod, descs, [(6, betas, 3)], "many")


def test_batch_equals_lone_lattices():
    descs = [dict(model=0, L=64, d=2, seed=workloads.seed(1), replica=0),
             dict(model=1, L=24, d=3, coupling_seed=workloads.seed(0x11), realisation=3,
                  seed=workloads.seed(0x10), replica=51)]
    b = spin.Batch(descs)
    b.sweep([50, 20], [workloads.BETA_2D_CRIT, 1.1])
    lone0 = spin.Lattice(0, 64, 2, workloads.seed(1))
    lone0.sweep(50, workloads.BETA_2D_CRIT)
    lone1 = spin.Lattice(1, 24, 3, workloads.seed(0x10), coupling_seed=workloads.seed(0x11), realisation=3,
                         replica=51)
    lone1.sweep(20, 1.1)
    np.testing.assert_array_equal(b.spins(0), lone0.spins())
    np.testing.assert_array_equal(b.spins(1), lone1.spins())
    b.close()
    lone0.close()
    lone1.close()


def test_batch_rejects_bad_shapes():
    with pytest.raises(spin.SpinError):
        spin.Batch([dict(model=0, L=12, d=2, seed=1)])      # L % 8 != 0
    with pytest.raises(spin.SpinError):
        spin.Batch([dict(model=0, L=128, d=3, seed=1)])     # does not fit LDS

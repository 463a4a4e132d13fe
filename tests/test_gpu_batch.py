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


def test_batch_rejects_bad_descs():
    J0 = np.ones(2 * 16 * 16, dtype=np.int8)
    J0[5] = 0
    for bad in (dict(model=0, L=7, d=2, seed=1),                      # odd L
                dict(model=0, L=2, d=2, seed=1),                      # L < 4
                dict(model=0, L=8, d=4, seed=1),                      # d
                dict(model=2, L=8, d=2, seed=1),                      # model
                dict(model=0, L=16, d=2, seed=1, couplings=np.ones(512, dtype=np.int8)),
                dict(model=1, L=16, d=2, seed=1, couplings=J0)):      # a coupling that is not +-1
        with pytest.raises(spin.SpinError):
            spin.Batch([dict(model=0, L=8, d=2, seed=1), bad])
    b = spin.Batch([dict(model=0, L=8, d=2, seed=1)])
    with pytest.raises(spin.SpinError):
        b.remove(1)
    with pytest.raises(spin.SpinError):
        b.add(dict(model=0, L=9, d=2, seed=1))
    assert b.count == 1 and b.members() == [0]
    b.remove(0)
    with pytest.raises(spin.SpinError):
        b.remove(0)
    # a free slot must get n == 0
    lib = spin.load()
    n = np.array([1], dtype=np.int32)
    beta = np.array([0.5])
    rc = lib.spin_batch_sweep(b.h, n.ctypes.data_as(spin._ip), beta.ctypes.data_as(spin._dp), 0, None, None)
    assert rc == spin.SPIN_EINVAL
    b.close()


class Pool:
    """A batch and the oracle chain of every slot it holds."""

    def __init__(self, oracle_mod):
        self.o = oracle_mod
        self.b = spin.Batch([])
        self.chains = {}
        self.descs = {}

    def add(self, desc):
        s = self.b.add(desc)
        assert s not in self.chains
        self.chains[s] = oracle_chain(self.o, desc)
        self.descs[s] = desc
        np.testing.assert_array_equal(self.b.spins(s), self.chains[s].spins)
        return s

    def remove(self, s):
        self.b.remove(s)
        del self.chains[s]
        del self.descs[s]

    def step(self, nsweeps, betas, every):
        S = self.b.count
        n = np.zeros(S, dtype=np.int32)
        beta = np.zeros(S)
        for s in self.chains:
            n[s] = nsweeps[s]
            beta[s] = betas[s]
        note("pool step", dict((s, (int(n[s]), self.descs[s]["L"], self.descs[s]["d"])) for s in self.chains))
        recs = self.b.sweep(n, beta, every)
        for s, ch in self.chains.items():
            if n[s] > 0:
                Eo, Mo = ch.sweep(int(n[s]), float(beta[s]), every=every)
            elif every:
                e, m = ch.measure()
                Eo, Mo = np.array([e]), np.array([m])
            else:
                Eo = Mo = np.zeros(0, dtype=np.int64)
            if every:
                np.testing.assert_array_equal(recs[s][0], Eo, err_msg="E of slot %d" % s)
                np.testing.assert_array_equal(recs[s][1], Mo, err_msg="M of slot %d" % s)
            got = self.b.spins(s)
            if not np.array_equal(got, ch.spins):
                raise AssertionError("slot %d (%s): spins differ at %d sites"
                                     % (s, self.descs[s], int((got != ch.spins).sum())))
            assert self.b.t(s) == ch.t
        for s in range(S):
            if s not in self.chains:
                assert recs[s][0].size == 0
        E, M = self.b.measure()
        for s, ch in self.chains.items():
            assert (E[s], M[s]) == ch.measure()


def test_pool_add_remove_and_large_members(oracle_mod):
    """Members too large for one workgroup (or with L % 8 != 0) go to the single-lattice kernels in the
    same call; removed slots are reused; every member stays on its own chain."""
    p = Pool(oracle_mod)
    cs = workloads.seed(0x11)
    a = p.add(dict(model=0, L=16, d=2, seed=workloads.seed(500), replica=0))
    b_ = p.add(dict(model=1, L=16, d=3, seed=workloads.seed(501), replica=1, coupling_seed=cs, realisation=2))
    c = p.add(dict(model=0, L=12, d=2, seed=workloads.seed(502), replica=2))          # L % 8 != 0
    d = p.add(dict(model=0, L=256, d=2, seed=workloads.seed(503), replica=3))         # LDS-sized, 1024 threads
    e = p.add(dict(model=1, L=72, d=3, seed=workloads.seed(504), replica=4, coupling_seed=cs, realisation=2))  # > LDS
    f = p.add(dict(model=1, L=100, d=2, seed=workloads.seed(505), replica=5, coupling_seed=cs, realisation=7))
    g = p.add(dict(model=0, L=1024, d=2, seed=workloads.seed(506), replica=6))        # beyond one workgroup
    betas = {a: workloads.BETA_2D_CRIT, b_: 0.9, c: 0.3, d: 0.5, e: 1.1, f: 3.0, g: workloads.BETA_2D_CRIT}
    p.step({a: 3, b_: 2, c: 4, d: 1, e: 2, f: 3, g: 2}, betas, 1)
    p.remove(b_)
    p.remove(e)
    h = p.add(dict(model=1, L=24, d=3, seed=workloads.seed(507), replica=7, coupling_seed=cs, realisation=2))
    assert h == e  # most recently freed slot first
    betas[h] = 0.8
    p.step({a: 2, c: 0, d: 2, f: 4, g: 2, h: 4}, betas, 2)
    i = p.add(dict(model=1, L=16, d=3, seed=workloads.seed(508), replica=8, coupling_seed=cs, realisation=2))
    assert i == b_
    betas[i] = math.inf
    p.step({a: 1, c: 2, d: 0, f: 1, g: 1, h: 2, i: 3}, betas, 0)
    p.step({a: 1, c: 1, d: 1, f: 1, g: 1, h: 1, i: 1}, betas, 1)
    assert p.b.footprint(g) == 2 * 1024 * 1024       # spins and the second buffer of the streaming kernels
    assert p.b.footprint(a) == 256
    assert p.b.footprint(p.b.count) == 0
    p.b.close()


def test_pool_member_equals_lone_run(oracle_mod):
    """A lattice's bits do not depend on what else is in the pool or when it was admitted."""
    desc = dict(model=1, L=32, d=3, seed=workloads.seed(600), replica=9, coupling_seed=workloads.seed(0x11),
                realisation=4)
    lone = spin.Batch([desc])
    lone.sweep(7, 0.95)
    want = lone.spins(0)
    lone.close()
    b = spin.Batch([dict(model=0, L=64, d=2, seed=workloads.seed(601), replica=r) for r in range(5)])
    b.sweep(3, 0.4)
    b.remove(2)
    s = b.add(desc)
    n = np.full(b.count, 2, dtype=np.int32)
    n[s] = 4
    b.sweep(n, 0.95)
    n[:] = 1
    n[s] = 3
    b.sweep(n, 0.95)
    np.testing.assert_array_equal(b.spins(s), want)
    b.close()

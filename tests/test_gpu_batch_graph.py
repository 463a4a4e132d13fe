"""A pool call captured into a HIP graph (torch.cuda.CUDAGraph on the pool's
stream) and replayed: every replay must equal one more uncaptured call on a
twin pool, records and spins bit for bit, with the program's own eager work
and synchronisations between the replays.  Capturing a call whose tables are
not on the device yet, or one that would sweep a member too large for LDS,
is refused before anything is enqueued.
"""
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    return t


def descs():
    out = []
    for k, (model, L, d) in enumerate([(0, 32, 2), (0, 128, 2), (1, 64, 2), (0, 24, 3), (1, 16, 3),
                                       (1, 32, 3), (0, 48, 3), (1, 16, 3)]):
        out.append(dict(model=model, L=L, d=d, seed=workloads.seed(0x700 + k), replica=k,
                        coupling_seed=workloads.seed(0x711), realisation=k % 3))
    return out


def test_captured_pool_call_replays_equal_eager_calls(torch):
    s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
    ds = descs()
    A = spin.Batch(ds, stream=s_a)
    B = spin.Batch(ds, stream=s_b)
    n = np.array([7, 5, 6, 4, 9, 3, 5, 8], dtype=np.int32)
    beta = np.array([0.44, 0.3, 1.2, 0.22, 0.9, float("inf"), 0.5, 3.0])
    every = 2
    tot = int(A.record_counts(n, every).sum())
    with torch.cuda.stream(s_a):
        Ea = torch.zeros(tot, dtype=torch.int64, device="cuda")
        Ma = torch.zeros(tot, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(s_b):
        Eb = torch.zeros(tot, dtype=torch.int64, device="cuda")
        Mb = torch.zeros(tot, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    note("graph: first (uncaptured) call on both pools")
    A.sweep_device(n, beta, every, Ea, Ma)
    B.sweep_device(n, beta, every, Eb, Mb)
    torch.cuda.synchronize()
    assert torch.equal(Ea, Eb) and torch.equal(Ma, Mb)
    note("graph: capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s_a):
        A.sweep_device(n, beta, every, Ea, Ma)
    torch.cuda.synchronize()
    for r in range(4):
        note("graph: replay %d" % (r + 1))
        Ea.fill_(-1)
        Ma.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        x = torch.randn(4096, device="cuda").square().sum()   # the program's own eager work
        torch.cuda.synchronize()
        B.sweep_device(n, beta, every, Eb, Mb)
        torch.cuda.synchronize()
        assert float(x) >= 0
        assert torch.equal(Ea, Eb) and torch.equal(Ma, Mb), "records of replay %d differ" % (r + 1)
        for i in range(len(ds)):
            np.testing.assert_array_equal(A.spins(i), B.spins(i), err_msg="lattice %d, replay %d" % (i, r + 1))
            assert A.t(i) == B.t(i) == int(n[i]) * (r + 2)
    # an uncaptured call after the replays continues from the replayed state
    A.sweep_device(n, beta, every, Ea, Ma)
    B.sweep_device(n, beta, every, Eb, Mb)
    torch.cuda.synchronize()
    assert torch.equal(Ea, Eb) and torch.equal(Ma, Mb)
    del g
    A.close()
    B.close()


def test_capture_refused_without_uploaded_tables(torch):
    s = torch.cuda.Stream()
    A = spin.Batch(descs()[:3], stream=s)
    n = np.array([3, 3, 3], dtype=np.int32)
    A.sweep_device(n, 0.5, 0, None, None)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(spin.SpinError) as ei:
        with torch.cuda.graph(g, stream=s):
            A.sweep_device(n + 1, 0.5, 0, None, None)     # other arguments than the previous call
    assert ei.value.code == spin.SPIN_ESTATE
    torch.cuda.synchronize()
    assert [A.t(i) for i in range(3)] == [3, 3, 3]
    A.close()


def test_capture_refused_for_members_beyond_lds(torch):
    s = torch.cuda.Stream()
    ds = descs()[:2] + [dict(model=0, L=1024, d=2, seed=workloads.seed(0x720))]
    A = spin.Batch(ds, stream=s)
    n = np.array([2, 2, 2], dtype=np.int32)
    A.sweep_device(n, 0.5, 0, None, None)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(spin.SpinError) as ei:
        with torch.cuda.graph(g, stream=s):
            A.sweep_device(n, 0.5, 0, None, None)
    assert ei.value.code == spin.SPIN_ESTATE
    torch.cuda.synchronize()
    A.close()

"""GPU parity of the multi-spin-coded +-J glass (32 systems per word) against the oracle.

Every one of the 32 systems' spins, and the 32 energies and magnetisations
after every sweep, equal the oracle's multi-spin-coded mode bit for bit, in
2D and 3D, at several inverse temperatures (including 0, inf and 3).
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


@pytest.mark.parametrize("L,d,kernel", [
    (8, 2, None), (16, 2, None), (64, 2, None), (8, 3, None), (16, 3, None), (24, 3, None),
    (16, 2, (0, 0, 0, 0)), (24, 3, (0, 0, 0, 0)),                 # one launch per colour
    (40, 2, (1, 0, 7, 512)), (24, 3, (1, 4, 5, 256)), (32, 3, (1, 16, 3, 512)), (16, 3, (1, 8, 16, 256)),
    # rows cut into segments of `width` sites (two neighbouring groups of halo each side)
    (40, 2, (1, 0, 7, 512, 8)), (64, 2, (1, 0, 5, 256, 16)), (24, 3, (1, 4, 5, 256, 8)),
    (32, 3, (1, 16, 3, 512, 16)), (48, 3, (1, 8, 16, 512, 16)), (16, 3, (1, 2, 4, 256, 8)),
])
def test_msc_matches_oracle(oracle_mod, L, d, kernel):
    cs, seed, r0, p0 = workloads.seed(0x60), workloads.seed(0x61), 5, 70
    note("msc", L, d, kernel)
    m = spin.Msc(L, d, cs, r0, seed, p0)
    if kernel is not None:
        m.set_kernel(*kernel)
    ch = oracle_mod.MscChain(L, d, cs, r0, seed, p0)
    for b in (0, 13, 31):
        np.testing.assert_array_equal(m.spins(b), ch.spins[b])
    np.testing.assert_array_equal(np.stack(m.measure()), np.stack(ch.measure()))
    for beta in (0.5, 1.1, 0.0, math.inf, 3.0, workloads.BETA_3D):
        E, M = m.sweep_record(2, beta, 1)
        Eo, Mo = ch.sweep(2, beta, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
    for b in range(32):
        np.testing.assert_array_equal(m.spins(b), ch.spins[b], err_msg="system %d" % b)
    assert m.t == ch.t
    m.close()


def test_msc_system_equals_its_own_lattice_inputs():
    """System b starts from the hot start and couplings a lone lattice of replica p0+b, realisation r0+b has."""
    L, d, cs, seed, r0, p0 = 16, 3, workloads.seed(0x62), workloads.seed(0x63), 9, 3
    m = spin.Msc(L, d, cs, r0, seed, p0)
    for b in (0, 31):
        lone = spin.Lattice(1, L, d, seed, coupling_seed=cs, realisation=r0 + b, replica=p0 + b)
        np.testing.assert_array_equal(m.spins(b), lone.spins())
        E, M = m.measure()
        assert (E[b], M[b]) == lone.measure()
        lone.close()
    m.close()


def test_msc_rejects_bad_shapes():
    for (L, d) in ((12, 2), (4, 3), (16, 4)):
        with pytest.raises(spin.SpinError):
            spin.Msc(L, d, 1, 0, 1)
    m = spin.Msc(24, 3, 1, 0, 1)
    # rows must divide L; threads 256/512; width a multiple of 8 dividing L; no negative sizes
    for k in ((1, 5, 8, 256), (1, 8, 8, 128), (1, 8, 8, 256, 12), (1, 8, 8, 256, 16), (1, -8, 8, 256)):
        with pytest.raises(spin.SpinError):
            m.set_kernel(*k)
    m.set_kernel(1, 8, 8, 256, 8)
    m.close()


def boundary_sites(L, rows, planes):
    """Sites on the edges of the kernels' tiles: slab rows (y = 0, rows-1, rows mod rows), strip planes,
    the periodic x wrap and the edges of 8-site groups."""
    ys = sorted({v % L for v in (0, 1, rows - 1, rows, rows + 1, L - 2, L - 1)})
    zs = sorted({v % L for v in (0, 1, planes - 1, planes, planes + 1, L - 2, L - 1)})
    xs = sorted({0, 1, 7, 8, L - 8, L - 1})
    return np.array([(z * L + y) * L + x for z in zs for y in ys for x in xs], dtype=np.int64)


@pytest.mark.parametrize("L,kernel", [(512, None), (512, (1, 8, 128, 512)), (512, (2, 8, 32)), (512, (2, 4, 16)),
                                      (512, (2, 8, 512)), (256, (2, 4, 64)), (256, (2, 8, 256)),
                                      (128, (2, 4, 32))])
def test_msc_full_size_sampled_sites(oracle_mod, L, kernel):
    """The 3D L = 512 handle: the launch shape the benchmark times (the default, register columns), the
    plane-streaming kernel and other register-column shapes; one sweep checked site by site on a sample that includes every tile edge.  A
    colour-0 site is decided from the state before the sweep (its neighbours are colour 1), a colour-1
    site from its old value and the final colour-0 neighbours; each decision is the oracle's rule
    (Eq. 2) with the shared Philox word of the site."""
    d = 3
    N = L ** d
    cs, seed, r0, p0 = workloads.seed(0x11), workloads.seed(0x10), 0, 0
    beta = workloads.ea_betas()[7]
    note("msc full size", L, d, kernel)
    m = spin.Msc(L, d, cs, r0, seed, p0)
    if kernel is not None:
        m.set_kernel(*kernel)
    m.sweep(2, beta)
    systems = (0, 19, 31)
    before = {b: m.spins(b) for b in systems}
    t = m.t
    m.sweep(1, beta)
    after = {b: m.spins(b) for b in systems}
    m.close()
    T = oracle_mod.table(beta, d)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    rng = np.random.default_rng(0x5A)
    rows, planes = (kernel[1], kernel[2]) if kernel else (4, 256)   # the default: register columns
    edge = boundary_sites(L, rows, planes)
    rand = rng.choice(N, 3000, replace=False)
    sites = np.unique(np.concatenate([edge, rand]))
    x, y, z = sites % L, (sites // L) % L, sites // (L * L)
    step = (1, L, L * L)
    coord = (x, y, z)
    draws = {}
    for s in sites.tolist():
        c = ((s % L) + (s // L) % L + s // (L * L)) & 1
        w = oracle_mod.philox4x32_10((s >> 3, t, p0, 4 + c), key)
        draws[s] = (c, int(w[(s >> 1) & 3]))
    for b in systems:
        J = oracle_mod.couplings(L, d, cs, r0 + b)
        old, new = before[b], after[b]
        for i, s in enumerate(sites.tolist()):
            c, r = draws[s]
            nbr = new if c == 1 else old   # colour-1 sites see final colour-0 neighbours
            h = 0
            for dr in range(d):
                v = int(coord[dr][i])
                sp = s + step[dr] if v + 1 < L else s - (L - 1) * step[dr]
                sm = s - step[dr] if v > 0 else s + (L - 1) * step[dr]
                h += int(J[dr * N + s]) * int(nbr[sp]) + int(J[dr * N + sm]) * int(nbr[sm])
            k = int(old[s]) * h
            flip = r < int(T[(k + 2 * d) // 2])
            expect = -int(old[s]) if flip else int(old[s])
            assert int(new[s]) == expect, ("system", b, "site", s, "colour", c)


@pytest.mark.parametrize("L,shape", [(512, (8, 32)), (512, (4, 64)), (512, (8, 2)), (256, (4, 64)), (256, (8, 16)),
                                     (128, (4, 32)), (128, (8, 128))])
def test_msc_column_kernel_equals_streaming_kernel(L, shape):
    """The register-column kernel (3D L = 512, 256, 128; below 512 a wavefront holds several copies of
    a row) against the plane-streaming kernel, whose chain is the oracle's at every size it was
    compared on: all 32 systems' spins (as the words of every site) and the 32 energies and
    magnetisations after every sweep, over sweeps at several temperatures."""
    import torch
    d = 3
    cs, seed, r0, p0 = workloads.seed(0x64), workloads.seed(0x65), 3, 11
    note("msc column vs stream", shape)
    a = spin.Msc(L, d, cs, r0, seed, p0)
    b = spin.Msc(L, d, cs, r0, seed, p0)
    a.set_kernel(2, shape[0], shape[1])
    b.set_kernel(1, 8, 16, 512 if L >= 256 else 256)
    for beta in (workloads.ea_betas()[3], math.inf, 0.0, 3.0):
        Ea, Ma = a.sweep_record(2, beta, 1)
        Eb, Mb = b.sweep_record(2, beta, 1)
        np.testing.assert_array_equal(Ea, Eb)
        np.testing.assert_array_equal(Ma, Mb)
    for sysb in (0, 7, 31):
        np.testing.assert_array_equal(a.spins(sysb), b.spins(sysb), err_msg="system %d" % sysb)
    assert a.t == b.t == 8
    a.close()
    b.close()


def test_msc_column_kernel_shapes():
    m = spin.Msc(512, 3, 1, 0, 1)
    for k in ((2, 6, 32), (2, 8, 3), (2, 8, 0, 512), (2, 8, 32, 0, 256), (3, 8, 32)):
        with pytest.raises(spin.SpinError):
            m.set_kernel(*k)
    m.set_kernel(2, 8, 32, 640)
    m.set_kernel(2, 4, 2)
    m.close()
    s = spin.Msc(64, 3, 1, 0, 1)     # the register-column kernel takes L = 128, 256 and 512
    with pytest.raises(spin.SpinError):
        s.set_kernel(2, 8, 32)
    s.close()

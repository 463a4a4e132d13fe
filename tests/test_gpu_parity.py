"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Spins, E and M are integers, so the bar is exact equality everywhere.  Every
kernel family and tile shape is run on the same seeded inputs; sizes span
several tiles and ragged (L % 8 != 0) lattices, the degenerate inverse
temperatures (beta = 0 flips every spin, beta = inf is a quench, beta = 3
has T = 0 entries) and the full benchmark sizes (sampled by sweeps).
"""
import math
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import spin, workloads

pytestmark = pytest.mark.gpu

B_CRIT = workloads.BETA_2D_CRIT
B_3D = workloads.BETA_3D
GEN, RES, TIL, FUS = (spin.SPIN_KERNEL_GENERIC, spin.SPIN_KERNEL_RESIDENT, spin.SPIN_KERNEL_TILED,
                      spin.SPIN_KERNEL_FUSED)
STR = spin.SPIN_KERNEL_STREAM


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


def make(model, L, d, seed, replica=0, J=None, cseed=None, kernel=spin.SPIN_KERNEL_AUTO, tile=(0, 0, 0, 0)):
    lat = spin.Lattice(model, L, d, seed, couplings=J, coupling_seed=cseed, replica=replica)
    if kernel != spin.SPIN_KERNEL_AUTO:
        lat.set_kernel(kernel, *tile)
    return lat


def compare_runs(oracle_mod, model, L, d, seed, schedule, replica=0, J=None, cseed=None, kernel=0,
                 tile=(0, 0, 0, 0), tag=""):
    """schedule: list of (n, beta, every); compares records and spins after every call."""
    note("parity", tag, "model", model, "L", L, "d", d, "kernel", kernel, "tile", tile)
    lat = make(model, L, d, seed, replica, J, cseed, kernel, tile)
    Jo = J
    if model == 1 and J is None:
        Jo = oracle_mod.couplings(L, d, cseed, 0)
        np.testing.assert_array_equal(lat.couplings(), Jo)
    ch = oracle_mod.Chain(L, d, seed, replica, J=Jo)
    np.testing.assert_array_equal(lat.spins(), ch.spins)
    for (n, beta, every) in schedule:
        if every:
            Eg, Mg = lat.sweep_record(n, beta, every)
            Eo, Mo = ch.sweep(n, beta, every=every)
            np.testing.assert_array_equal(Eg, Eo)
            np.testing.assert_array_equal(Mg, Mo)
        else:
            lat.sweep(n, beta)
            ch.sweep(n, beta)
        got = lat.spins()
        if not np.array_equal(got, ch.spins):
            bad = np.flatnonzero(got != ch.spins)
            raise AssertionError("spins differ at %d sites, first %s (t=%d)" % (bad.size, bad[:8], ch.t))
        assert lat.t == ch.t
        assert lat.measure() == ch.measure()
    lat.close()


# ----------------------------------------------------------- hot start etc.

@pytest.mark.parametrize("L,d,replica", [(4, 2, 0), (6, 2, 3), (64, 2, 0), (8192, 2, 0), (10, 3, 1), (64, 3, 7)])
def test_hot_start_matches_oracle(oracle_mod, L, d, replica):
    s = workloads.seed(2)
    lat = make(0, L, d, s, replica)
    np.testing.assert_array_equal(lat.spins(), oracle_mod.init_spins(L, d, s, replica))
    E, M = lat.measure()
    assert (E, M) == oracle_mod.measure(L, d, None, oracle_mod.init_spins(L, d, s, replica))
    lat.close()


@pytest.mark.parametrize("L,d,real", [(6, 2, 0), (16, 3, 4), (64, 3, 511)])
def test_generated_couplings_match_oracle(oracle_mod, L, d, real):
    lat = spin.Lattice(1, L, d, 5, coupling_seed=workloads.seed(0x11), realisation=real)
    np.testing.assert_array_equal(lat.couplings(), oracle_mod.couplings(L, d, workloads.seed(0x11), real))
    lat.close()


# ------------------------------------------------- small-lattice configs

def test_ising2d_L64_full_record(oracle_mod):
    """2D Ising L=64 at 0.4406868, 1000 sweeps, E/M every sweep, spins at 1,2,10,100,1000."""
    cfg = workloads.CONFIGS["ising2d_L64"]
    sched = [(1, B_CRIT, 1), (1, B_CRIT, 1), (8, B_CRIT, 1), (90, B_CRIT, 1), (900, B_CRIT, 1)]
    compare_runs(oracle_mod, 0, 64, 2, cfg["seed"], sched, tag="ising2d_L64")


def test_L4_parity(oracle_mod):
    compare_runs(oracle_mod, 0, 4, 2, workloads.seed(4), [(1000, B_CRIT, 1)], tag="L4")


# ---------------------------------------------- every family, every tile

BETAS = [0.30, B_CRIT, 0.60, 0.0, math.inf, 3.0]

CASES_2D = [
    (GEN, (0, 0, 0, 0), 32), (GEN, (0, 0, 0, 0), 34),
    (RES, (0, 0, 0, 64), 32), (RES, (0, 0, 0, 1024), 64), (RES, (0, 0, 0, 256), 18),
    (RES, (0, 0, 0, 0), 8), (RES, (0, 0, 0, 256), 512), (RES, (0, 0, 0, 0), 552),
    (TIL, (16, 8, 0, 64), 32), (TIL, (64, 8, 0, 64), 128), (TIL, (128, 16, 0, 256), 256),
    (TIL, (256, 32, 0, 256), 512), (TIL, (512, 32, 0, 512), 1024),
    (FUS, (16, 8, 0, 64), 32), (FUS, (16, 8, 0, 64), 48), (FUS, (128, 16, 0, 256), 256),
    (FUS, (256, 32, 0, 256), 512), (FUS, (512, 32, 0, 512), 1024), (FUS, (256, 32, 0, 256), 256),
    (FUS, (512, 16, 0, 256), 512), (FUS, (512, 32, 0, 256), 1024), (FUS, (512, 64, 0, 256), 1024),
    (FUS, (512, 64, 0, 256), 2048),
    (STR, (0, 1, 8, 256), 16), (STR, (0, 1, 5, 512), 40), (STR, (0, 1, 3, 256), 72),
    (STR, (0, 1, 16, 256), 1024), (STR, (0, 1, 7, 512), 2056),
]


@pytest.mark.parametrize("kernel,tile,L", CASES_2D)
def test_ising2d_all_kernels(oracle_mod, kernel, tile, L):
    sched = [(3, b, 1) for b in BETAS] + [(4, B_CRIT, 2)]
    compare_runs(oracle_mod, 0, L, 2, workloads.seed(20 + L), sched, replica=2, kernel=kernel, tile=tile,
                 tag="2d")


CASES_3D = [
    (GEN, (0, 0, 0, 0), 16), (GEN, (0, 0, 0, 0), 10),
    (RES, (0, 0, 0, 256), 16), (RES, (0, 0, 0, 512), 32), (RES, (0, 0, 0, 128), 6),
    (RES, (0, 0, 0, 0), 8), (RES, (0, 0, 0, 1024), 64),
    (STR, (0, 8, 16, 256), 16), (STR, (0, 4, 5, 256), 24), (STR, (0, 16, 16, 512), 64),
    (STR, (0, 8, 7, 256), 72), (STR, (0, 32, 16, 256), 128), (STR, (0, 16, 3, 512), 48),
    (TIL, (16, 4, 4, 64), 16), (TIL, (16, 4, 4, 64), 32), (TIL, (32, 8, 4, 128), 64),
    (TIL, (64, 8, 8, 256), 64), (TIL, (128, 8, 4, 256), 128),
    # register-column plane streaming below L = 512 (the wavefront holds copies of its rows)
    (FUS, (256, 16, 16, 576), 256), (FUS, (256, 8, 32, 320), 256), (FUS, (128, 16, 8, 576), 128),
    (FUS, (128, 8, 128, 320), 128),
]


@pytest.mark.parametrize("kernel,tile,L", CASES_3D)
def test_ising3d_all_kernels(oracle_mod, kernel, tile, L):
    sched = [(2, b, 1) for b in [B_3D, 0.5, 0.0, math.inf, 3.0]]
    compare_runs(oracle_mod, 0, L, 3, workloads.seed(30 + L), sched, replica=1, kernel=kernel, tile=tile,
                 tag="3d")


@pytest.mark.parametrize("kernel,tile,L,d", [
    (GEN, (0, 0, 0, 0), 16, 2), (GEN, (0, 0, 0, 0), 10, 3), (GEN, (0, 0, 0, 0), 24, 3),
    (RES, (0, 0, 0, 256), 14, 2), (RES, (0, 0, 0, 512), 16, 3), (RES, (0, 0, 0, 1024), 24, 3),
    (RES, (0, 0, 0, 0), 64, 3), (RES, (0, 0, 0, 512), 40, 2),
    (STR, (0, 1, 8, 256), 64, 2), (STR, (0, 1, 6, 512), 1000, 2), (STR, (0, 8, 16, 256), 48, 3),
    (STR, (0, 16, 16, 512), 96, 3), (STR, (0, 8, 5, 256), 16, 3), (STR, (0, 0, 0, 0), 136, 3),
    # the streaming kernel's word-pair form (rows of an even number of words, pairs >= threads)
    (STR, (0, 32, 8, 256), 128, 3), (STR, (0, 1, 8, 256), 4096, 2),
])
def test_ea_all_kernels(oracle_mod, kernel, tile, L, d):
    sched = [(3, b, 1) for b in [0.5, 1.2, 0.0, math.inf, 3.0]]
    compare_runs(oracle_mod, 1, L, d, workloads.seed(40 + L), sched, replica=5, cseed=workloads.seed(0x11),
                 kernel=kernel, tile=tile, tag="ea")


def test_ea_host_couplings(oracle_mod):
    rng = np.random.default_rng(9)
    L, d = 12, 3
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d)
    compare_runs(oracle_mod, 1, L, d, 77, [(5, 0.8, 1)], J=J, tag="ea-host")
    L = 40
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d)
    compare_runs(oracle_mod, 1, L, d, 78, [(4, 0.8, 2), (3, 1.9, 1)], J=J, kernel=STR, tile=(0, 8, 8, 256),
                 tag="ea-host-stream")


@pytest.mark.parametrize("model,L,d", [(1, 128, 3), (1, 72, 3), (0, 72, 3), (1, 1024, 2)])
def test_auto_picks_stream(oracle_mod, model, L, d):
    """Shapes no specialised kernel covers (any +-J lattice beyond LDS size, 3D L not a multiple of 16)."""
    lat = make(model, L, d, workloads.seed(60 + L), 3, None, workloads.seed(0x11) if model else None, 0,
               (0, 0, 0, 0))
    assert lat.kernel == STR, spin.KERNEL_NAMES[lat.kernel]
    lat.close()
    compare_runs(oracle_mod, model, L, d, workloads.seed(60 + L), [(2, 0.7, 1)], replica=3,
                 cseed=workloads.seed(0x11) if model else None, tag="auto-stream")


def test_auto_3d_L256_register_columns(oracle_mod):
    """3D Ising L = 256 runs the register-column plane streaming by default (16-row slabs, strips of
    8 planes; the wavefront holds two copies of each row), with and without records."""
    seed = workloads.seed(0x256)
    lat = make(0, 256, 3, seed, 1)
    assert lat.kernel == FUS and lat.tile == (256, 16, 8, 576), (spin.KERNEL_NAMES[lat.kernel], lat.tile)
    lat.close()
    compare_runs(oracle_mod, 0, 256, 3, seed, [(1, B_3D, 1), (2, 0.3, 0), (1, 0.9, 1)], replica=1,
                 tag="auto-3d-L256")


@pytest.mark.parametrize("model,L", [(0, 160), (1, 200), (0, 320), (1, 384)])
def test_auto_3d_stream_defaults(oracle_mod, model, L):
    """Large 3D lattices stream with the size-dependent default tiles (slab rows, strip planes and
    threads chosen by L); the bits are the oracle's."""
    lat = make(model, L, 3, workloads.seed(80 + L), 1, None, workloads.seed(0x11) if model else None)
    assert lat.kernel == STR, spin.KERNEL_NAMES[lat.kernel]
    lat.close()
    compare_runs(oracle_mod, model, L, 3, workloads.seed(80 + L), [(1, 0.3, 1), (1, 0.9, 1)], replica=1,
                 cseed=workloads.seed(0x11) if model else None, tag="auto-3d-stream")


def test_auto_choice_and_switching(oracle_mod):
    """Switch families between calls of one chain; bits must not change."""
    L, s = 64, workloads.seed(50)
    lat = make(0, L, 2, s)
    ch = oracle_mod.Chain(L, 2, s)
    for kern, tile in [(FUS, (16, 8, 0, 64)), (TIL, (16, 8, 0, 64)), (GEN, (0, 0, 0, 0)), (RES, (0, 0, 0, 256)),
                       (FUS, (16, 8, 0, 64)), (spin.SPIN_KERNEL_AUTO, (0, 0, 0, 0))]:
        lat.set_kernel(kern, *tile)
        E, M = lat.sweep_record(3, B_CRIT, 1)
        Eo, Mo = ch.sweep(3, B_CRIT, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
        np.testing.assert_array_equal(lat.spins(), ch.spins)
    lat.close()


def test_resume_from_saved_state(oracle_mod):
    L, s = 256, workloads.seed(51)
    a = make(0, L, 2, s)
    a.sweep(7, 0.5)
    saved, t = a.spins(), a.t
    a.sweep(5, 0.5)
    b = make(0, L, 2, s)
    b.set_spins(saved)
    b.t = t
    b.sweep(5, 0.5)
    np.testing.assert_array_equal(a.spins(), b.spins())
    a.close()
    b.close()


def test_set_replica_continues_as_that_replica(oracle_mod):
    """spin_set_replica: after it the chain is the given replica's from the present state (equal to
    a handle created with that replica and resumed from the same spins and sweep index, and unlike
    the old replica's continuation); refused in an LCG draw mode."""
    L, s = 256, workloads.seed(52)
    a = make(0, L, 2, s)
    a.sweep(7, 0.5)
    saved, t = a.spins(), a.t
    a.set_replica(3)
    a.sweep(5, 0.5)
    b = make(0, L, 2, s, replica=3)
    b.set_spins(saved)
    b.t = t
    b.sweep(5, 0.5)
    c = make(0, L, 2, s)
    c.set_spins(saved)
    c.t = t
    c.sweep(5, 0.5)
    np.testing.assert_array_equal(a.spins(), b.spins())
    assert not np.array_equal(a.spins(), c.spins())
    d = make(0, 64, 2, s)
    d.set_rng(spin.SPIN_RNG_LCG32_ARRAY)
    with pytest.raises(spin.SpinError) as ei:
        d.set_replica(1)
    assert ei.value.code == spin.SPIN_ESTATE
    for h in (a, b, c, d):
        h.close()


def test_device_records_and_torch_stream(oracle_mod, gpu):
    torch = gpu
    L, s = 512, workloads.seed(52)
    stream = torch.cuda.Stream()
    E = torch.full((10,), -7, dtype=torch.int64, device="cuda")
    M = torch.full((10,), -7, dtype=torch.int64, device="cuda")
    stream.wait_stream(torch.cuda.current_stream())
    lat = spin.Lattice(0, L, 2, s, stream=stream)
    lat.sweep_record_device(20, B_CRIT, 2, E, M)
    lat.synchronize()
    ch = oracle_mod.Chain(L, 2, s)
    Eo, Mo = ch.sweep(20, B_CRIT, every=2)
    np.testing.assert_array_equal(E.cpu().numpy(), Eo)
    np.testing.assert_array_equal(M.cpu().numpy(), Mo)
    lat.close()


def test_torch_allocator(oracle_mod, gpu):
    spin.use_torch_allocator()
    try:
        compare_runs(oracle_mod, 0, 128, 2, 3, [(4, 0.4, 1)], kernel=FUS, tile=(16, 8, 0, 64), tag="torch-alloc")
    finally:
        spin.use_hip_allocator()


@pytest.mark.parametrize("tile,L", [
    ((4096, 16, 0, 512), 4096), ((4096, 8, 0, 512), 4096), ((4096, 64, 0, 512), 4096), ((4096, 8, 0, 256), 4096),
    ((8192, 32, 0, 1024), 8192), ((8192, 16, 0, 512), 8192),
])
def test_ising2d_streaming_rows(oracle_mod, tile, L):
    """Row-streaming fused kernel: several strips, wrap rows, beta with T == 0 entries."""
    sched = [(2, B_CRIT, 1), (1, 3.0, 1), (4, 0.6, 2), (1, 0.0, 0)]
    compare_runs(oracle_mod, 0, L, 2, workloads.seed(60 + L), sched, replica=4, kernel=FUS, tile=tile,
                 tag="stream")


@pytest.mark.parametrize("tile,L", [
    ((4096, 16, 1, 512), 4096), ((4096, 8, 1, 256), 4096), ((4096, 64, 1, 512), 4096),
    ((8192, 16, 1, 1024), 8192), ((8192, 32, 1, 512), 8192), ((8192, 4, 1, 1024), 8192),
])
def test_ising2d_register_columns(oracle_mod, tile, L):
    """Register-column form of the row-streaming kernel (tile_z = 1), with and without E/M counted
    inside the sweep (records every 2 and 5 sweeps, one of them at a beta with T == 0 entries).
    Several strips, one and two 8-site groups per thread, the periodic x wrap between the first
    and last segment, and betas with T == 0 entries (3, inf) and 0."""
    sched = [(3, B_CRIT, 0), (2, 3.0, 2), (5, 0.6, 5), (1, 0.0, 0), (2, math.inf, 0), (4, 0.3, 0)]
    compare_runs(oracle_mod, 0, L, 2, workloads.seed(0x90 + L), sched, replica=2, kernel=FUS, tile=tile,
                 tag="columns")


@pytest.mark.parametrize("model,L,d", [(0, 96, 3), (1, 96, 3), (0, 4112, 2), (1, 48, 3)])
def test_measure_ragged_row_ranges(oracle_mod, model, L, d):
    """E/M counting when the rows do not divide evenly among the counting workgroups (3D L = 96:
    5 rows per workgroup and 1 in the last; 2D L = 4112: 257 chunks per row, more than the 256
    threads, 3 rows per workgroup and 2 in the last), Ising and +-J."""
    sched = [(2, 0.3, 1), (1, 0.7, 0), (2, 1.2, 2)]
    compare_runs(oracle_mod, model, L, d, workloads.seed(0x70 + L + model), sched, replica=1,
                 cseed=workloads.seed(0x71) if model else None, tag="measure-ragged")


# ------------------------------------------------------ full-size configs

@pytest.mark.parametrize("beta", workloads.BETA_2D)
def test_ising2d_L8192_first_sweeps(oracle_mod, beta):
    """Full benchmark size, the kernel the benchmark times: two sweeps, records each sweep."""
    cfg = workloads.CONFIGS["ising2d_L8192"]
    lat = make(0, 8192, 2, cfg["seed"])
    note("L8192 beta", beta, "kernel", spin.KERNEL_NAMES[lat.kernel])
    assert lat.kernel == FUS
    E, M = lat.sweep_record(2, beta, 1)
    ch = oracle_mod.Chain(8192, 2, cfg["seed"])
    Eo, Mo = ch.sweep(2, beta, every=1)
    np.testing.assert_array_equal(E, Eo)
    np.testing.assert_array_equal(M, Mo)
    np.testing.assert_array_equal(lat.spins(), ch.spins)
    lat.close()


def test_ising3d_L512_first_sweep(oracle_mod):
    """Full benchmark size, the kernel the benchmark times (plane streaming), then the other
    plane-streaming shapes continuing the same chain."""
    cfg = workloads.CONFIGS["ising3d_L512"]
    lat = make(0, 512, 3, cfg["seed"])
    note("L512 3d kernel", spin.KERNEL_NAMES[lat.kernel])
    assert lat.kernel == FUS
    ch = oracle_mod.Chain(512, 3, cfg["seed"])
    for tile, beta in [(None, B_3D), ((512, 8, 32, 640), 3.0), ((512, 32, 64, 704), 0.0),
                       ((512, 16, 16, 384), 0.5), ((512, 8, 64, 320), B_3D)]:
        if tile:
            lat.set_kernel(FUS, *tile)
        E, M = lat.sweep_record(1, beta, 1)
        Eo, Mo = ch.sweep(1, beta, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
        np.testing.assert_array_equal(lat.spins(), ch.spins)
    lat.close()


def test_ising3d_L512_register_column_shapes(oracle_mod):
    """The register-column plane-streaming kernel (the 3D L = 512 default) at every slab height and at
    strip heights from 2 planes to the whole lattice (one strip: the z wrap inside one workgroup's
    pipeline), continuing one chain across shapes and temperatures: a typical beta, beta = 3 (classes
    with T = 0), beta = 0 (every spin flips) and a zero-temperature quench; E/M counted in the sweep."""
    s = workloads.seed(0xB3)
    lat = make(0, 512, 3, s, 5)
    ch = oracle_mod.Chain(512, 3, s, 5)
    for tile, beta in [((512, 16, 32, 576), B_3D), ((512, 16, 2, 576), 3.0), ((512, 8, 4, 320), 0.0),
                       ((512, 16, 512, 576), math.inf), ((512, 8, 64, 320), 0.5), ((512, 16, 8, 576), B_3D)]:
        lat.set_kernel(FUS, *tile)
        note("register-column", tile, beta)
        E, M = lat.sweep_record(1, beta, 1)
        Eo, Mo = ch.sweep(1, beta, every=1)
        np.testing.assert_array_equal(E, Eo)
        np.testing.assert_array_equal(M, Mo)
        np.testing.assert_array_equal(lat.spins(), ch.spins)
    lat.close()


@pytest.mark.parametrize("model,L,d", [(0, 256, 3), (1, 96, 3), (0, 2048, 2), (1, 48, 3)])
def test_autotune_keeps_chain_and_parity(oracle_mod, model, L, d):
    """spin_autotune leaves the handle's chain untouched, and the family it picks (also taken by new
    AUTO handles of the shape) gives the oracle's bits."""
    s = workloads.seed(70 + L)
    cs = workloads.seed(0x11) if model else None
    lat = make(model, L, d, s, 2, None, cs)
    lat.sweep(2, 0.6)
    before, t = lat.spins(), lat.t
    k = lat.autotune(0.6, 2)
    note("autotune", model, L, d, "->", spin.KERNEL_NAMES[k])
    assert k == lat.kernel and k in spin.KERNEL_NAMES and k != spin.SPIN_KERNEL_AUTO
    np.testing.assert_array_equal(lat.spins(), before)
    assert lat.t == t
    other = make(model, L, d, s, 2, None, cs)
    assert other.kernel == k
    other.close()
    Jo = oracle_mod.couplings(L, d, cs, 0) if model else None
    ch = oracle_mod.Chain(L, d, s, 2, J=Jo)
    ch.sweep(2, 0.6)
    E, M = lat.sweep_record(3, 0.6, 1)
    Eo, Mo = ch.sweep(3, 0.6, every=1)
    np.testing.assert_array_equal(E, Eo)
    np.testing.assert_array_equal(M, Mo)
    np.testing.assert_array_equal(lat.spins(), ch.spins)
    lat.close()


def check_sweep_sampled(oracle_mod, old, new, L, d, J, seed, replica, t, beta, n_sites, rng_seed):
    """One canonical sweep verified site by site on a sample: a colour-0 site is decided from the state
    before the sweep (its neighbours are colour 1), a colour-1 site from its old value and the final
    colour-0 neighbours; each decision is Eq. 2 with the site's own Philox word."""
    T = oracle_mod.table(beta, d)
    N = L ** d
    key = (seed & 0xFFFFFFFF, seed >> 32)
    step = (1, L, L * L)
    rng = np.random.default_rng(rng_seed)
    for s in rng.choice(N, n_sites, replace=False).tolist():
        x = [s % L, (s // L) % L, s // (L * L)][:d]
        c = sum(x) & 1
        nb = new if c == 1 else old
        h = 0
        for dr in range(d):
            sp = s + step[dr] if x[dr] + 1 < L else s - (L - 1) * step[dr]
            sm = s - step[dr] if x[dr] > 0 else s + (L - 1) * step[dr]
            jp = int(J[dr * N + s]) if J is not None else 1
            jm = int(J[dr * N + sm]) if J is not None else 1
            h += jp * int(nb[sp]) + jm * int(nb[sm])
        k = int(old[s]) * h
        r = int(oracle_mod.philox4x32_10((s >> 3, t, replica, c), key)[(s >> 1) & 3])
        flip = r < int(T[(k + 2 * d) // 2])
        assert int(new[s]) == (-int(old[s]) if flip else int(old[s])), ("site", s, "colour", c)


@pytest.mark.parametrize("L,d,beta,tile,every", [
    (16384, 2, B_CRIT, (16384, 16, 0, 1024), 1),   # row-streaming kernel, two 8-site groups per thread
    (16384, 2, B_CRIT, (16384, 16, 1, 1024), 0),   # its register-column form (no record)
    (16384, 2, B_CRIT, (512, 16, 0, 256), 1),      # tiled fused kernel
    (1024, 3, B_3D, None, 1)])
def test_largest_sizes_whole_lattice(oracle_mod, L, d, beta, tile, every):
    """The largest lattices the specialised kernels take, every site: from the same hot start as the
    oracle's chain, one sweep (with its record when every = 1); spins at every site and (E, M)."""
    kern, t = (spin.SPIN_KERNEL_FUSED, tile) if tile else (spin.SPIN_KERNEL_AUTO, (0, 0, 0, 0))
    compare_runs(oracle_mod, 0, L, d, workloads.seed(0xA0 + d), [(1, beta, every)], replica=1, kernel=kern,
                 tile=t, tag="largest, whole lattice")


@pytest.mark.parametrize("model,L,d,beta,tile", [
    (0, 16384, 2, B_CRIT, (16384, 16, 0, 1024)),   # row-streaming kernel, two 8-site groups per thread
    (0, 16384, 2, B_CRIT, (512, 16, 0, 256)),      # tiled fused kernel on the same lattice
    (0, 1024, 3, B_3D, None),
    (1, 512, 3, 1.0, None)])
def test_largest_sizes_sampled(oracle_mod, model, L, d, beta, tile):
    """The largest lattices the specialised kernels take (2D L = 16384 on the row-streaming kernel,
    whose buffer descriptor spans 2^28 bytes, and on the tiled fused kernel; 3D L = 1024) and a 3D
    +-J lattice of the benchmark's size: the second sweep checked site by site on a sample."""
    seed, rep = workloads.seed(0xA0 + d), 1
    cs = workloads.seed(0x11) if model else None
    lat = make(model, L, d, seed, rep, None, cs)
    if tile is not None:
        lat.set_kernel(spin.SPIN_KERNEL_FUSED, *tile)
        assert lat.kernel == spin.SPIN_KERNEL_FUSED
    note("largest", model, L, d, "kernel", spin.KERNEL_NAMES[lat.kernel], "tile", tile)
    lat.sweep(1, beta)
    old = lat.spins()
    t = lat.t
    lat.sweep(1, beta)
    new = lat.spins()
    lat.close()
    J = oracle_mod.couplings(L, d, cs, 0) if model else None
    check_sweep_sampled(oracle_mod, old, new, L, d, J, seed, rep, t, beta, 3000, 0xA1)

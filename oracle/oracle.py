"""ctypes wrapper of the C oracle (test infrastructure only; see ``spin_oracle.c``).

Every function mirrors one C function; numpy arrays carry the spins (int8,
site index ``x + L*(y + L*z)``) and couplings (int8, layout ``[dir][site]``).
``OracleLib(path)`` binds any build of ``spin_oracle.c`` (the tests use this
to load deliberately broken copies); the module-level functions use the
default build next to this file.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "spin_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def compile_oracle(src, out):
    """gcc build of one oracle source file into a shared library."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force=True):
    """Compile spin_oracle.c into liboracle.so next to it."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(SOURCE):
        return _LIB
    return compile_oracle(SOURCE, _LIB)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleLib:
    """One loaded build of the oracle."""

    def __init__(self, path):
        lib = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i8p = ctypes.POINTER(ctypes.c_int8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_table.argtypes = [ctypes.c_double, ctypes.c_int, u64p]
        lib.oracle_table.restype = None
        lib.oracle_init_spins.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, i8p]
        lib.oracle_init_spins.restype = ctypes.c_int
        lib.oracle_couplings.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, i8p]
        lib.oracle_couplings.restype = ctypes.c_int
        lib.oracle_measure.argtypes = [ctypes.c_int, ctypes.c_int, i8p, i8p, i64p, i64p]
        lib.oracle_measure.restype = None
        lib.oracle_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i8p, i8p, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      i64p, i64p, ctypes.c_int, u64p]
        lib.oracle_sweeps.restype = ctypes.c_int
        lib.oracle_coarse_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i8p, i8p, ctypes.c_uint64, ctypes.c_uint32,
                                             ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, i64p, i64p]
        lib.oracle_coarse_sweeps.restype = ctypes.c_int
        lib.oracle_msc_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i8p, i8p, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int, i64p, i64p]
        lib.oracle_msc_sweeps.restype = ctypes.c_int
        lib.oracle_lcg_skip.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_lcg_skip.restype = ctypes.c_uint64
        lib.oracle_lcg_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, u64p]
        lib.oracle_lcg_init.restype = ctypes.c_int
        lib.oracle_lcg_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i8p, i8p, u64p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int, i64p, i64p]
        lib.oracle_lcg_sweeps.restype = ctypes.c_int
        f32p, f64p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        lib.oracle_heis_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, f32p]
        lib.oracle_heis_init.restype = ctypes.c_int
        lib.oracle_heis_measure.argtypes = [ctypes.c_int, ctypes.c_int, f32p, f64p, f64p]
        lib.oracle_heis_measure.restype = None
        lib.oracle_heis_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, f32p, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int, f64p, f64p]
        lib.oracle_heis_sweeps.restype = ctypes.c_int
        lib.oracle_heis_direction.argtypes = [ctypes.c_uint32, ctypes.c_uint32, f32p]
        lib.oracle_heis_direction.restype = None
        lib.oracle_heis_accept.argtypes = [ctypes.c_float, ctypes.c_float]
        lib.oracle_heis_accept.restype = ctypes.c_int
        self.lib = lib

    def philox4x32_10(self, ctr, key):
        """Philox4x32-10 block for counter (c0..c3) and key (k0, k1) -> 4 uint32 words."""
        c = np.asarray(ctr, dtype=np.uint32).copy()
        k = np.asarray(key, dtype=np.uint32).copy()
        out = np.zeros(4, dtype=np.uint32)
        self.lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                                      _ptr(out, ctypes.c_uint32))
        return out

    def table(self, beta, d):
        """Acceptance thresholds T[(k+z)/2] as uint64 (Eq. 2)."""
        out = np.zeros(2 * d + 1, dtype=np.uint64)
        self.lib.oracle_table(float(beta), int(d), _ptr(out, ctypes.c_uint64))
        return out

    def init_spins(self, L, d, seed, replica=0):
        spins = np.empty(L ** d, dtype=np.int8)
        if self.lib.oracle_init_spins(L, d, seed, replica, _ptr(spins, ctypes.c_int8)) != 0:
            raise ValueError("bad lattice shape")
        return spins

    def couplings(self, L, d, cseed, realisation=0):
        J = np.empty(d * L ** d, dtype=np.int8)
        if self.lib.oracle_couplings(L, d, cseed, realisation, _ptr(J, ctypes.c_int8)) != 0:
            raise ValueError("bad lattice shape")
        return J

    def measure(self, L, d, J, spins):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        Jarr = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        Jp = None if Jarr is None else _ptr(Jarr, ctypes.c_int8)
        E = ctypes.c_int64()
        M = ctypes.c_int64()
        self.lib.oracle_measure(L, d, Jp, _ptr(spins, ctypes.c_int8), ctypes.byref(E), ctypes.byref(M))
        return E.value, M.value

    def sweeps(self, L, d, J, spins, seed, replica, t0, n, beta, every=0, order=0, stats=None):
        """Advance ``spins`` in place by n sweeps starting at absolute sweep t0.

        Returns (E, M) int64 arrays with n//every records (empty if every == 0).
        ``stats`` (uint64 array of 2*(2d+1)) accumulates per-class attempts and
        acceptances when given.
        """
        assert spins.dtype == np.int8 and spins.flags.c_contiguous
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1), dtype=np.int64)
        M = np.zeros(max(nrec, 1), dtype=np.int64)
        Jarr = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        Jp = None if Jarr is None else _ptr(Jarr, ctypes.c_int8)
        sp = None
        if stats is not None:
            assert stats.dtype == np.uint64 and stats.size == 2 * (2 * d + 1)
            sp = _ptr(stats, ctypes.c_uint64)
        rc = self.lib.oracle_sweeps(L, d, Jp, _ptr(spins, ctypes.c_int8), seed, replica, t0, n, float(beta),
                                    every, _ptr(E, ctypes.c_int64), _ptr(M, ctypes.c_int64), order, sp)
        if rc != 0:
            raise ValueError("oracle_sweeps rejected its arguments")
        return E[:nrec].copy(), M[:nrec].copy()

    def coarse_sweeps(self, L, d, J, spins, seed, replica, t0, n, beta, T, k, every=0):
        """The paper's coarse-tile schedule (tile edge T, k hits per tile load): n sweeps in place."""
        assert spins.dtype == np.int8 and spins.flags.c_contiguous
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1), dtype=np.int64)
        M = np.zeros(max(nrec, 1), dtype=np.int64)
        Jarr = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        Jp = None if Jarr is None else _ptr(Jarr, ctypes.c_int8)
        rc = self.lib.oracle_coarse_sweeps(L, d, Jp, _ptr(spins, ctypes.c_int8), seed, replica, t0, n, float(beta),
                                           T, k, every, _ptr(E, ctypes.c_int64), _ptr(M, ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle_coarse_sweeps rejected its arguments")
        return E[:nrec].copy(), M[:nrec].copy()

    def msc_sweeps(self, L, d, J, spins, seed, p0, t0, n, beta, every=0):
        """Multi-spin-coded +-J glass: spins int8[32, N], J int8[32, d, N]; n sweeps in place.
        Returns E, M int64[n//every, 32]."""
        assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.size == 32 * L ** d
        Jarr = np.ascontiguousarray(J, dtype=np.int8)
        assert Jarr.size == 32 * d * L ** d
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1) * 32, dtype=np.int64)
        M = np.zeros(max(nrec, 1) * 32, dtype=np.int64)
        rc = self.lib.oracle_msc_sweeps(L, d, _ptr(Jarr, ctypes.c_int8), _ptr(spins, ctypes.c_int8), seed, p0, t0, n,
                                        float(beta), every, _ptr(E, ctypes.c_int64), _ptr(M, ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle_msc_sweeps rejected its arguments")
        return E[:nrec * 32].reshape(nrec, 32).copy(), M[:nrec * 32].reshape(nrec, 32).copy()

    def lcg_skip(self, mode, x, k):
        """State x of LCG mode 1/2 (32-bit) or 3 (64-bit) advanced by k steps."""
        return int(self.lib.oracle_lcg_skip(int(mode), int(x), int(k)))

    def lcg_init(self, L, d, mode, seed, replica=0):
        """Initial generator states (uint64[L^d/8]) of LCG mode 1, 2 or 3."""
        st = np.zeros((L ** d) // 8, dtype=np.uint64)
        if self.lib.oracle_lcg_init(L, d, int(mode), seed, replica, _ptr(st, ctypes.c_uint64)) != 0:
            raise ValueError("oracle_lcg_init rejected its arguments")
        return st

    def lcg_sweeps(self, L, d, J, spins, state, mode, n, beta, every=0):
        """n sweeps of the canonical chain drawing from per-group LCG states (advanced in place)."""
        assert spins.dtype == np.int8 and spins.flags.c_contiguous
        assert state.dtype == np.uint64 and state.flags.c_contiguous and state.size == (L ** d) // 8
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1), dtype=np.int64)
        M = np.zeros(max(nrec, 1), dtype=np.int64)
        Jarr = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        Jp = None if Jarr is None else _ptr(Jarr, ctypes.c_int8)
        rc = self.lib.oracle_lcg_sweeps(L, d, Jp, _ptr(spins, ctypes.c_int8), _ptr(state, ctypes.c_uint64), int(mode),
                                        n, float(beta), every, _ptr(E, ctypes.c_int64), _ptr(M, ctypes.c_int64))
        if rc != 0:
            raise ValueError("oracle_lcg_sweeps rejected its arguments")
        return E[:nrec].copy(), M[:nrec].copy()

    def heis_init(self, L, d, seed, replica=0):
        """Heisenberg hot start: float32[N, 4] (x, y, z, 0) per site."""
        sp = np.zeros((L ** d, 4), dtype=np.float32)
        if self.lib.oracle_heis_init(L, d, seed, replica, _ptr(sp, ctypes.c_float)) != 0:
            raise ValueError("oracle_heis_init rejected its arguments")
        return sp

    def heis_measure(self, L, d, spins):
        """(E, M vector) of a Heisenberg configuration, in double."""
        E = ctypes.c_double()
        M = np.zeros(3, dtype=np.float64)
        self.lib.oracle_heis_measure(L, d, _ptr(spins, ctypes.c_float), ctypes.byref(E), _ptr(M, ctypes.c_double))
        return E.value, M

    def heis_direction(self, w0, w1):
        """Trial direction (float32[3]) of the Philox words w0, w1."""
        v = np.zeros(3, dtype=np.float32)
        self.lib.oracle_heis_direction(int(w0), int(w1), _ptr(v, ctypes.c_float))
        return v

    def heis_accept(self, u, y):
        """The acceptance test u < exp(y) for float u and y, as the sweep takes it."""
        return bool(self.lib.oracle_heis_accept(float(u), float(y)))

    def heis_sweeps(self, L, d, spins, seed, replica, t0, n, beta, every=0):
        """n Heisenberg sweeps in place (float32[N, 4]); records (E, |M|) after every every-th sweep."""
        assert spins.dtype == np.float32 and spins.flags.c_contiguous and spins.shape == (L ** d, 4)
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1), dtype=np.float64)
        M = np.zeros(max(nrec, 1), dtype=np.float64)
        rc = self.lib.oracle_heis_sweeps(L, d, _ptr(spins, ctypes.c_float), seed, replica, t0, n, float(beta), every,
                                         _ptr(E, ctypes.c_double), _ptr(M, ctypes.c_double))
        if rc != 0:
            raise ValueError("oracle_heis_sweeps rejected its arguments")
        return E[:nrec].copy(), M[:nrec].copy()


_default = None


def default():
    global _default
    if _default is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(SOURCE):
            build()
        _default = OracleLib(_LIB)
    return _default


def philox4x32_10(ctr, key):
    return default().philox4x32_10(ctr, key)


def table(beta, d):
    return default().table(beta, d)


def init_spins(L, d, seed, replica=0):
    return default().init_spins(L, d, seed, replica)


def couplings(L, d, cseed, realisation=0):
    return default().couplings(L, d, cseed, realisation)


def measure(L, d, J, spins):
    return default().measure(L, d, J, spins)


def sweeps(L, d, J, spins, seed, replica, t0, n, beta, every=0, order=0, stats=None):
    return default().sweeps(L, d, J, spins, seed, replica, t0, n, beta, every, order, stats)


def coarse_sweeps(L, d, J, spins, seed, replica, t0, n, beta, T, k, every=0):
    return default().coarse_sweeps(L, d, J, spins, seed, replica, t0, n, beta, T, k, every)


def msc_sweeps(L, d, J, spins, seed, p0, t0, n, beta, every=0):
    return default().msc_sweeps(L, d, J, spins, seed, p0, t0, n, beta, every)


def lcg_skip(mode, x, k):
    return default().lcg_skip(mode, x, k)


def lcg_init(L, d, mode, seed, replica=0):
    return default().lcg_init(L, d, mode, seed, replica)


def lcg_sweeps(L, d, J, spins, state, mode, n, beta, every=0):
    return default().lcg_sweeps(L, d, J, spins, state, mode, n, beta, every)


def heis_init(L, d, seed, replica=0):
    return default().heis_init(L, d, seed, replica)


def heis_measure(L, d, spins):
    return default().heis_measure(L, d, spins)


def heis_direction(w0, w1):
    return default().heis_direction(w0, w1)


def heis_accept(u, y):
    return default().heis_accept(u, y)


def heis_sweeps(L, d, spins, seed, replica, t0, n, beta, every=0):
    return default().heis_sweeps(L, d, spins, seed, replica, t0, n, beta, every)


class MscChain:
    """32 multi-spin-coded +-J systems: realisations r0 + b, hot starts of replicas p0 + b."""

    def __init__(self, L, d, cseed, r0, seed, p0, lib=None):
        self.lib = lib or default()
        self.L, self.d, self.seed, self.p0 = L, d, seed, p0
        self.J = np.stack([self.lib.couplings(L, d, cseed, r0 + b) for b in range(32)])
        self.spins = np.stack([self.lib.init_spins(L, d, seed, p0 + b) for b in range(32)])
        self.t = 0

    def sweep(self, n, beta, every=0):
        E, M = self.lib.msc_sweeps(self.L, self.d, self.J, self.spins, self.seed, self.p0, self.t, n, beta, every)
        self.t += n
        return E, M

    def measure(self):
        out = [self.lib.measure(self.L, self.d, self.J[b], self.spins[b]) for b in range(32)]
        return np.array([e for e, _ in out]), np.array([m for _, m in out])

class LcgChain:
    """One lattice of the canonical chain whose draws come from per-group LCG streams (mode 1..3)."""

    def __init__(self, L, d, seed, mode, replica=0, J=None, lib=None):
        self.lib = lib or default()
        self.L, self.d, self.mode, self.J = L, d, mode, J
        self.spins = self.lib.init_spins(L, d, seed, replica)
        self.state = self.lib.lcg_init(L, d, mode, seed, replica)

    def sweep(self, n, beta, every=0):
        return self.lib.lcg_sweeps(self.L, self.d, self.J, self.spins, self.state, self.mode, n, beta, every)

    def measure(self):
        return self.lib.measure(self.L, self.d, self.J, self.spins)


class HeisChain:
    """One classical Heisenberg lattice (float32 unit vectors) advanced by the oracle."""

    def __init__(self, L, d, seed, replica=0, lib=None):
        self.lib = lib or default()
        self.L, self.d, self.seed, self.replica = L, d, seed, replica
        self.spins = self.lib.heis_init(L, d, seed, replica)
        self.t = 0

    def sweep(self, n, beta, every=0):
        E, M = self.lib.heis_sweeps(self.L, self.d, self.spins, self.seed, self.replica, self.t, n, beta, every)
        self.t += n
        return E, M

    def measure(self):
        return self.lib.heis_measure(self.L, self.d, self.spins)


class Chain:
    """Convenience state holder: one lattice advanced by an oracle build."""

    def __init__(self, L, d, seed, replica=0, J=None, spins=None, lib=None):
        self.lib = lib or default()
        self.L, self.d, self.seed, self.replica, self.J = L, d, seed, replica, J
        self.spins = (self.lib.init_spins(L, d, seed, replica) if spins is None
                      else np.array(spins, dtype=np.int8))
        self.t = 0

    def sweep(self, n, beta, every=0, order=0, stats=None):
        E, M = self.lib.sweeps(self.L, self.d, self.J, self.spins, self.seed, self.replica, self.t, n, beta,
                               every, order, stats)
        self.t += n
        return E, M

    def coarse_sweep(self, n, beta, T, k, every=0):
        E, M = self.lib.coarse_sweeps(self.L, self.d, self.J, self.spins, self.seed, self.replica, self.t, n, beta,
                                      T, k, every)
        self.t += n
        return E, M

    def measure(self):
        return self.lib.measure(self.L, self.d, self.J, self.spins)

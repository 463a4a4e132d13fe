"""ctypes binding of libspin.so: the C ABI of include/spin.h under the same names.

Argument marshalling only; every step of the path runs in the library's HIP
kernels.  Loading fails loudly (``RuntimeError``) when the built library is
missing: there is no CPU fallback.  PyTorch is used only for device memory
(``use_torch_allocator``) and streams (``Lattice(..., stream=...)``).
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspin.so")

SPIN_ISING, SPIN_EA_PMJ = 0, 1
SPIN_OK, SPIN_EINVAL, SPIN_ENOMEM, SPIN_EDEVICE, SPIN_ESTATE = 0, -1, -2, -3, -4
SPIN_KERNEL_AUTO, SPIN_KERNEL_GENERIC, SPIN_KERNEL_RESIDENT, SPIN_KERNEL_TILED, SPIN_KERNEL_FUSED = 0, 1, 2, 3, 4
SPIN_KERNEL_STREAM = 5
SPIN_SCHEDULE_CHECKERBOARD, SPIN_SCHEDULE_COARSE = 0, 1
SPIN_RNG_PHILOX, SPIN_RNG_LCG32_ARRAY, SPIN_RNG_LCG32_DISJOINT, SPIN_RNG_LCG64_DISJOINT = 0, 1, 2, 3
KERNEL_NAMES = {0: "auto", 1: "generic", 2: "resident", 3: "tiled", 4: "fused", 5: "stream"}

# Every symbol include/spin.h declares, with (restype, argtypes).
_c = ctypes
_P = _c.c_void_p
_i8p = _c.POINTER(_c.c_int8)
_i64p = _c.POINTER(_c.c_int64)
_u64p = _c.POINTER(_c.c_uint64)
_f32p = _c.POINTER(_c.c_float)
_f64p = _c.POINTER(_c.c_double)
ALLOC_FN = _c.CFUNCTYPE(_c.c_void_p, _c.c_size_t, _c.c_void_p)
RELEASE_FN = _c.CFUNCTYPE(None, _c.c_void_p, _c.c_void_p)


class spin_config(_c.Structure):
    _fields_ = [("model", _c.c_int), ("L", _c.c_int), ("d", _c.c_int), ("couplings", _i8p),
                ("coupling_seed", _c.c_uint64), ("realisation", _c.c_uint32), ("seed", _c.c_uint64),
                ("replica", _c.c_uint32), ("stream", _c.c_void_p)]


class spin_desc(_c.Structure):
    _fields_ = [("model", _c.c_int), ("L", _c.c_int), ("d", _c.c_int), ("couplings", _i8p),
                ("coupling_seed", _c.c_uint64), ("realisation", _c.c_uint32), ("seed", _c.c_uint64),
                ("replica", _c.c_uint32)]


_ip = _c.POINTER(_c.c_int)
_dp = _c.POINTER(_c.c_double)

SIGNATURES = {
    "spin_create": (_P, [_c.c_int, _c.c_int, _c.c_int, _i8p, _c.c_uint64]),
    "spin_create_config": (_P, [_c.POINTER(spin_config)]),
    "spin_free": (None, [_P]),
    "spin_sweep": (_c.c_int, [_P, _c.c_int, _c.c_double]),
    "spin_sweep_record": (_c.c_int, [_P, _c.c_int, _c.c_double, _c.c_int, _i64p, _i64p]),
    "spin_sweep_record_device": (_c.c_int, [_P, _c.c_int, _c.c_double, _c.c_int, _c.c_void_p, _c.c_void_p]),
    "spin_sweep_record_noalloc": (_c.c_int, [_P, _c.c_int, _c.c_double, _c.c_int, _c.c_void_p, _c.c_void_p]),
    "spin_measure": (_c.c_int, [_P, _i64p, _i64p]),
    "spin_get_spins": (_c.c_int, [_P, _i8p, _c.c_size_t]),
    "spin_set_spins": (_c.c_int, [_P, _i8p, _c.c_size_t]),
    "spin_get_couplings": (_c.c_int, [_P, _i8p, _c.c_size_t]),
    "spin_sweeps_done": (_c.c_uint64, [_P]),
    "spin_set_sweeps_done": (_c.c_int, [_P, _c.c_uint64]),
    "spin_set_replica": (_c.c_int, [_P, _c.c_uint32]),
    "spin_set_stream": (_c.c_int, [_P, _c.c_void_p]),
    "spin_set_kernel": (_c.c_int, [_P, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "spin_get_kernel": (_c.c_int, [_P]),
    "spin_get_tile": (_c.c_int, [_P, _ip, _ip, _ip, _ip]),
    "spin_autotune": (_c.c_int, [_P, _c.c_double, _c.c_int]),
    "spin_set_schedule": (_c.c_int, [_P, _c.c_int, _c.c_int, _c.c_int]),
    "spin_set_rng": (_c.c_int, [_P, _c.c_int]),
    "spin_heis_create": (_P, [_c.c_int, _c.c_int, _c.c_uint64, _c.c_uint32, _P]),
    "spin_heis_free": (None, [_P]),
    "spin_heis_sweep": (_c.c_int, [_P, _c.c_int, _c.c_double]),
    "spin_heis_sweep_record": (_c.c_int, [_P, _c.c_int, _c.c_double, _c.c_int, _f64p, _f64p]),
    "spin_heis_measure": (_c.c_int, [_P, _f64p, _f64p]),
    "spin_heis_get_spins": (_c.c_int, [_P, _f32p, _c.c_size_t]),
    "spin_heis_sweeps_done": (_c.c_uint64, [_P]),
    "spin_heis_set_spins": (_c.c_int, [_P, _f32p, _c.c_size_t]),
    "spin_heis_set_sweeps_done": (_c.c_int, [_P, _c.c_uint64]),
    "spin_heis_synchronize": (_c.c_int, [_P]),
    "spin_get_rng_state": (_c.c_int, [_P, _u64p, _c.c_size_t]),
    "spin_msc_create": (_P, [_c.c_int, _c.c_int, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32, _c.c_void_p]),
    "spin_msc_free": (None, [_P]),
    "spin_msc_sweep": (_c.c_int, [_P, _c.c_int, _c.c_double]),
    "spin_msc_sweep_record": (_c.c_int, [_P, _c.c_int, _c.c_double, _c.c_int, _i64p, _i64p]),
    "spin_msc_measure": (_c.c_int, [_P, _i64p, _i64p]),
    "spin_msc_get_spins": (_c.c_int, [_P, _c.c_int, _i8p, _c.c_size_t]),
    "spin_msc_sweeps_done": (_c.c_uint64, [_P]),
    "spin_msc_set_kernel": (_c.c_int, [_P, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "spin_msc_synchronize": (_c.c_int, [_P]),
    "spin_msc_kernel": (_c.c_int, [_P]),
    "spin_synchronize": (_c.c_int, [_P]),
    "spin_device_spins": (_c.c_void_p, [_P]),
    "spin_threshold_table": (_c.c_int, [_c.c_double, _c.c_int, _u64p]),
    "spin_set_allocator": (None, [ALLOC_FN, RELEASE_FN, _c.c_void_p]),
    "spin_debug_fault_alloc": (_c.c_int, [_c.c_int64]),
    "spin_debug_live_allocations": (_c.c_int64, []),
    "spin_last_error": (_c.c_char_p, []),
    "spin_last_status": (_c.c_int, []),
    "spin_version": (_c.c_char_p, []),
    "spin_batch_create": (_P, [_c.c_int, _c.POINTER(spin_desc), _c.c_void_p]),
    "spin_batch_free": (None, [_P]),
    "spin_batch_size": (_c.c_int, [_P]),
    "spin_batch_add": (_c.c_int, [_P, _c.POINTER(spin_desc)]),
    "spin_batch_remove": (_c.c_int, [_P, _c.c_int]),
    "spin_batch_is_member": (_c.c_int, [_P, _c.c_int]),
    "spin_batch_footprint": (_c.c_uint64, [_P, _c.c_int]),
    "spin_batch_autotune": (_c.c_int, [_P, _c.c_double, _c.c_int]),
    "spin_batch_plan": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)]),
    "spin_batch_sweep": (_c.c_int, [_P, _ip, _dp, _c.c_int, _i64p, _i64p]),
    "spin_batch_sweep_device": (_c.c_int, [_P, _ip, _dp, _c.c_int, _c.c_void_p, _c.c_void_p]),
    "spin_batch_measure": (_c.c_int, [_P, _i64p, _i64p]),
    "spin_batch_get_spins": (_c.c_int, [_P, _c.c_int, _i8p, _c.c_size_t]),
    "spin_batch_set_spins": (_c.c_int, [_P, _c.c_int, _i8p, _c.c_size_t]),
    "spin_batch_sweeps_done": (_c.c_uint64, [_P, _c.c_int]),
    "spin_batch_set_workgroups_per_cu": (_c.c_int, [_P, _c.c_int]),
    "spin_batch_synchronize": (_c.c_int, [_P]),
}

# The ceiling probes of include/spin_probe.h (measurement only).
PROBE_SIGNATURES = {
    "spin_probe_alu": (_c.c_int, [_c.c_int, _c.c_void_p, _c.c_uint32, _c.c_uint32, _c.c_uint64, _c.c_void_p]),
    "spin_probe_copy": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_uint64, _c.c_uint32, _c.c_void_p]),
}
SPIN_PROBE_PHILOX, SPIN_PROBE_MAD64, SPIN_PROBE_ALU32 = 0, 1, 2

_lib = None


def load():
    """Load libspin.so (built by ``paper_1006_3865_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libspin.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        lib = _c.CDLL(LIB_PATH)
        for name, (res, args) in list(SIGNATURES.items()) + list(PROBE_SIGNATURES.items()):
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SpinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("spin error %d: %s" % (code, msg))
        self.code = code


def _null_status():
    """Status of the constructor call that just returned NULL (EINVAL if none was set)."""
    rc = load().spin_last_status()
    return rc if rc < 0 else SPIN_EINVAL


def _check(rc):
    """Raise on a negative status; return rc (a slot index for spin_batch_add)."""
    if rc < 0:
        raise SpinError(rc, load().spin_last_error().decode())
    return rc


def _i8(a):
    return a.ctypes.data_as(_i8p)


def check_record_tensors(E, M, need):
    """Validate device record arrays before their pointers reach the C ABI: torch int64 tensors on a
    GPU, contiguous, with at least `need` elements each.  A wrong dtype, host memory or a short
    tensor would make the record kernels write outside the allocation, so they raise ValueError."""
    if need <= 0:
        return
    for name, t in (("E", E), ("M", M)):
        if t is None:
            raise ValueError("%s: a device int64 tensor of >= %d elements is required" % (name, need))
        dtype = getattr(t, "dtype", None)
        if dtype is None or str(dtype) != "torch.int64":
            raise ValueError("%s must be a torch.int64 tensor (got %s)" % (name, dtype))
        if not getattr(t, "is_cuda", False):
            raise ValueError("%s must live in GPU memory (got device %s)" % (name, getattr(t, "device", "?")))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.numel() < need:
            raise ValueError("%s holds %d elements, the call writes %d" % (name, t.numel(), need))


# --------------------------------------------------------------- C names

def spin_create(model, L, d, couplings, seed):
    lib = load()
    J = None if couplings is None else np.ascontiguousarray(couplings, dtype=np.int8)
    h = lib.spin_create(model, L, d, None if J is None else _i8(J), seed)
    if not h:
        raise SpinError(_null_status(), lib.spin_last_error().decode())
    return h


def spin_create_config(model, L, d, couplings=None, coupling_seed=0, realisation=0, seed=0, replica=0,
                       stream=None):
    lib = load()
    J = None if couplings is None else np.ascontiguousarray(couplings, dtype=np.int8)
    cfg = spin_config(model, L, d, None if J is None else _i8(J), coupling_seed, realisation, seed, replica,
                      stream)
    h = lib.spin_create_config(_c.byref(cfg))
    if not h:
        raise SpinError(_null_status(), lib.spin_last_error().decode())
    return h


def spin_free(h):
    load().spin_free(h)


def spin_sweep(h, n, beta):
    return _check(load().spin_sweep(h, n, beta))


def spin_sweep_record(h, n, beta, every):
    nrec = n // every if every > 0 else 0
    E = np.zeros(max(nrec, 1), dtype=np.int64)
    M = np.zeros(max(nrec, 1), dtype=np.int64)
    _check(load().spin_sweep_record(h, n, beta, every, E.ctypes.data_as(_i64p), M.ctypes.data_as(_i64p)))
    return E[:nrec], M[:nrec]


def spin_sweep_record_device(h, n, beta, every, E_ptr, M_ptr):
    return _check(load().spin_sweep_record_device(h, n, beta, every, E_ptr, M_ptr))


def spin_sweep_record_noalloc(h, n, beta, every, E_ptr, M_ptr):
    return _check(load().spin_sweep_record_noalloc(h, n, beta, every, E_ptr, M_ptr))


# bytes of the device scratch array behind spin_sweep_record_noalloc (SPIN_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 2 << 20


def spin_measure(h):
    E, M = _c.c_int64(), _c.c_int64()
    _check(load().spin_measure(h, _c.byref(E), _c.byref(M)))
    return E.value, M.value


def spin_get_spins(h, n):
    out = np.empty(n, dtype=np.int8)
    _check(load().spin_get_spins(h, _i8(out), n))
    return out


def spin_set_spins(h, spins):
    a = np.ascontiguousarray(spins, dtype=np.int8)
    return _check(load().spin_set_spins(h, _i8(a), a.size))


def spin_get_couplings(h, n):
    out = np.empty(n, dtype=np.int8)
    _check(load().spin_get_couplings(h, _i8(out), n))
    return out


def spin_sweeps_done(h):
    return int(load().spin_sweeps_done(h))


def spin_set_sweeps_done(h, t):
    return _check(load().spin_set_sweeps_done(h, t))


def spin_set_replica(h, replica):
    return _check(load().spin_set_replica(h, replica))


def spin_set_stream(h, stream):
    return _check(load().spin_set_stream(h, stream))


def spin_set_kernel(h, kernel, tile_x=0, tile_y=0, tile_z=0, threads=0):
    return _check(load().spin_set_kernel(h, kernel, tile_x, tile_y, tile_z, threads))


def spin_get_kernel(h):
    k = load().spin_get_kernel(h)
    if k < 0:
        _check(k)
    return k


def spin_synchronize(h):
    return _check(load().spin_synchronize(h))


def spin_device_spins(h):
    return load().spin_device_spins(h)


def spin_threshold_table(beta, d):
    T = np.zeros(2 * d + 1, dtype=np.uint64)
    _check(load().spin_threshold_table(beta, d, T.ctypes.data_as(_u64p)))
    return T


def spin_last_error():
    return load().spin_last_error().decode()


def spin_version():
    return load().spin_version().decode()


# ------------------------------------------------- torch device memory hook

_torch_hooks = None


def use_torch_allocator():
    """Route the library's device allocations through torch's caching allocator."""
    global _torch_hooks
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
        except Exception:
            return None

    def _release(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    _torch_hooks = (ALLOC_FN(_alloc), RELEASE_FN(_release))
    load().spin_set_allocator(_torch_hooks[0], _torch_hooks[1], None)


def fault_alloc(after):
    """Make the library's allocation after `after` more successful ones fail (-1: off)."""
    _check(load().spin_debug_fault_alloc(int(after)))


def live_allocations():
    """Device blocks the library holds now."""
    return int(load().spin_debug_live_allocations())


def batch_plan(d, model, L):
    """(threads, workgroups per CU) of the persistent kernel's plan for a shape, or None."""
    t, w = _c.c_int(), _c.c_int()
    return (t.value, w.value) if load().spin_batch_plan(d, model, L, _c.byref(t), _c.byref(w)) else None


def use_hip_allocator():
    load().spin_set_allocator(ALLOC_FN(), RELEASE_FN(), None)


# ---------------------------------------------------------------- wrapper

class Lattice:
    """One lattice owned by the library.  Mirrors the C calls one to one."""

    def __init__(self, model, L, d, seed, couplings=None, coupling_seed=None, realisation=0, replica=0,
                 stream=None):
        if model == SPIN_EA_PMJ and couplings is None and coupling_seed is None:
            raise ValueError("EA lattice needs couplings or a coupling_seed")
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        self.h = spin_create_config(model, L, d, couplings, coupling_seed or 0, realisation, seed, replica, sp)
        self.model, self.L, self.d, self.N = model, L, d, L ** d

    def close(self):
        if self.h:
            spin_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n, beta):
        spin_sweep(self.h, n, beta)

    def sweep_record(self, n, beta, every):
        return spin_sweep_record(self.h, n, beta, every)

    def sweep_record_device(self, n, beta, every, E, M):
        """E, M: torch int64 CUDA tensors with >= n//every elements."""
        if every < 1:
            raise ValueError("every must be >= 1")
        check_record_tensors(E, M, n // every if n > 0 else 0)
        spin_sweep_record_device(self.h, n, beta, every, E.data_ptr() if E is not None else None,
                                 M.data_ptr() if M is not None else None)

    def sweep_record_noalloc(self, n, beta, every, E, M):
        """As sweep_record_device, on the library's fixed scratch array: no device allocation."""
        if every < 1:
            raise ValueError("every must be >= 1")
        check_record_tensors(E, M, n // every if n > 0 else 0)
        spin_sweep_record_noalloc(self.h, n, beta, every, E.data_ptr() if E is not None else None,
                                  M.data_ptr() if M is not None else None)

    def measure(self):
        return spin_measure(self.h)

    def spins(self):
        return spin_get_spins(self.h, self.N)

    def set_spins(self, s):
        spin_set_spins(self.h, s)

    def couplings(self):
        return spin_get_couplings(self.h, self.d * self.N)

    @property
    def t(self):
        return spin_sweeps_done(self.h)

    @t.setter
    def t(self, value):
        spin_set_sweeps_done(self.h, value)

    def set_replica(self, replica):
        """Later updates draw as replica `replica` (spins and sweep index stay)."""
        spin_set_replica(self.h, replica)

    def set_kernel(self, kernel, tile_x=0, tile_y=0, tile_z=0, threads=0):
        spin_set_kernel(self.h, kernel, tile_x, tile_y, tile_z, threads)

    def set_schedule(self, schedule, tile=0, hits=1):
        """SPIN_SCHEDULE_COARSE with tile edge and hits: the paper's coarse-tile multi-hit order."""
        _check(load().spin_set_schedule(self.h, int(schedule), int(tile), int(hits)))

    def set_rng(self, rng):
        """SPIN_RNG_PHILOX (the canonical chain) or one of the LCG modes of the RNG-quality experiment."""
        _check(load().spin_set_rng(self.h, int(rng)))

    def rng_state(self):
        """The LCG modes' generator states, one uint64 per 8-site group."""
        out = np.empty(self.N // 8, dtype=np.uint64)
        _check(load().spin_get_rng_state(self.h, out.ctypes.data_as(_u64p), out.size))
        return out

    def autotune(self, beta=0.44, sweeps=4):
        """Time every kernel family and tile for this shape, keep the fastest (see spin_autotune)."""
        return _check(load().spin_autotune(self.h, float(beta), int(sweeps)))

    @property
    def kernel(self):
        return spin_get_kernel(self.h)

    @property
    def tile(self):
        """(tile_x, tile_y, tile_z, threads) of the next sweep's kernel."""
        v = [_c.c_int(0) for _ in range(4)]
        _check(load().spin_get_tile(self.h, *[_c.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_stream(self, stream):
        spin_set_stream(self.h, stream if isinstance(stream, int) or stream is None else stream.cuda_stream)

    def synchronize(self):
        spin_synchronize(self.h)


# ------------------------------------------------------------------ batches

def _desc(d, keep):
    J = d.get("couplings")
    Jp = None
    if J is not None:
        J = np.ascontiguousarray(J, dtype=np.int8)
        keep.append(J)
        Jp = _i8(J)
    return spin_desc(d["model"], d["L"], d["d"], Jp, d.get("coupling_seed", 0), d.get("realisation", 0),
                     d.get("seed", 0), d.get("replica", 0))


def spin_batch_create(descs, stream=None):
    """descs: list of dicts with model, L, d and optional couplings, coupling_seed, realisation, seed, replica."""
    lib = load()
    arr = (spin_desc * max(len(descs), 1))()
    keep = []
    for i, d in enumerate(descs):
        arr[i] = _desc(d, keep)
    h = lib.spin_batch_create(len(descs), arr, stream)
    if not h:
        raise SpinError(_null_status(), lib.spin_last_error().decode())
    return h


class Batch:
    """A pool of lattices advanced together (slots; see spin_batch_* in spin.h)."""

    def __init__(self, descs=(), stream=None):
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        descs = list(descs)
        self.h = spin_batch_create(descs, sp)
        self.N = [d["L"] ** d["d"] for d in descs]
        self._mask = np.ones(len(descs), dtype=bool)   # slot holds a lattice

    @property
    def count(self):
        """Number of slots (members and free slots)."""
        return int(load().spin_batch_size(self.h))

    def add(self, desc):
        """Add a lattice; returns its slot."""
        keep = []
        d = _desc(desc, keep)
        slot = _check(load().spin_batch_add(self.h, _c.byref(d)))
        while len(self.N) <= slot:
            self.N.append(0)
            self._mask = np.append(self._mask, False)
        self.N[slot] = desc["L"] ** desc["d"]
        self._mask[slot] = True
        return slot

    def remove(self, i):
        _check(load().spin_batch_remove(self.h, i))
        self.N[i] = 0
        self._mask[i] = False

    def is_member(self, i):
        return bool(load().spin_batch_is_member(self.h, i))

    def members(self):
        return [int(i) for i in np.flatnonzero(self._mask)]

    def footprint(self, i):
        return int(load().spin_batch_footprint(self.h, i))

    def close(self):
        if self.h:
            load().spin_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, n, beta):
        S = len(self._mask)
        n = np.array(np.broadcast_to(np.asarray(n, dtype=np.int32), (S,)), dtype=np.int32)
        n[~self._mask] = 0
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (S,)), dtype=np.float64)
        return n, b

    def record_counts(self, n, every):
        n, _ = self._args(n, 0.0)
        if every <= 0:
            return np.zeros(len(self._mask), dtype=np.int64)
        counts = np.where(n > 0, n // every, 1).astype(np.int64)
        counts[~self._mask] = 0
        return counts

    def sweep(self, n, beta, every=0):
        """Returns a list of (E, M) record arrays per slot (empty when every == 0 or the slot is free)."""
        n, b = self._args(n, beta)
        counts = self.record_counts(n, every)
        tot = int(counts.sum())
        E = np.zeros(max(tot, 1), dtype=np.int64)
        M = np.zeros(max(tot, 1), dtype=np.int64)
        _check(load().spin_batch_sweep(self.h, n.ctypes.data_as(_ip), b.ctypes.data_as(_dp), every,
                                       E.ctypes.data_as(_i64p), M.ctypes.data_as(_i64p)))
        out, o = [], 0
        for c in counts:
            out.append((E[o:o + c].copy(), M[o:o + c].copy()))
            o += c
        return out

    def sweep_device(self, n, beta, every, E, M):
        """E, M: torch int64 CUDA tensors holding record_counts(n, every).sum() values."""
        n, b = self._args(n, beta)
        if every > 0:
            check_record_tensors(E, M, int(self.record_counts(n, every).sum()))
        self._hold = (n, b)
        _check(load().spin_batch_sweep_device(self.h, n.ctypes.data_as(_ip), b.ctypes.data_as(_dp), every,
                                              E.data_ptr() if E is not None else None,
                                              M.data_ptr() if M is not None else None))

    def measure(self):
        S = max(self.count, 1)
        E = np.zeros(S, dtype=np.int64)
        M = np.zeros(S, dtype=np.int64)
        _check(load().spin_batch_measure(self.h, E.ctypes.data_as(_i64p), M.ctypes.data_as(_i64p)))
        return E[:self.count], M[:self.count]

    def spins(self, i):
        out = np.empty(self.N[i], dtype=np.int8)
        _check(load().spin_batch_get_spins(self.h, i, _i8(out), out.size))
        return out

    def set_spins(self, i, s):
        a = np.ascontiguousarray(s, dtype=np.int8)
        _check(load().spin_batch_set_spins(self.h, i, _i8(a), a.size))

    def t(self, i):
        return int(load().spin_batch_sweeps_done(self.h, i))

    def autotune(self, beta, sweeps=20):
        """Time the persistent kernel's launch shapes per lattice shape of the pool; returns the
        number of shapes tuned (their plans apply to every pool and are persisted)."""
        return _check(load().spin_batch_autotune(self.h, float(beta), int(sweeps)))

    def set_workgroups_per_cu(self, w):
        _check(load().spin_batch_set_workgroups_per_cu(self.h, w))

    def synchronize(self):
        _check(load().spin_batch_synchronize(self.h))


# ------------------------------------------------------------ multi-spin coding

class Msc:
    """32 +-J systems in the bits of one word per site (see spin_msc_* in spin.h)."""

    def __init__(self, L, d, coupling_seed, realisation0, seed, replica0=0, stream=None):
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        lib = load()
        self.h = lib.spin_msc_create(L, d, coupling_seed, realisation0, seed, replica0, sp)
        if not self.h:
            raise SpinError(_null_status(), lib.spin_last_error().decode())
        self.L, self.d, self.N = L, d, L ** d

    def close(self):
        if self.h:
            load().spin_msc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n, beta):
        _check(load().spin_msc_sweep(self.h, int(n), float(beta)))

    def sweep_record(self, n, beta, every):
        nrec = n // every
        E = np.zeros(max(nrec, 1) * 32, dtype=np.int64)
        M = np.zeros(max(nrec, 1) * 32, dtype=np.int64)
        _check(load().spin_msc_sweep_record(self.h, int(n), float(beta), int(every), E.ctypes.data_as(_i64p),
                                            M.ctypes.data_as(_i64p)))
        return E[:nrec * 32].reshape(nrec, 32), M[:nrec * 32].reshape(nrec, 32)

    def measure(self):
        E = np.zeros(32, dtype=np.int64)
        M = np.zeros(32, dtype=np.int64)
        _check(load().spin_msc_measure(self.h, E.ctypes.data_as(_i64p), M.ctypes.data_as(_i64p)))
        return E, M

    def spins(self, system):
        out = np.empty(self.N, dtype=np.int8)
        _check(load().spin_msc_get_spins(self.h, int(system), _i8(out), out.size))
        return out

    @property
    def t(self):
        return int(load().spin_msc_sweeps_done(self.h))

    def set_kernel(self, streaming, rows=0, planes=0, threads=0, width=0):
        _check(load().spin_msc_set_kernel(self.h, int(streaming), int(rows), int(planes), int(threads), int(width)))

    @property
    def kernel(self):
        """0: one launch per colour; 1: streamed over planes; 2: register columns (3D L = 128, 256, 512)."""
        return int(load().spin_msc_kernel(self.h))

    def synchronize(self):
        _check(load().spin_msc_synchronize(self.h))


class Heis:
    """Classical Heisenberg lattice (continuous spins, float) owned by the library."""

    def __init__(self, L, d, seed, replica=0, stream=None):
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        self.h = load().spin_heis_create(int(L), int(d), int(seed), int(replica), sp)
        if not self.h:
            raise SpinError(_null_status(), load().spin_last_error().decode())
        self.L, self.d, self.N = L, d, L ** d

    def close(self):
        if self.h:
            load().spin_heis_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n, beta):
        _check(load().spin_heis_sweep(self.h, int(n), float(beta)))

    def sweep_record(self, n, beta, every):
        nrec = n // every if every > 0 else 0
        E = np.zeros(max(nrec, 1), dtype=np.float64)
        M = np.zeros(max(nrec, 1), dtype=np.float64)
        _check(load().spin_heis_sweep_record(self.h, int(n), float(beta), int(every), E.ctypes.data_as(_f64p),
                                             M.ctypes.data_as(_f64p)))
        return E[:nrec], M[:nrec]

    def measure(self):
        E = np.zeros(1, dtype=np.float64)
        M = np.zeros(3, dtype=np.float64)
        _check(load().spin_heis_measure(self.h, E.ctypes.data_as(_f64p), M.ctypes.data_as(_f64p)))
        return float(E[0]), M

    def spins(self):
        out = np.empty((self.N, 4), dtype=np.float32)
        _check(load().spin_heis_get_spins(self.h, out.ctypes.data_as(_f32p), out.size))
        return out

    def set_spins(self, spins):
        a = np.ascontiguousarray(spins, dtype=np.float32).reshape(self.N, 4)
        _check(load().spin_heis_set_spins(self.h, a.ctypes.data_as(_f32p), a.size))

    @property
    def t(self):
        return int(load().spin_heis_sweeps_done(self.h))

    @t.setter
    def t(self, value):
        _check(load().spin_heis_set_sweeps_done(self.h, int(value)))

    def synchronize(self):
        _check(load().spin_heis_synchronize(self.h))

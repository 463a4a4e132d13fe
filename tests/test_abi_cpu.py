"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, rejects bad arguments before touching the device, and its host-side
threshold table equals the oracle's (both follow Eq. 2 in IEEE double)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1006_3865_amd import spin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="spin.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(spin_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(spin.LIB_PATH):
        pytest.fail("libspin.so not built; run __graft_entry__.build()")
    return spin.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(spin.SIGNATURES), "binding and header disagree"


def test_probe_symbols_are_exported(lib):
    names = declared_functions("spin_probe.h")
    assert names == sorted(spin.PROBE_SIGNATURES)
    for n in names:
        assert hasattr(lib, n), n
    # argument errors come back before any launch
    assert lib.spin_probe_alu(7, None, 1, 1, 0, None) == spin.SPIN_EINVAL
    assert lib.spin_probe_copy(None, None, 16, 1, None) == spin.SPIN_EINVAL


def test_version(lib):
    assert spin.spin_version().startswith("spin-gfx950")


@pytest.mark.parametrize("beta", [0.0, 0.1, 0.2216544, 0.30, 0.4406868, 0.60, 1.0, 2.5, 3.0, math.inf])
@pytest.mark.parametrize("d", [2, 3])
def test_threshold_table_equals_oracle(lib, oracle_mod, beta, d):
    np.testing.assert_array_equal(spin.spin_threshold_table(beta, d), oracle_mod.table(beta, d))


@pytest.mark.parametrize("args", [
    (0, 5, 2), (0, 2, 2), (0, 8, 4), (2, 8, 2), (0, -8, 2), (1, 9, 3),
])
def test_create_rejects_bad_shapes(lib, args):
    model, L, d = args
    with pytest.raises(spin.SpinError) as e:
        spin.spin_create_config(model, L, d, couplings=None, coupling_seed=1, seed=1)
    assert e.value.code == spin.SPIN_EINVAL


def test_create_rejects_bad_couplings(lib):
    with pytest.raises(spin.SpinError):
        spin.spin_create(0, 8, 2, np.ones(128, dtype=np.int8), 1)  # Ising with couplings
    bad = np.ones(2 * 64, dtype=np.int8)
    bad[17] = 0
    with pytest.raises(spin.SpinError) as e:
        spin.spin_create(1, 8, 2, bad, 1)
    assert "coupling 17" in str(e.value)
    with pytest.raises(spin.SpinError):
        spin.spin_create(1, 8, 2, None, 1)  # EA without couplings via the short form


def test_null_handle_and_bad_beta(lib):
    assert lib.spin_sweep(None, 1, 0.5) == spin.SPIN_EINVAL
    assert "NULL" in spin.spin_last_error()
    T = np.zeros(5, dtype=np.uint64)
    assert lib.spin_threshold_table(float("nan"), 2, T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) == spin.SPIN_EINVAL
    assert lib.spin_threshold_table(-0.1, 2, T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) == spin.SPIN_EINVAL
    assert lib.spin_threshold_table(0.5, 4, T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) == spin.SPIN_EINVAL
    assert lib.spin_set_replica(None, 1) == spin.SPIN_EINVAL
    assert lib.spin_set_sweeps_done(None, 1) == spin.SPIN_EINVAL
    lib.spin_free(None)  # NULL-safe


def test_record_tensors_rejected_before_the_abi():
    """Device record arrays are checked in the binding: a wrong dtype, host memory, a strided view or
    too few elements raise ValueError, so no bad pointer reaches a record kernel."""
    import torch
    ok64 = torch.zeros(8, dtype=torch.int64)
    with pytest.raises(ValueError, match="int64"):
        spin.check_record_tensors(torch.zeros(8, dtype=torch.int32), ok64, 4)
    with pytest.raises(ValueError, match="GPU"):
        spin.check_record_tensors(ok64, ok64, 4)          # host tensors
    with pytest.raises(ValueError, match="required"):
        spin.check_record_tensors(None, ok64, 1)
    spin.check_record_tensors(None, None, 0)              # nothing recorded: nothing checked

    class FakeCuda:
        """Stands for a device tensor (no GPU here): dtype, device flag, layout and size."""
        def __init__(self, n, contiguous=True, dtype=torch.int64):
            self.dtype, self.is_cuda, self._n, self._c = dtype, True, n, contiguous

        def is_contiguous(self):
            return self._c

        def numel(self):
            return self._n

    spin.check_record_tensors(FakeCuda(4), FakeCuda(5), 4)
    with pytest.raises(ValueError, match="contiguous"):
        spin.check_record_tensors(FakeCuda(8, contiguous=False), FakeCuda(8), 4)
    with pytest.raises(ValueError, match="writes 6"):
        spin.check_record_tensors(FakeCuda(6), FakeCuda(5), 6)

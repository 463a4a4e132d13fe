"""CPU oracle for checkerboard Metropolis sweeps (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``spin_oracle.c`` (plain,
single-threaded C, built with gcc) through ctypes and shares no code with the
GPU library.  The definition it follows is stated in the header of
``spin_oracle.c`` with the passages of the paper it rests on.
"""
from .oracle import (  # noqa: F401
    OracleLib,
    SOURCE,
    build,
    compile_oracle,
    default,
    philox4x32_10,
    table,
    init_spins,
    couplings,
    measure,
    sweeps,
    coarse_sweeps,
    msc_sweeps,
    lcg_skip,
    lcg_init,
    lcg_sweeps,
    heis_accept,
    heis_direction,
    heis_init,
    heis_measure,
    heis_sweeps,
    MscChain,
    LcgChain,
    HeisChain,
    Chain,
)

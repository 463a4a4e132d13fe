"""MI355X (gfx950) checkerboard Metropolis sweeps of 2D/3D Ising and +-J EA spin models.

``spin``       ctypes binding of the C ABI (include/spin.h, libspin.so)
``workloads``  seeded synthetic inputs of the benchmark configurations
``build``      in-tree hipcc build of libspin.so

Importing the package loads nothing; ``spin.load()`` opens the library.
"""
__all__ = ["spin", "workloads", "build"]

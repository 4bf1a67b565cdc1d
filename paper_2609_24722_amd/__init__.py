"""MI355X (gfx950) engine for N unit charges with 1/r repulsion in the unit disk.

The compute lives in ``libcoulombdisk.so`` (hand-written HIP kernels behind the
C ABI declared in ``include/coulomb_disk.h``).  ``ops`` is a thin ctypes binding
with the same names; ``autograd`` wraps it in ``torch.autograd.Function``s;
``workloads`` draws seeded synthetic inputs.  Importing the package loads
nothing; the first call into ``ops`` loads the library and raises if it is
missing.
"""

FP64 = 0
MIXED = 1

__all__ = ["FP64", "MIXED"]

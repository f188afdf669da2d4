"""MI355X-native batched LSM dictionary (GPU LSM, Ashkiani et al.).

The method runs in hand-written HIP kernels for gfx950 behind the C ABI in
``include/lsm.h``; :mod:`paper_1707_05354_amd.lsm` is the thin ctypes binding
(argument marshalling only) and :mod:`paper_1707_05354_amd.workload` the
seeded synthetic input generator.  Importing the package loads nothing; the
HIP library is loaded on first use of the binding and a missing library is
an error, never a fallback.
"""

__all__ = ["lsm", "workload", "build"]

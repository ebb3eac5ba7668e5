"""MI355X-native grid-refined entropic (KBC) lattice Boltzmann.

The method (arXiv:1608.06915) runs in the HIP library libelbm.so behind the C ABI of
include/elbm.h; :mod:`paper_1608_06915_amd.elbm` is its ctypes binding and
:mod:`paper_1608_06915_amd.synth` the seeded workload generator.
"""
__all__ = ["elbm", "synth", "build"]

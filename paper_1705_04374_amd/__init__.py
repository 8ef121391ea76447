"""MI355X-native optimal-fidelity MLMC for cloud cavitation collapse.

A C-ABI HIP library (``libofm.so``, declared in ``include/ofm.h``) runs the
whole hot path on the GPU: sampled cloud geometry -> level-l finite-volume
solves of the five-equation two-phase model -> peak-pressure QoI -> OF-MLMC
moments, optimal coefficients, errors and sample allocation.  ``capi`` is the
thin ctypes binding; ``driver`` is the adaptive OF-MLMC loop on top of it.
"""
from . import capi  # noqa: F401

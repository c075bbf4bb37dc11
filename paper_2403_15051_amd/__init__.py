"""MI355X-native FDLB solver for the simplified Enskog equation in curvilinear geometries.

The hot path (one TVD-RK3 step over radial nodes x a mixed half/full-range Gauss-Hermite
velocity set) runs in the HIP kernels of ``csrc/`` behind the C ABI of ``include/lbe.h``;
``lbe`` is its thin Python binding.
"""
from . import workloads  # noqa: F401

"""PHOBIC minimal perfect hashing on AMD Instinct MI355X.

The compute path is the HIP library ``libphobic.so`` (C ABI in ``include/phobic.h``); this package
holds its sources (``csrc/``), the build script (``build_lib``), the ctypes binding (``binding``)
and the seeded input generators shared by tests and benchmark (``synth``).
"""

from .binding import (MPHF, Params, PhobicError, build_str, build_u64, deserialize, params,  # noqa: F401
                      partition_u64)

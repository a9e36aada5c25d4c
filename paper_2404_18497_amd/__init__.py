"""PHOBIC minimal perfect hashing on AMD Instinct MI355X.

The compute path is the HIP library ``libphobic.so`` (C ABI in ``include/phobic.h``); this package
holds its sources (``csrc/``), the build script (``build_lib``), the ctypes binding (``binding``)
and the seeded input generators shared by tests and benchmark (``synth``).
"""

from .binding import (MPHF, BatchKeys, BatchMPHFs, Params, PhobicError, Server, build_batch_u64, build_str,  # noqa: F401
                      build_u64,
                      deserialize, get_search_config, params, partition_u64, query_multi_u64, set_search_config)

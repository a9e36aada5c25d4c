"""ctypes marshalling for the CPU oracle (``phobic_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark, never by the product library. It adds no arithmetic of its own: every function below
converts numpy arrays to pointers and calls the C oracle.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "phobic_oracle.c")
LIB = os.path.join(HERE, "libphobic_oracle.so")

STATUS = {0: "OK", 1: "INVALID", 2: "DUPLICATE", 3: "OOM", 4: "PILOT_OVERFLOW", 5: "DEVICE",
          6: "FORMAT", 7: "CAPACITY"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code} ({STATUS.get(code, '?')})")
        self.code = code


class RefParams(C.Structure):
    _fields_ = [("partition_size", C.c_uint32), ("coding", C.c_uint32), ("lambda_", C.c_double),
                ("alpha_num", C.c_uint32), ("alpha_den", C.c_uint32), ("hash_seed", C.c_uint64),
                ("pilot_limit", C.c_uint64), ("n_compact", C.c_uint32), ("bucket_fn", C.c_uint32)]


BUCKET_FNS = {"optimized": 0, "beta_star": 1, "skew": 2, "uniform": 3}


def build_library(force: bool = False) -> str:
    """Compile the oracle with gcc (it is plain C11 + pthreads)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build_library())
        u64p, u32p, u8p = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint8)
        vp = C.c_void_p
        L.phobic_ref_build_u64.argtypes = [u64p, C.c_uint64, C.POINTER(RefParams), C.c_int, C.POINTER(vp)]
        L.phobic_ref_build_str.argtypes = [u8p, u64p, C.c_uint64, C.POINTER(RefParams), C.c_int, C.POINTER(vp)]
        L.phobic_ref_build_hashes.argtypes = [u64p, u64p, C.c_uint64, C.POINTER(RefParams), C.c_int, C.POINTER(vp)]
        L.phobic_ref_query_u64.argtypes = [vp, u64p, C.c_uint64, u64p]
        L.phobic_ref_query_str.argtypes = [vp, u8p, u64p, C.c_uint64, u64p]
        L.phobic_ref_query_image_u64.argtypes = [u64p, C.c_uint64, u64p, C.c_uint64, u64p]
        L.phobic_ref_query_image_str.argtypes = [u64p, C.c_uint64, u8p, u64p, C.c_uint64, u64p]
        L.phobic_ref_num_words.argtypes = [vp]
        L.phobic_ref_num_words.restype = C.c_uint64
        L.phobic_ref_words.argtypes = [vp]
        L.phobic_ref_words.restype = u64p
        L.phobic_ref_num_partitions.argtypes = [vp]
        L.phobic_ref_num_partitions.restype = C.c_uint64
        L.phobic_ref_num_buckets.argtypes = [vp]
        L.phobic_ref_num_buckets.restype = C.c_uint32
        L.phobic_ref_get_pilots.argtypes = [vp, u32p]
        L.phobic_ref_get_offsets.argtypes = [vp, u64p]
        L.phobic_ref_get_counters.argtypes = [vp, u64p]
        L.phobic_ref_free.argtypes = [vp]
        L.phobic_ref_hash_u64.argtypes = [u64p, C.c_uint64, C.c_uint64, u64p, u64p]
        L.phobic_ref_hash_str.argtypes = [u8p, u64p, C.c_uint64, C.c_uint64, u64p, u64p]
        L.phobic_ref_pos_hash.argtypes = [C.c_uint64] * 4
        L.phobic_ref_pos_hash.restype = C.c_uint64
        L.phobic_ref_mix_a.argtypes = [C.c_uint64]
        L.phobic_ref_mix_a.restype = C.c_uint64
        L.phobic_ref_mix_b.argtypes = [C.c_uint64]
        L.phobic_ref_mix_b.restype = C.c_uint64
        L.phobic_ref_partition_of.argtypes = [C.c_uint64, C.c_uint64]
        L.phobic_ref_partition_of.restype = C.c_uint64
        L.phobic_ref_beta_star.argtypes = [C.c_double]
        L.phobic_ref_beta_star.restype = C.c_double
        L.phobic_ref_beta_eps.argtypes = [C.c_double, C.c_double]
        L.phobic_ref_beta_eps.restype = C.c_double
        L.phobic_ref_epsilon.argtypes = [C.c_double, C.c_uint32]
        L.phobic_ref_epsilon.restype = C.c_double
        L.phobic_ref_bucket_table.argtypes = [C.c_double, C.c_uint32, C.c_uint32, C.c_uint32, u64p]
        L.phobic_ref_bucket_table_fn.argtypes = [C.c_double, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, u64p]
        L.phobic_ref_gamma.argtypes = [C.c_double, C.c_uint32, C.c_double]
        L.phobic_ref_gamma.restype = C.c_double
        L.phobic_ref_bucket_of.argtypes = [C.c_uint64, u64p, C.c_uint32]
        L.phobic_ref_bucket_of.restype = C.c_uint32
        L.phobic_ref_buckets.argtypes = [u64p, C.c_uint64, u64p, C.c_uint32, u32p]
        L.phobic_ref_search_partition.argtypes = [u64p, u64p, C.c_uint64, C.c_uint64, C.POINTER(RefParams), u32p,
                                                  u64p]
        L.phobic_ref_rice_param.argtypes = [C.c_uint64, C.c_uint64]
        L.phobic_ref_rice_param.restype = C.c_uint32
        L.phobic_ref_num_partitions_for.argtypes = [C.c_uint64, C.c_uint32]
        L.phobic_ref_num_partitions_for.restype = C.c_uint64
        L.phobic_ref_num_buckets_for.argtypes = [C.c_uint32, C.c_double]
        L.phobic_ref_num_buckets_for.restype = C.c_uint32
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def params(partition_size=2500, lam=7.0, alpha=(1, 1), coding="rice", hash_seed=0x5EED,
           pilot_limit=0, n_compact=0, bucket_fn="optimized") -> RefParams:
    return RefParams(partition_size, 0 if coding == "rice" else 1, float(lam), alpha[0], alpha[1],
                     hash_seed, pilot_limit, n_compact, BUCKET_FNS[bucket_fn])


class RefMPHF:
    """An oracle-built MPHF (owns the C handle)."""

    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if getattr(self, "h", None):
            lib().phobic_ref_free(self.h)
            self.h = None

    @property
    def K(self) -> int:
        return lib().phobic_ref_num_partitions(self.h)

    @property
    def B(self) -> int:
        return lib().phobic_ref_num_buckets(self.h)

    def image(self) -> np.ndarray:
        n = lib().phobic_ref_num_words(self.h)
        return np.ctypeslib.as_array(lib().phobic_ref_words(self.h), shape=(n,)).copy()

    def size_bits(self) -> int:
        return 64 * lib().phobic_ref_num_words(self.h)

    def pilots(self) -> np.ndarray:
        out = np.zeros(self.K * self.B, dtype=np.uint32)
        lib().phobic_ref_get_pilots(self.h, _p(out, C.c_uint32))
        return out.reshape(self.K, self.B)

    def offsets(self) -> np.ndarray:
        out = np.zeros(self.K + 1, dtype=np.uint64)
        lib().phobic_ref_get_offsets(self.h, _p(out, C.c_uint64))
        return out

    def counters(self) -> dict:
        out = np.zeros(4, dtype=np.uint64)
        lib().phobic_ref_get_counters(self.h, _p(out, C.c_uint64))
        return {"hash_evals": int(out[0]), "slot_probes": int(out[1]), "seeds_tried": int(out[2]),
                "buckets": int(out[3])}

    def query_u64(self, keys: np.ndarray) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(keys.size, dtype=np.uint64)
        lib().phobic_ref_query_u64(self.h, _p(keys, C.c_uint64), keys.size, _p(out, C.c_uint64))
        return out

    def query_str(self, buf: np.ndarray, offs: np.ndarray) -> np.ndarray:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        out = np.zeros(offs.size - 1, dtype=np.uint64)
        lib().phobic_ref_query_str(self.h, _p(buf, C.c_uint8), _p(offs, C.c_uint64), offs.size - 1,
                                   _p(out, C.c_uint64))
        return out


def _finish(st: int, h) -> RefMPHF:
    if st != 0:
        raise OracleError(st)
    return RefMPHF(h)


def build_u64(keys: np.ndarray, prm: RefParams, threads: int = 1) -> RefMPHF:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    h = C.c_void_p()
    st = lib().phobic_ref_build_u64(_p(keys, C.c_uint64), keys.size, C.byref(prm), threads, C.byref(h))
    return _finish(st, h)


def build_str(buf: np.ndarray, offs: np.ndarray, prm: RefParams, threads: int = 1) -> RefMPHF:
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    h = C.c_void_p()
    st = lib().phobic_ref_build_str(_p(buf, C.c_uint8), _p(offs, C.c_uint64), offs.size - 1, C.byref(prm),
                                    threads, C.byref(h))
    return _finish(st, h)


def build_hashes(hi: np.ndarray, lo: np.ndarray, prm: RefParams, threads: int = 1) -> RefMPHF:
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    h = C.c_void_p()
    st = lib().phobic_ref_build_hashes(_p(hi, C.c_uint64), _p(lo, C.c_uint64), hi.size, C.byref(prm), threads,
                                       C.byref(h))
    return _finish(st, h)


def search_partition(hi: np.ndarray, lo: np.ndarray, m: int, prm: RefParams):
    """Pilots (B entries) of one partition with codes (hi, lo) and table size m, plus counters."""
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    B = num_buckets(prm.partition_size, prm.lambda_)
    out = np.zeros(B, dtype=np.uint32)
    cnt = np.zeros(4, dtype=np.uint64)
    st = lib().phobic_ref_search_partition(_p(hi, C.c_uint64), _p(lo, C.c_uint64), hi.size, m, C.byref(prm),
                                           _p(out, C.c_uint32), _p(cnt, C.c_uint64))
    if st != 0:
        raise OracleError(st)
    return out, cnt


def query_image_u64(image: np.ndarray, keys: np.ndarray) -> np.ndarray:
    image = np.ascontiguousarray(image, dtype=np.uint64)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(keys.size, dtype=np.uint64)
    st = lib().phobic_ref_query_image_u64(_p(image, C.c_uint64), image.size, _p(keys, C.c_uint64), keys.size,
                                          _p(out, C.c_uint64))
    if st != 0:
        raise OracleError(st)
    return out


def query_image_str(image: np.ndarray, buf: np.ndarray, offs: np.ndarray) -> np.ndarray:
    image = np.ascontiguousarray(image, dtype=np.uint64)
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    out = np.zeros(offs.size - 1, dtype=np.uint64)
    st = lib().phobic_ref_query_image_str(_p(image, C.c_uint64), image.size, _p(buf, C.c_uint8), _p(offs, C.c_uint64),
                                          offs.size - 1, _p(out, C.c_uint64))
    if st != 0:
        raise OracleError(st)
    return out


def hash_u64(keys: np.ndarray, seed: int):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    hi = np.zeros(keys.size, dtype=np.uint64)
    lo = np.zeros(keys.size, dtype=np.uint64)
    lib().phobic_ref_hash_u64(_p(keys, C.c_uint64), keys.size, seed, _p(hi, C.c_uint64), _p(lo, C.c_uint64))
    return hi, lo


def hash_str(buf: np.ndarray, offs: np.ndarray, seed: int):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    n = offs.size - 1
    hi = np.zeros(n, dtype=np.uint64)
    lo = np.zeros(n, dtype=np.uint64)
    lib().phobic_ref_hash_str(_p(buf, C.c_uint8), _p(offs, C.c_uint64), n, seed, _p(hi, C.c_uint64),
                              _p(lo, C.c_uint64))
    return hi, lo


def bucket_table(lam: float, P: int, alpha=(1, 1), bucket_fn="optimized") -> np.ndarray:
    T = np.zeros(2049, dtype=np.uint64)
    lib().phobic_ref_bucket_table_fn(float(lam), P, alpha[0], alpha[1], BUCKET_FNS[bucket_fn], _p(T, C.c_uint64))
    return T


def gamma(x: float, bucket_fn="optimized", eps: float = 0.0) -> float:
    """The bucket assignment function selected by bucket_fn at x (eps only for "optimized")."""
    return lib().phobic_ref_gamma(float(x), BUCKET_FNS[bucket_fn], float(eps))


def bucket_of(lo: int, T: np.ndarray, B: int) -> int:
    return lib().phobic_ref_bucket_of(lo, _p(T, C.c_uint64), B)


def buckets(lo: np.ndarray, T: np.ndarray, B: int) -> np.ndarray:
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    out = np.zeros(lo.size, dtype=np.uint32)
    lib().phobic_ref_buckets(_p(lo, C.c_uint64), lo.size, _p(T, C.c_uint64), B, _p(out, C.c_uint32))
    return out


def pos_hash(hi: int, lo: int, s: int, m: int) -> int:
    return lib().phobic_ref_pos_hash(hi, lo, s, m)


def partition_of(hi: int, K: int) -> int:
    return lib().phobic_ref_partition_of(hi, K)


def rice_param(total: int, count: int) -> int:
    return lib().phobic_ref_rice_param(total, count)


def beta_star(x: float) -> float:
    return lib().phobic_ref_beta_star(x)


def beta_eps(x: float, eps: float) -> float:
    return lib().phobic_ref_beta_eps(x, eps)


def epsilon(lam: float, P: int) -> float:
    return lib().phobic_ref_epsilon(lam, P)


def num_partitions(n: int, P: int) -> int:
    return lib().phobic_ref_num_partitions_for(n, P)


def num_buckets(P: int, lam: float) -> int:
    return lib().phobic_ref_num_buckets_for(P, lam)


def mix_a(z: int) -> int:
    return lib().phobic_ref_mix_a(z)


def mix_b(z: int) -> int:
    return lib().phobic_ref_mix_b(z)

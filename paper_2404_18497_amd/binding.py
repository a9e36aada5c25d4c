"""ctypes binding of ``libphobic.so`` (declared in ``include/phobic.h``).

Argument marshalling only: torch supplies device memory and the current HIP stream; every step of
building and querying runs in the library's HIP kernels. There is no fallback: if the library is not
built, loading it raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libphobic.so")

OK, E_INVALID, E_DUPLICATE, E_OOM, E_PILOT_OVERFLOW, E_DEVICE, E_FORMAT, E_CAPACITY = range(8)
RICE, COMPACT = 0, 1
BUCKET_FNS = {"optimized": 0, "beta_star": 1, "skew": 2, "uniform": 3}
FLAG_KEEP_PILOTS = 1

EXPORTS = [
    "phobic_params_default", "phobic_build_u64", "phobic_build_str", "phobic_query_u64", "phobic_query_str",
    "phobic_size_bits", "phobic_num_keys", "phobic_num_partitions", "phobic_num_buckets", "phobic_get_pilots",
    "phobic_get_build_info", "phobic_serialize", "phobic_deserialize", "phobic_partition_u64", "phobic_free",
    "phobic_status_str", "phobic_last_error", "phobic_set_search_config", "phobic_get_search_config",
    "phobic_build_batch_u64", "phobic_query_multi_u64", "phobic_query_multi_u64_noalloc",
    "phobic_server_create", "phobic_server_submit_build",
    "phobic_server_submit_query", "phobic_server_poll", "phobic_server_mphf", "phobic_server_release",
    "phobic_server_get_stats", "phobic_server_now", "phobic_server_destroy",
]
REQ_BUILD, REQ_QUERY = 0, 1
NOALLOC_MAX_REQUESTS = 4096


class PhobicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"phobic status {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("partition_size", C.c_uint32), ("coding", C.c_uint32), ("lambda_", C.c_double),
                ("alpha_num", C.c_uint32), ("alpha_den", C.c_uint32), ("hash_seed", C.c_uint64),
                ("pilot_limit", C.c_uint64), ("n_compact", C.c_uint32), ("flags", C.c_uint32),
                ("bucket_function", C.c_uint32), ("reserved", C.c_uint32)]


class SearchConfig(C.Structure):
    _fields_ = [("waves_per_group", C.c_uint32), ("groups_per_cu", C.c_uint32), ("items_per_grab", C.c_uint32),
                ("reserved", C.c_uint32)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("workers", C.c_uint32), ("max_query_batch", C.c_uint32),
                ("max_build_batch", C.c_uint32), ("query_workers", C.c_uint32)]


class RequestResult(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("mphf_id", C.c_uint64), ("n", C.c_uint64), ("status", C.c_int32),
                ("kind", C.c_uint32), ("batch", C.c_uint32), ("reserved", C.c_uint32), ("submit_s", C.c_double),
                ("start_s", C.c_double), ("done_s", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in ["resident_mphfs", "resident_bytes", "reserved_bytes", "peak_bytes",
                                          "query_launches", "build_launches", "completed", "pending"]]


class BuildInfo(C.Structure):
    _fields_ = [("hash_count_ms", C.c_double), ("scan_ms", C.c_double), ("scatter_ms", C.c_double),
                ("bucket_sort_ms", C.c_double), ("search_ms", C.c_double), ("encode_ms", C.c_double),
                ("total_ms", C.c_double), ("max_partition_keys", C.c_uint64), ("max_bucket_keys", C.c_uint32),
                ("partition_path", C.c_uint32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2404_18497_amd.build_lib")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        P = C.POINTER(Params)
        L.phobic_params_default.argtypes = [P]
        L.phobic_params_default.restype = None
        L.phobic_build_u64.argtypes = [vp, u64, P, vp, C.POINTER(vp)]
        L.phobic_build_str.argtypes = [vp, vp, u64, P, vp, C.POINTER(vp)]
        L.phobic_query_u64.argtypes = [vp, vp, u64, vp, vp]
        L.phobic_query_str.argtypes = [vp, vp, vp, u64, vp, vp]
        for name, rt in [("phobic_size_bits", u64), ("phobic_num_keys", u64), ("phobic_num_partitions", u64),
                         ("phobic_num_buckets", u32)]:
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = rt
        L.phobic_get_pilots.argtypes = [vp, vp, u64]
        L.phobic_get_build_info.argtypes = [vp, C.POINTER(BuildInfo)]
        L.phobic_serialize.argtypes = [vp, vp, C.POINTER(u64)]
        L.phobic_deserialize.argtypes = [vp, u64, vp, C.POINTER(vp)]
        L.phobic_partition_u64.argtypes = [vp, u64, P, vp, vp, vp]
        L.phobic_build_batch_u64.argtypes = [C.POINTER(vp), C.POINTER(u64), u32, P, vp, C.POINTER(vp)]
        L.phobic_set_search_config.argtypes = [C.POINTER(SearchConfig)]
        L.phobic_get_search_config.argtypes = [C.POINTER(SearchConfig)]
        L.phobic_query_multi_u64.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(u64), C.POINTER(vp), u32, vp]
        L.phobic_query_multi_u64_noalloc.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(u64), C.POINTER(vp), u32,
                                                     vp]
        L.phobic_server_create.argtypes = [C.POINTER(ServerConfig), P, C.POINTER(vp)]
        L.phobic_server_submit_build.argtypes = [vp, vp, u64, C.POINTER(u64)]
        L.phobic_server_submit_query.argtypes = [vp, u64, vp, u64, vp, C.POINTER(u64)]
        L.phobic_server_poll.argtypes = [vp, C.POINTER(RequestResult), u32, C.POINTER(u32), u32]
        L.phobic_server_mphf.argtypes = [vp, u64]
        L.phobic_server_mphf.restype = vp
        L.phobic_server_release.argtypes = [vp, u64]
        L.phobic_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.phobic_server_now.argtypes = [vp]
        L.phobic_server_now.restype = C.c_double
        L.phobic_server_destroy.argtypes = [vp]
        L.phobic_server_destroy.restype = None
        L.phobic_free.argtypes = [vp]
        L.phobic_free.restype = None
        L.phobic_status_str.argtypes = [C.c_int]
        L.phobic_status_str.restype = C.c_char_p
        L.phobic_last_error.argtypes = []
        L.phobic_last_error.restype = C.c_char_p
        for name in ["phobic_build_u64", "phobic_build_str", "phobic_query_u64", "phobic_query_str",
                     "phobic_get_pilots", "phobic_get_build_info", "phobic_serialize", "phobic_deserialize",
                     "phobic_partition_u64", "phobic_build_batch_u64", "phobic_set_search_config",
                     "phobic_get_search_config", "phobic_query_multi_u64", "phobic_query_multi_u64_noalloc",
                     "phobic_server_create",
                     "phobic_server_submit_build", "phobic_server_submit_query", "phobic_server_poll",
                     "phobic_server_release", "phobic_server_get_stats"]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise PhobicError(code, lib().phobic_last_error().decode(errors="replace"))


def params(partition_size=2500, lam=7.0, alpha=(1, 1), coding="rice", hash_seed=0x5EED, pilot_limit=0,
           keep_pilots=False, n_compact=0, bucket_fn="optimized") -> Params:
    p = Params()
    lib().phobic_params_default(C.byref(p))
    p.partition_size = partition_size
    p.lambda_ = float(lam)
    p.alpha_num, p.alpha_den = alpha
    p.coding = RICE if coding == "rice" else COMPACT
    p.hash_seed = hash_seed
    p.pilot_limit = pilot_limit
    p.n_compact = n_compact
    p.bucket_function = BUCKET_FNS[bucket_fn]
    p.flags = FLAG_KEEP_PILOTS if keep_pilots else 0
    return p


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t) -> C.c_void_p:
    import torch

    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    assert t.dtype in (torch.int64, torch.uint64, torch.uint8), t.dtype
    return C.c_void_p(t.data_ptr())


class MPHF:
    """A device-resident PHOBIC MPHF (owns the library handle unless borrowed from a server)."""

    def __init__(self, handle: C.c_void_p, owned: bool = True):
        self.h = handle
        self.owned = owned

    def close(self):
        if getattr(self, "h", None) and self.owned and _lib is not None:
            _lib.phobic_free(self.h)
        self.h = None

    __del__ = close

    @property
    def n(self) -> int:
        return lib().phobic_num_keys(self.h)

    @property
    def K(self) -> int:
        return lib().phobic_num_partitions(self.h)

    @property
    def B(self) -> int:
        return lib().phobic_num_buckets(self.h)

    def size_bits(self) -> int:
        return lib().phobic_size_bits(self.h)

    def query_u64(self, keys, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
        _check(lib().phobic_query_u64(self.h, _dptr(keys), keys.numel(), _dptr(out), _stream(stream)))
        return out

    def query_str(self, data, offsets, out=None, stream=None):
        import torch

        n = offsets.numel() - 1
        if out is None:
            out = torch.empty(n, dtype=torch.int64, device=data.device)
        _check(lib().phobic_query_str(self.h, _dptr(data), _dptr(offsets), n, _dptr(out), _stream(stream)))
        return out

    def pilots(self) -> np.ndarray:
        out = np.zeros(self.K * self.B, dtype=np.uint32)
        _check(lib().phobic_get_pilots(self.h, out.ctypes.data_as(C.c_void_p), out.size))
        return out.reshape(self.K, self.B)

    def build_info(self) -> dict:
        bi = BuildInfo()
        _check(lib().phobic_get_build_info(self.h, C.byref(bi)))
        return {f: getattr(bi, f) for f, _ in BuildInfo._fields_}

    def serialize(self) -> np.ndarray:
        size = C.c_uint64(0)
        _check(lib().phobic_serialize(self.h, None, C.byref(size)))
        buf = np.zeros(size.value // 8, dtype=np.uint64)
        _check(lib().phobic_serialize(self.h, buf.ctypes.data_as(C.c_void_p), C.byref(size)))
        return buf


def build_u64(keys, prm: Params, stream=None) -> MPHF:
    h = C.c_void_p()
    _check(lib().phobic_build_u64(_dptr(keys), keys.numel(), C.byref(prm), _stream(stream), C.byref(h)))
    return MPHF(h)


def build_str(data, offsets, prm: Params, stream=None) -> MPHF:
    h = C.c_void_p()
    n = offsets.numel() - 1
    _check(lib().phobic_build_str(_dptr(data), _dptr(offsets), n, C.byref(prm), _stream(stream), C.byref(h)))
    return MPHF(h)


class BatchKeys:
    """The key sets of a batched build, checked once, with the host arrays the C-ABI takes (device
    pointers and counts); reusable across builds of the same tensors, which it keeps alive."""

    def __init__(self, key_tensors):
        self.tensors = list(key_tensors)
        self.count = len(self.tensors)
        for t in self.tensors:
            _dptr(t)
        n = max(self.count, 1)
        self.ptrs = (C.c_void_p * n)(*[t.data_ptr() if t.numel() else None for t in self.tensors])
        self.counts = (C.c_uint64 * n)(*[t.numel() for t in self.tensors])


class BatchMPHFs:
    """The handles of a batched build, in order.  Member t's MPHF wrapper is made when it is first
    read and owns its handle from then on; the handles never read are freed with this object."""

    def __init__(self, outs, count: int):
        self._outs = outs
        self._count = count
        self._made = [None] * count

    def __len__(self) -> int:
        return self._count

    def __getitem__(self, t):
        if isinstance(t, slice):
            return [self[i] for i in range(*t.indices(self._count))]
        if t < 0:
            t += self._count
        if not 0 <= t < self._count:
            raise IndexError(t)
        if self._made[t] is None:
            self._made[t] = MPHF(C.c_void_p(self._outs[t]))
        return self._made[t]

    def __iter__(self):
        return (self[t] for t in range(self._count))

    def close(self):
        made = getattr(self, "_made", None)
        if made is None or _lib is None:
            return
        for t, m in enumerate(made):  # wrappers already made free their own handles
            if m is None and self._outs[t]:
                _lib.phobic_free(C.c_void_p(self._outs[t]))
        self._made = None

    __del__ = close


def build_batch_u64(key_tensors, prm: Params, stream=None) -> BatchMPHFs:
    """Builds one MPHF per key set in a single batched pass; returns the handles in order.
    key_tensors: a list of device tensors or a BatchKeys made from one (checked once, reusable)."""
    bk = key_tensors if isinstance(key_tensors, BatchKeys) else BatchKeys(key_tensors)
    outs = (C.c_void_p * max(bk.count, 1))()
    _check(lib().phobic_build_batch_u64(bk.ptrs, bk.counts, bk.count, C.byref(prm), _stream(stream), outs))
    return BatchMPHFs(outs, bk.count)


def query_multi_u64(handles, key_tensors, out_tensors, stream=None, noalloc=False):
    """One launch for several (MPHF, keys) requests; out_tensors receive the positions. noalloc=True
    calls the allocation-free entry point (at most NOALLOC_MAX_REQUESTS requests)."""
    count = len(handles)
    hs = (C.c_void_p * max(count, 1))(*[h.h.value if isinstance(h.h, C.c_void_p) else h.h for h in handles])
    ks = (C.c_void_p * max(count, 1))(*[_dptr(k).value for k in key_tensors])
    ns = (C.c_uint64 * max(count, 1))(*[k.numel() for k in key_tensors])
    os_ = (C.c_void_p * max(count, 1))(*[_dptr(o).value for o in out_tensors])
    fn = lib().phobic_query_multi_u64_noalloc if noalloc else lib().phobic_query_multi_u64
    _check(fn(hs, ks, ns, os_, count, _stream(stream)))


class Server:
    """The library's serving loop (resident MPHFs, HBM-budget admission, continuous batching).

    Keeps a reference to every tensor of a request until its completion is polled."""

    def __init__(self, prm: Params, budget_bytes: int, workers: int = 4, max_query_batch: int = 32,
                 max_build_batch: int = 8, query_workers: int = 0):
        cfg = ServerConfig(budget_bytes, workers, max_query_batch, max_build_batch, query_workers)
        self.s = C.c_void_p()
        _check(lib().phobic_server_create(C.byref(cfg), C.byref(prm), C.byref(self.s)))
        self._live = {}

    def submit_build(self, keys) -> int:
        rid = C.c_uint64()
        _check(lib().phobic_server_submit_build(self.s, _dptr(keys), keys.numel(), C.byref(rid)))
        self._live[rid.value] = (keys,)
        return rid.value

    def submit_query(self, mphf_id: int, keys, out) -> int:
        rid = C.c_uint64()
        _check(lib().phobic_server_submit_query(self.s, mphf_id, _dptr(keys), keys.numel(), _dptr(out),
                                                C.byref(rid)))
        self._live[rid.value] = (keys, out)
        return rid.value

    def poll(self, cap: int = 1024, wait_ms: int = 0) -> list:
        buf = (RequestResult * cap)()
        got = C.c_uint32()
        _check(lib().phobic_server_poll(self.s, buf, cap, C.byref(got), wait_ms))
        out = []
        for i in range(got.value):
            r = buf[i]
            self._live.pop(r.request_id, None)
            out.append({"request_id": r.request_id, "mphf_id": r.mphf_id, "n": r.n, "status": r.status,
                        "kind": "build" if r.kind == REQ_BUILD else "query", "batch": r.batch,
                        "submit_s": r.submit_s, "start_s": r.start_s, "done_s": r.done_s})
        return out

    def mphf(self, mphf_id: int):
        p = lib().phobic_server_mphf(self.s, mphf_id)
        return MPHF(C.c_void_p(p), owned=False) if p else None

    def release(self, mphf_id: int):
        _check(lib().phobic_server_release(self.s, mphf_id))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().phobic_server_get_stats(self.s, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def now(self) -> float:
        return lib().phobic_server_now(self.s)

    def close(self):
        if getattr(self, "s", None) and _lib is not None:
            _lib.phobic_server_destroy(self.s)
        self.s = None
        self._live = {}

    __del__ = close


def set_search_config(waves_per_group=4, groups_per_cu=0, items_per_grab=1):
    cfg = SearchConfig(waves_per_group, groups_per_cu, items_per_grab, 0)
    _check(lib().phobic_set_search_config(C.byref(cfg)))


def get_search_config() -> dict:
    cfg = SearchConfig()
    _check(lib().phobic_get_search_config(C.byref(cfg)))
    return {"waves_per_group": cfg.waves_per_group, "groups_per_cu": cfg.groups_per_cu,
            "items_per_grab": cfg.items_per_grab}


def deserialize(image: np.ndarray, stream=None) -> MPHF:
    image = np.ascontiguousarray(image, dtype=np.uint64)
    h = C.c_void_p()
    _check(lib().phobic_deserialize(image.ctypes.data_as(C.c_void_p), image.nbytes, _stream(stream), C.byref(h)))
    return MPHF(h)


def partition_u64(keys, prm: Params, stream=None):
    """Hashing and partitioning only: (offsets[K+1], codes[n, 2]) as device tensors."""
    import torch

    n = keys.numel()
    K = max(1, -(-n // prm.partition_size))
    offs = torch.empty(K + 1, dtype=torch.int64, device=keys.device)
    codes = torch.empty(max(n, 1), 2, dtype=torch.int64, device=keys.device)
    _check(lib().phobic_partition_u64(_dptr(keys), n, C.byref(prm), _stream(stream), _dptr(offs), _dptr(codes)))
    return offs, codes[:n]

"""CPU-side checks of the boundary: the library loads and exports every entry point its header
declares; host-only calls behave (no device work is issued here)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phobic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phobic_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2404_18497_amd import binding

    return binding.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["phobic_build_u64", "phobic_build_str", "phobic_query_u64", "phobic_query_str", "phobic_size_bits",
                 "phobic_serialize", "phobic_deserialize", "phobic_free"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2404_18497_amd import binding

    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(binding.EXPORTS)


def test_host_only_calls(lib):
    from paper_2404_18497_amd import binding

    p = binding.params()
    assert p.partition_size == 2500 and p.lambda_ == 7.0 and p.alpha_num == p.alpha_den == 1
    assert lib.phobic_status_str(2) == b"duplicate keys"
    assert lib.phobic_size_bits(None) == 0
    # malformed images are rejected on the host before any device call
    bad = (C.c_uint64 * 30)()
    h = C.c_void_p()
    assert lib.phobic_deserialize(bad, 8 * 30, None, C.byref(h)) == binding.E_FORMAT
    assert not h.value
    assert b"magic" in lib.phobic_last_error()
    # invalid parameters are rejected before any device call
    q = binding.params(lam=0.0)
    assert lib.phobic_build_u64(None, 10, C.byref(q), None, C.byref(h)) == binding.E_INVALID
    q = binding.params(alpha=(3, 2))
    assert lib.phobic_build_u64(None, 10, C.byref(q), None, C.byref(h)) == binding.E_INVALID
    q = binding.params(pilot_limit=1 << 33)
    assert lib.phobic_build_u64(None, 10, C.byref(q), None, C.byref(h)) == binding.E_INVALID


def test_header_and_oracle_agree_on_status_codes():
    import oracle

    text = open(HEADER).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"PHOBIC_(E_[A-Z_]+|OK)\s*=\s*(\d+)", text)}
    for code, name in oracle.STATUS.items():
        key = "OK" if name == "OK" else "E_" + name
        assert codes[key] == code


def test_search_config_validation(lib):
    from paper_2404_18497_amd import binding

    before = binding.get_search_config()
    for bad in [dict(waves_per_group=3), dict(waves_per_group=16), dict(groups_per_cu=65),
                dict(groups_per_cu=2, items_per_grab=0)]:
        with pytest.raises(binding.PhobicError):
            binding.set_search_config(**bad)
    binding.set_search_config(waves_per_group=2, groups_per_cu=4, items_per_grab=8)
    assert binding.get_search_config() == {"waves_per_group": 2, "groups_per_cu": 4, "items_per_grab": 8}
    binding.set_search_config(**before)


def test_batch_rejects_bad_arguments_on_host(lib):
    from paper_2404_18497_amd import binding

    outs = (C.c_void_p * 2)()
    ptrs = (C.c_void_p * 2)(None, None)
    counts = (C.c_uint64 * 2)(5, 0)
    p = binding.params()
    assert lib.phobic_build_batch_u64(ptrs, counts, 2, C.byref(p), None, outs) == binding.E_INVALID
    q = binding.params(alpha=(99, 100))
    counts0 = (C.c_uint64 * 2)(0, 0)
    assert lib.phobic_build_batch_u64(ptrs, counts0, 2, C.byref(q), None, outs) == binding.E_INVALID
    assert not outs[0] and not outs[1]


def test_server_config_rejected_on_host():
    from paper_2404_18497_amd import binding

    p = binding.params()
    for bad in [dict(workers=0), dict(workers=2, query_workers=2), dict(max_query_batch=0), dict(max_build_batch=0)]:
        kw = dict(workers=4, max_query_batch=8, max_build_batch=4, query_workers=0) | bad
        with pytest.raises(binding.PhobicError) as e:
            binding.Server(p, budget_bytes=1 << 30, **kw)
        assert e.value.code == binding.E_INVALID
    with pytest.raises(binding.PhobicError):
        binding.Server(p, budget_bytes=0)


def test_batch_handles_are_made_on_first_use(monkeypatch):
    """The batch result makes a member's wrapper when it is first read, keeps it, and frees only the
    handles never handed out (here stand-in handle values and a recording free, no device work)."""
    from paper_2404_18497_amd import binding

    freed = []

    class FakeLib:
        def phobic_free(self, h):
            freed.append(h.value)

    monkeypatch.setattr(binding, "_lib", FakeLib())
    outs = (C.c_void_p * 4)(0x1000, 0x2000, 0x3000, 0x4000)
    b = binding.BatchMPHFs(outs, 4)
    assert len(b) == 4
    m1 = b[1]
    assert b[1] is m1 and m1.h.value == 0x2000
    assert [m.h.value for m in b[-2:]] == [0x3000, 0x4000]
    with pytest.raises(IndexError):
        b[4]
    m1.owned = False  # keep the stand-in handle away from the recording free at garbage collection
    for t in (2, 3):
        b[t].owned = False
    b.close()
    assert freed == [0x1000]  # only member 0 was never handed out
    b.close()  # a second close frees nothing more
    assert freed == [0x1000]

"""The pilot-search kernel's logic run on the CPU against the oracle, with bounds checks.

`tests/emu/search_emu.cpp` compiles `search_partition` from the library's search.hip with g++,
against a host stand-in of the HIP runtime that runs one 64-lane wavefront as coroutines, and with
AddressSanitizer over the wavefront's LDS block (exactly the size the library gives it) and the
global arrays.  Each case feeds one partition, in the processing order the bucket sort produces
(buckets by size descending, then index descending), and compares the pilots with the oracle's
search of the same codes (Sec. 4, Sec. 4.2): the kernel's single-pass, multi-pass and wide paths,
minimal and non-minimal tables, and the duplicate and pilot-limit errors.  No GPU is used; this
checks the search logic and its LDS layout before any device run.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2404_18497_amd import binding, synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# EMU_SEARCH_SRC: check another copy of search.hip (a change in progress) with the same cases
SEARCH_SRC = os.environ.get("EMU_SEARCH_SRC", os.path.join(ROOT, "paper_2404_18497_amd", "csrc", "search.hip"))
M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("emu") / "search_emu")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-Wno-attributes",
           "-I", os.path.join(HERE, "emu"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2404_18497_amd", "csrc"), f'-DSEARCH_SRC="{SEARCH_SRC}"',
           "-x", "c++", os.path.join(HERE, "emu", "search_emu.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _mix_b(k):
    # the library's fingerprint mixer (MurmurHash3 fmix64), for the fingerprints the kernel reads
    k ^= k >> 33
    k = (k * 0xFF51AFD7ED558CCD) & M64
    k ^= k >> 33
    k = (k * 0xC4CEB9FE1A85EC53) & M64
    return k ^ (k >> 33)


def _partition(P, lam, j, seed=11, nparts=4, dup=False):
    keys = synth.u64_keys(P * nparts, seed)
    if dup:
        keys = np.concatenate([keys, keys[:1]])
    hi, lo = oracle.hash_u64(keys, 0x5EED)
    K = oracle.num_partitions(keys.size, P)
    part = np.array([(int(h) * K) >> 64 for h in hi])
    sel = np.nonzero(part == (int(part[-1]) if dup else j))[0]
    return hi[sel], lo[sel]


def _run(emu, tmp_path, mode, hi, lo, m, prm, limit):
    B = oracle.num_buckets(prm.partition_size, prm.lambda_)
    T = oracle.bucket_table(prm.lambda_, prm.partition_size, (prm.alpha_num, prm.alpha_den))
    b = oracle.buckets(lo, T, B)
    sz = np.bincount(b, minlength=B)
    order = sorted((i for i in range(B) if sz[i]), key=lambda i: (-int(sz[i]), -i))
    fps, ent = [], []
    for i in order:
        for k in np.nonzero(b == i)[0]:
            fps.append(int(lo[k]) ^ _mix_b(int(hi[k])))
        ent.append((int(sz[i]) << 16) | i)
    fi, fo = str(tmp_path / "in"), str(tmp_path / "out")
    with open(fi, "wb") as f:
        np.array([m, limit, B, len(fps), len(ent)], dtype=np.uint64).tofile(f)
        np.array(fps, dtype=np.uint64).tofile(f)
        np.array(ent, dtype=np.uint32).tofile(f)
    r = subprocess.run([emu, str(mode), fi, fo], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    out = np.fromfile(fo, dtype=np.uint32)
    return out[:B], int(out[B])


@pytest.mark.parametrize("lam,j", [(5.0, 0), (7.0, 1), (9.0, 2), (11.0, 3)])
def test_single_pass_matches_oracle(emu, tmp_path, lam, j):
    prm = oracle.params(lam=lam)
    hi, lo = _partition(2500, lam, j)
    want, _ = oracle.search_partition(hi, lo, hi.size, prm)
    got, err = _run(emu, tmp_path, 0, hi, lo, hi.size, prm, 0xFFFFFFFF)
    assert err == 0 and np.array_equal(got, want)


@pytest.mark.parametrize("mode", [1, 2])
def test_multi_pass_and_wide_match_oracle(emu, tmp_path, mode):
    prm = oracle.params(partition_size=10_000, lam=7.0)
    hi, lo = _partition(10_000, 7.0, 0, nparts=2)
    want, _ = oracle.search_partition(hi, lo, hi.size, prm)
    got, err = _run(emu, tmp_path, mode, hi, lo, hi.size, prm, 0xFFFFFFFF)
    assert err == 0 and np.array_equal(got, want)


def test_nonminimal_table_matches_oracle(emu, tmp_path):
    prm = oracle.params(lam=7.0, alpha=(9, 10))
    hi, lo = _partition(2500, 7.0, 0)
    m = -(-hi.size * 10 // 9)
    want, _ = oracle.search_partition(hi, lo, m, prm)
    got, err = _run(emu, tmp_path, 0, hi, lo, m, prm, 0xFFFFFFFF)
    assert err == 0 and np.array_equal(got, want)


def test_duplicate_key_is_reported(emu, tmp_path):
    prm = oracle.params(lam=7.0)
    hi, lo = _partition(2500, 7.0, 0, dup=True)
    with pytest.raises(oracle.OracleError) as e:
        oracle.search_partition(hi, lo, hi.size, prm)
    assert e.value.code == binding.E_DUPLICATE
    _, err = _run(emu, tmp_path, 0, hi, lo, hi.size, prm, 0xFFFFFFFF)
    assert err & (1 << binding.E_DUPLICATE)


def test_pilot_limit_is_reported(emu, tmp_path):
    hi, lo = _partition(2500, 9.0, 0)
    limit = hi.size // 2  # seed 0 only, and not even all of its displacements
    prm = oracle.params(lam=9.0, pilot_limit=limit)
    with pytest.raises(oracle.OracleError) as e:
        oracle.search_partition(hi, lo, hi.size, prm)
    assert e.value.code == binding.E_PILOT_OVERFLOW
    _, err = _run(emu, tmp_path, 0, hi, lo, hi.size, prm, limit)
    assert err & (1 << binding.E_PILOT_OVERFLOW)


@pytest.mark.parametrize("lam,j", [(9.0, 1), (11.0, 0)])
def test_pilot_limit_boundary_matches_oracle(emu, tmp_path, lam, j):
    # limits at, just below and just above the largest pilot of a small bucket (2 .. 24 keys): the
    # seed that reaches the limit and the last displacement allowed with it decide the outcome
    hi, lo = _partition(2500, lam, j)
    prm = oracle.params(lam=lam)
    pil, _ = oracle.search_partition(hi, lo, hi.size, prm)
    B = oracle.num_buckets(prm.partition_size, lam)
    sz = np.bincount(oracle.buckets(lo, oracle.bucket_table(lam, 2500), B), minlength=B)
    small = (sz >= 2) & (sz <= 24)
    top = int(pil[small].max())
    assert top >= hi.size  # the bucket needed a seed past 0
    for limit in (top - 1, top, top + 1):
        p = oracle.params(lam=lam, pilot_limit=limit)
        try:
            want, _ = oracle.search_partition(hi, lo, hi.size, p)
            code = 0
        except oracle.OracleError as e:
            want, code = None, e.code
        got, err = _run(emu, tmp_path, 0, hi, lo, hi.size, p, limit)
        if code == 0:
            assert err == 0 and np.array_equal(got, want), limit
        else:
            assert err & (1 << code), (limit, err)

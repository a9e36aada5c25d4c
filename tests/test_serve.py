"""Serving loop and multi-request queries on the GPU: results are the same alone and in the mix.

A request served alone (one worker, no batching, submitted only after the previous one completed)
and the same request served in a mix (several workers, queries coalesced into one launch, builds
coalesced into batched builds, everything submitted at once) must give identical MPHF images and
identical positions, and both must equal the oracle's image and positions word for word.
"""

import numpy as np
import pytest

import oracle
from paper_2404_18497_amd import binding, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def test_query_multi_matches_single_queries(torch):
    # the last MPHF has 1667 buckets per partition (P = 10000), beyond what a workgroup stages in LDS
    prms = [(2500, 6.0)] * 4 + [(10_000, 6.0)]
    sets = [synth.u64_keys(n, 40 + n) for n in (1000, 50_000, 7, 250_000, 30_000)]
    hs = [binding.build_u64(_dev(torch, k), binding.params(partition_size=P, lam=lam))
          for k, (P, lam) in zip(sets, prms)]
    assert hs[-1].B > 1024
    empty = binding.build_u64(_dev(torch, np.zeros(0, np.uint64)), binding.params(lam=6.0))
    rng = np.random.default_rng(3)
    reqs = []
    for r in range(16):
        t = int(rng.integers(0, len(sets)))
        q = sets[t][rng.integers(0, sets[t].size, int(rng.integers(0, 30_000)))]
        reqs.append((t, _dev(torch, q)))
    # keys of a non-empty set against the empty MPHF: every position is 0, as for a single query
    stray = _dev(torch, sets[1][:5000])
    handles = [hs[t] for t, _ in reqs] + [empty]
    keys = [q for _, q in reqs] + [stray]
    outs = [torch.empty(q.numel(), dtype=torch.int64, device="cuda") for q in keys]
    binding.query_multi_u64(handles, keys, outs)
    for h, q, o in zip(handles, keys, outs):
        assert torch.equal(o, h.query_u64(q))
    assert int(outs[-1].abs().sum()) == 0
    # and against the oracle's positions for the same key sets
    refs = [oracle.build_u64(k, oracle.params(partition_size=P, lam=lam), threads=8) for k, (P, lam) in zip(sets, prms)]
    for (t, q), o in zip(reqs, outs):
        qh = q.cpu().numpy().view(np.uint64)
        assert np.array_equal(o.cpu().numpy().view(np.uint64), refs[t].query_u64(qh))


def _trace(seed, nbuild=10, nquery=60):
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in np.clip(rng.lognormal(np.log(20_000), 1.2, nbuild), 1, 400_000)]
    keysets = [synth.u64_keys(n, 7000 + i) for i, n in enumerate(sizes)]
    queries = []
    for q in range(nquery):
        b = int(rng.integers(0, nbuild))
        m = int(rng.integers(1, 20_000))
        queries.append((b, keysets[b][rng.integers(0, keysets[b].size, m)]))
    return keysets, queries


def _run(torch, keysets, queries, workers, qb, bb, alone, query_workers=0):
    prm = binding.params(lam=7.0)
    srv = binding.Server(prm, budget_bytes=8 << 30, workers=workers, max_query_batch=qb, max_build_batch=bb,
                         query_workers=query_workers)
    dk = [_dev(torch, k) for k in keysets]
    dq = [(b, _dev(torch, q)) for b, q in queries]
    outs = [torch.full((q.numel(),), -1, dtype=torch.int64, device="cuda") for _, q in dq]
    ids, results = [], {}

    def drain(block):
        for r in srv.poll(wait_ms=200 if block else 0):
            results[r["request_id"]] = r

    for k in dk:
        ids.append(srv.submit_build(k))
        if alone:
            while ids[-1] not in results:
                drain(True)
    qids = []
    for (b, q), o in zip(dq, outs):
        qids.append(srv.submit_query(ids[b], q, o))
        if alone:
            while qids[-1] not in results:
                drain(True)
    while len(results) < len(ids) + len(qids):
        drain(True)
    assert all(results[i]["status"] == 0 for i in ids + qids)
    images = [srv.mphf(i).serialize() for i in ids]
    pos = [o.cpu().numpy() for o in outs]
    batches = max(r["batch"] for r in results.values())
    stats = srv.stats()
    srv.close()
    return images, pos, batches, stats


def test_server_same_alone_and_in_the_mix(torch):
    keysets, queries = _trace(1)
    _say("alone")
    img_a, pos_a, batch_a, _ = _run(torch, keysets, queries, workers=1, qb=1, bb=1, alone=True)
    _say("mix")
    img_m, pos_m, batch_m, stats = _run(torch, keysets, queries, workers=4, qb=16, bb=4, alone=False,
                                        query_workers=1)
    assert batch_a == 1 and batch_m > 1  # the mix really batched
    refs = [oracle.build_u64(k, oracle.params(lam=7.0), threads=8) for k in keysets]
    for t, (r, a, m) in enumerate(zip(refs, img_a, img_m)):
        want = r.image()
        assert np.array_equal(a, want), f"build {t} alone differs from the oracle"
        assert np.array_equal(m, want), f"build {t} in the mix differs from the oracle"
    for x, ((b, q), a, m) in enumerate(zip(queries, pos_a, pos_m)):
        want = refs[b].query_u64(q)
        assert np.array_equal(a.view(np.uint64), want), f"query {x} alone differs from the oracle"
        assert np.array_equal(m.view(np.uint64), want), f"query {x} in the mix differs from the oracle"
    assert stats["resident_mphfs"] == len(keysets)


def test_server_budget_admission(torch):
    prm = binding.params(lam=7.0)
    keys = [_dev(torch, synth.u64_keys(200_000, 60 + i)) for i in range(4)]
    est = 32 * 200_000 + (64 << 20)
    # room for exactly one build in flight: all succeed, never two at once
    srv = binding.Server(prm, budget_bytes=est + est // 2, workers=4, max_query_batch=8, max_build_batch=4)
    ids = [srv.submit_build(k) for k in keys]
    got = {}
    while len(got) < len(ids):
        for r in srv.poll(wait_ms=200):
            got[r["request_id"]] = r
    assert all(got[i]["status"] == 0 for i in ids)
    st = srv.stats()
    assert st["peak_bytes"] <= est + est // 2 and st["build_launches"] == 4
    # a build that can never fit is refused at once
    big = srv.submit_build(_dev(torch, synth.u64_keys(3_000_000, 99)))
    r = srv.poll(wait_ms=1000)
    assert r and r[0]["request_id"] == big and r[0]["status"] == binding.E_OOM
    with pytest.raises(binding.PhobicError):
        srv.submit_query(big, keys[0], torch.empty(200_000, dtype=torch.int64, device="cuda"))
    srv.release(ids[0])
    assert srv.stats()["resident_mphfs"] == 3
    with pytest.raises(binding.PhobicError):
        srv.submit_query(ids[0], keys[0], torch.empty(200_000, dtype=torch.int64, device="cuda"))
    srv.close()

"""The allocation-free multi-request query (phobic_query_multi_u64_noalloc) against the allocating
one (phobic_query_multi_u64) through the C ABI: identical positions on two calls in a row, the second
with fewer and smaller requests; more requests than the fixed table holds are refused."""

import numpy as np
import pytest

from paper_2404_18497_amd import binding, synth

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def test_noalloc_query_matches_the_allocating_entry_point():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    prm = binding.params(lam=7.0)
    sets = [synth.u64_keys(n, 70 + i) for i, n in enumerate((120_000, 5_000, 37, 400_000))]
    hs = [binding.build_u64(_dev(torch, k), prm) for k in sets]
    rng = np.random.default_rng(12)
    for call, (nreq, most) in enumerate([(40, 200_000), (7, 3_000)]):
        reqs = []
        for _ in range(nreq):
            t = int(rng.integers(0, len(sets)))
            reqs.append((t, _dev(torch, sets[t][rng.integers(0, sets[t].size, int(rng.integers(0, most)))])))
        a = [torch.full((q.numel(),), -1, dtype=torch.int64, device="cuda") for _, q in reqs]
        b = [torch.full((q.numel(),), -2, dtype=torch.int64, device="cuda") for _, q in reqs]
        binding.query_multi_u64([hs[t] for t, _ in reqs], [q for _, q in reqs], a)
        binding.query_multi_u64([hs[t] for t, _ in reqs], [q for _, q in reqs], b, noalloc=True)
        torch.cuda.synchronize()
        for r, (x, y) in enumerate(zip(a, b)):
            assert torch.equal(x, y), f"call {call}, request {r}"
    # more requests than the table holds: refused, nothing written
    n = binding.NOALLOC_MAX_REQUESTS + 1
    q = _dev(torch, sets[2])
    outs = [torch.full((q.numel(),), -3, dtype=torch.int64, device="cuda") for _ in range(n)]
    with pytest.raises(binding.PhobicError) as e:
        binding.query_multi_u64([hs[2]] * n, [q] * n, outs, noalloc=True)
    assert e.value.code == binding.E_INVALID
    torch.cuda.synchronize()
    assert all(int(o.max()) == -3 for o in outs[:3])

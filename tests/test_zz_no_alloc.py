"""The allocation-free sort entry point (ems_sort_keys_noalloc) against the
allocating one (ems_debug_sort): bit-identical permutations on two calls in a
row, the second with a smaller input (the fixed scratch array keeps the first
call's contents, which must not leak into the second), and the size limit
rejected with CAPACITY before any launch."""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import session_for

pytestmark = pytest.mark.gpu


def test_noalloc_sort_equals_allocating_sort_two_calls_then_smaller():
    import torch

    from paper_2503_17608_amd import emstep
    w = workloads.small_electron_showers(1)
    s = session_for(w, n_slots=1024)
    rng = np.random.default_rng(77)
    stream = s.stream
    for n, policy, nb in ((3_000_017, "radix", 128), (100_003, "partition", 16), (4097, "radix", 128)):
        keys = rng.integers(0, nb, n).astype(np.uint8)
        ref = s.sort(keys, policy)
        assert np.array_equal(ref, np.argsort(keys, kind="stable").astype(np.uint32))
        dk = torch.from_numpy(keys).to("cuda")
        dp = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            s.sort_device(dk, dp, policy)
        stream.synchronize()
        got = dp.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), (n, policy)
    # the size limit is checked before any device work
    big = torch.zeros((1 << 23) + 1, dtype=torch.uint8, device="cuda")
    outp = torch.empty((1 << 23) + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(emstep.EmsError) as e:
        s.sort_device(big, outp, "partition")
    assert e.value.status == emstep.ERR_CAPACITY
    # the largest size still runs, and equals numpy's stable sort
    n = 1 << 23
    keys = rng.integers(0, 16, n).astype(np.uint8)
    dk = torch.from_numpy(keys).to("cuda")
    dp = torch.empty(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    s.sort_device(dk, dp, "partition")
    stream.synchronize()
    assert np.array_equal(dp.cpu().numpy().view(np.uint32), np.argsort(keys, kind="stable").astype(np.uint32))
    s.close()

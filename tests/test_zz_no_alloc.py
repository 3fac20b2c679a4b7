"""The allocation-free scan (txs_exclusive_scan_noalloc) against the scan with a
caller workspace (txs_exclusive_scan): bit for bit, on two calls in a row, the
second on a smaller input, both through the C ABI."""
import numpy as np
import pytest
import torch

import scenes
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _counts(seed, n):
    g = scenes.rng(seed)
    c = g.integers(0, 700, n).astype(np.int32)
    c[g.random(n) < 0.3] = 0
    return c


def test_noalloc_scan_matches_workspace_scan_twice(gpu_lib):
    assert gpu_lib.exclusive_scan_noalloc_max_rays() == 1 << 26
    for seed, n in ((31, (1 << 20) + 4099), (32, 5001), (33, 0)):
        counts = dev(_counts(seed, n))
        ref_info, ref_total = gpu_lib.exclusive_scan(counts)
        info = torch.full((n, 2), -7, dtype=torch.int32, device="cuda")
        total = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        gpu_lib.exclusive_scan_noalloc(counts, info, total)
        torch.cuda.synchronize()
        assert int(total.item()) == int(ref_total.item())
        assert torch.equal(info, ref_info)
        # and the exact sums, independently of either scan
        c = host(counts).astype(np.int64)
        assert int(total.item()) == int(c.sum())
        if n:
            assert np.array_equal(host(info)[:, 0], np.concatenate([[0], np.cumsum(c)[:-1]]))


def test_noalloc_scan_refuses_sizes_beyond_its_scratch(gpu_lib):
    n = (1 << 26) + 1
    counts = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(gpu_lib.TxsError) as e:
        gpu_lib.exclusive_scan_noalloc(counts, info, total)
    assert e.value.status == gpu_lib.TXS_ECAPACITY

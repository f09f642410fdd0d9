"""The tree build's radix sort and exclusive scan (hand-written, deterministic) through the
C ABI against numpy: stable order bit for bit, ragged tiles, several scan levels."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,end_bit", [(1, 3), (2047, 1), (2049, 7), (300_001, 21), (1_000_000, 24),
                                       (70_000, 32)])
def test_radix_sort_is_stable_sort(n, end_bit):
    import torch
    from paper_1902_05875_amd import api
    rng = np.random.default_rng(n + end_bit)
    hi = 1 << end_bit
    # many repeated keys (leaf keys repeat), values = original positions
    k = rng.integers(0, min(hi, max(2, n // 3)), n, dtype=np.uint64) * (hi // min(hi, max(2, n // 3)))
    k = (k % hi).astype(np.uint32)
    keys = torch.from_numpy(k.view(np.int32).copy()).cuda()
    vals = torch.arange(n, dtype=torch.int32).cuda()
    api.radix_sort(keys, vals, end_bit)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), k[order])
    assert np.array_equal(vals.cpu().numpy(), order.astype(np.int32))


@pytest.mark.parametrize("n", [1, 2048, 2049, 100_000, 5_000_000])
def test_exclusive_scan(n):
    import torch
    from paper_1902_05875_amd import api
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1 << 12, n).astype(np.uint32)
    if n > 1000:
        x[::997] = 0xFFFFFFF0  # wrapping sums
    t = torch.from_numpy(x.view(np.int32).copy()).cuda()
    out = torch.empty_like(t)
    api.exclusive_scan(t, out)
    ref = np.zeros(n, np.uint64)
    ref[1:] = np.cumsum(x.astype(np.uint64))[:-1]
    assert np.array_equal(out.cpu().numpy().view(np.uint32), (ref % (1 << 32)).astype(np.uint32))
    api.exclusive_scan(t, t)  # in place
    assert np.array_equal(t.cpu().numpy().view(np.uint32), (ref % (1 << 32)).astype(np.uint32))

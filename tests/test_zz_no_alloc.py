"""The network forward pass that allocates nothing (fixed device workspace) against
tefmm_mlp_forward, through the C ABI: bitwise equal on two calls in a row, the second
with fewer rows, and the row limit rejected on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DIMS = (3, 128, 4, 240)


def _net(seed):
    from paper_1902_05875_amd import api
    net = api.MLP(*DIMS, seed=seed)
    rng = np.random.default_rng(seed)
    th = net.get_params()
    th += rng.normal(scale=0.05, size=th.shape).astype(np.float32)  # non-zero biases too
    net.set_params(th)
    return net


@pytest.mark.parametrize("split", [0, 1])
def test_noalloc_forward_matches_forward(split):
    """Both product forms: one BF16 MFMA per product, and BF16 hi + lo operand pairs."""
    import torch
    from paper_1902_05875_amd import api
    net = _net(3)
    net.set_split(split)
    rng = np.random.default_rng(7)
    limit = api.lib().tefmm_mlp_forward_noalloc  # exported
    assert limit is not None
    for n in (20_011, 1_237):  # second call smaller: stale rows of the first stay in the workspace
        x = torch.from_numpy(rng.uniform(-1, 1, size=(n, DIMS[0]))).float().cuda()
        ref = net.forward(x)
        y = torch.full((n, DIMS[3]), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert torch.equal(y, ref), float((y - ref).abs().max())
    net.close()


def test_noalloc_forward_rejects_too_many_rows():
    import torch
    from paper_1902_05875_amd import api
    net = _net(4)
    max_rows = (32 << 20) // (8 * DIMS[1])
    x = torch.zeros(max_rows + 1, DIMS[0], dtype=torch.float32, device="cuda")
    y = torch.zeros(max_rows + 1, DIMS[3], dtype=torch.float32, device="cuda")
    with pytest.raises(api.TefmmError) as ei:
        net.forward_noalloc(x, y)
    assert "rows per call" in str(ei.value)
    # exactly the limit is accepted
    net.forward_noalloc(x[:max_rows], y[:max_rows])
    torch.cuda.synchronize()
    assert torch.equal(y[:max_rows], net.forward(x[:max_rows]))
    net.close()

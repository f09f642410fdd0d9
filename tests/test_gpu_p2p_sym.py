"""Near field with each pair of particles in different leaves evaluated once (the
kernel value applied in both directions) against the kernel that evaluates every
ordered pair on its own: same pairs, same arithmetic per pair, different sums.  FP32
(the default near field of the mixed mode) and FP64 (chosen by p2p_targets > 0)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K3 = (0.8, 1.5, 2.0)
D3 = (0.0, -1.2)


def _run(xyz, q, **opt):
    import torch
    from paper_1902_05875_amd import api
    f = api.TEFMM(K3, D3, **opt)
    f.set_particles(xyz)
    phi = f.evaluate(torch.from_numpy(np.ascontiguousarray(q)).cuda())
    torch.cuda.synchronize()
    st = f.stats()
    f.close()
    return phi.cpu().numpy(), st


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("tpl", [1, 2, 4])
def test_sym_matches_one_sided(tpl, depth):
    """30,000 particles plus 16 pairs 1e-6 apart; depth 2 (~470 per leaf: several target
    passes per leaf for every lane width) and depth 3 (~59 per leaf, ragged passes)."""
    from paper_1902_05875_amd import inputs
    xyz, q = inputs.workload("c2", n=30_000)
    xyz, q, _ = inputs.with_close_pairs(xyz, q, 16, 1e-6, seed=7)
    a, sa = _run(xyz, q, p=6, precision="fp32", depth=depth, p2p_targets=tpl)
    b, sb = _run(xyz, q, p=6, precision="fp32", depth=depth, p2p_targets=-1)
    e = _rel(a, b)
    print(f"symmetric ({tpl} targets/lane) vs one-sided, depth {depth}: rel diff {e:.3e}")
    assert sa["p2p_pairs"] == sb["p2p_pairs"]
    assert e < 1e-5


@pytest.mark.parametrize("tpl", [1, 4])
def test_sym_empty_leaves(tpl):
    """Two small clusters in opposite corners of the root cube: most leaves are empty, and
    leaves on the grid boundary lack backward neighbours."""
    rng = np.random.default_rng(11)
    n = 6000
    c1 = np.array([-0.3, -0.3, -0.9]) + rng.uniform(-0.05, 0.05, size=(n, 3))
    c2 = np.array([0.3, 0.3, -0.3]) + rng.uniform(-0.05, 0.05, size=(n, 3))
    xyz = np.concatenate([c1, c2])
    q = rng.uniform(-1, 1, 2 * n) + 1j * rng.uniform(-1, 1, 2 * n)
    a, _ = _run(xyz, q, p=6, precision="fp32", depth=4, p2p_targets=tpl)
    b, _ = _run(xyz, q, p=6, precision="fp32", depth=4, p2p_targets=-1)
    e = _rel(a, b)
    print(f"clusters, symmetric ({tpl}) vs one-sided: rel diff {e:.3e}")
    assert e < 1e-5


def test_sym_deterministic():
    """The source-side sums are combined in a fixed order: repeats are bitwise equal."""
    import torch
    from paper_1902_05875_amd import api, inputs
    xyz, q = inputs.workload("c2", n=40_000)
    f = api.TEFMM(K3, D3, p=6, precision="fp32")
    f.set_particles(xyz)
    qt = torch.from_numpy(q).cuda()
    a = f.evaluate(qt).cpu().numpy()
    b = f.evaluate(qt).cpu().numpy()
    f.close()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("depth", [2, 3, 5])
@pytest.mark.parametrize("tpl", [1, 2])
def test_sym_fp64_matches_one_sided(tpl, depth):
    """FP64: only the order of the sums differs.  Depths 2 and 3 take the sine and
    cosine with argument reduction (k r above pi/4 inside a leaf block), depth 5 the
    short series (about one particle per leaf: mostly one-target passes)."""
    from paper_1902_05875_amd import inputs
    xyz, q = inputs.workload("c2", n=30_000)
    xyz, q, _ = inputs.with_close_pairs(xyz, q, 16, 1e-6, seed=7)
    a, sa = _run(xyz, q, p=8, precision="fp64", depth=depth, p2p_targets=tpl)
    b, sb = _run(xyz, q, p=8, precision="fp64", depth=depth, p2p_targets=-1)
    e = _rel(a, b)
    print(f"FP64 symmetric ({tpl} targets/lane) vs one-sided, depth {depth}: rel diff {e:.3e}")
    assert sa["p2p_pairs"] == sb["p2p_pairs"]
    assert e < 1e-12


def test_sym_fp64_empty_leaves_and_deterministic():
    """FP64 on two clusters (mostly empty leaves), and a bitwise-equal repeat."""
    import torch
    from paper_1902_05875_amd import api
    rng = np.random.default_rng(12)
    n = 5000
    c1 = np.array([-0.3, -0.3, -0.9]) + rng.uniform(-0.05, 0.05, size=(n, 3))
    c2 = np.array([0.3, 0.3, -0.3]) + rng.uniform(-0.05, 0.05, size=(n, 3))
    xyz = np.concatenate([c1, c2])
    q = rng.uniform(-1, 1, 2 * n) + 1j * rng.uniform(-1, 1, 2 * n)
    b, _ = _run(xyz, q, p=8, precision="fp64", depth=4, p2p_targets=-1)
    f = api.TEFMM(K3, D3, p=8, precision="fp64", depth=4, p2p_targets=2)
    f.set_particles(xyz)
    qt = torch.from_numpy(q).cuda()
    a1 = f.evaluate(qt).cpu().numpy()
    a2 = f.evaluate(qt).cpu().numpy()
    f.close()
    e = _rel(a1, b)
    print(f"FP64 clusters, symmetric vs one-sided: rel diff {e:.3e}")
    assert e < 1e-12
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("depth,tpl", [(4, 1), (4, 2), (3, 2)])
def test_poly_pair_value(depth, tpl):
    """FP32 near field with the pair value from quadratics in r^2 (the default where their
    fit is within 3e-7) against the hardware sine and cosine, close pairs included.  At
    depth 3 the mid layer's k r over a leaf block is too large for the fit: both runs then
    take the hardware path and agree bitwise."""
    from paper_1902_05875_amd import inputs
    xyz, q = inputs.workload("c2", n=60_000)
    xyz, q, _ = inputs.with_close_pairs(xyz, q, 16, 1e-6, seed=9)
    a, sa = _run(xyz, q, p=6, precision="fp32", depth=depth, p2p_targets=tpl)
    b, sb = _run(xyz, q, p=6, precision="fp32", depth=depth, p2p_targets=tpl, p2p_poly=-1)
    e = _rel(a, b)
    print(f"depth {depth}, {tpl} targets/lane: fit error {sa['p2p_poly_err']:.2e}, rel diff {e:.3e}")
    assert sb["p2p_poly_err"] == 0
    if depth == 4:
        assert 0 < sa["p2p_poly_err"] <= 3e-7
        assert e < 1e-6
    else:
        assert sa["p2p_poly_err"] == 0
        assert np.array_equal(a, b)


def test_poly_option_checked():
    from paper_1902_05875_amd import api
    with pytest.raises(api.TefmmError):
        api.TEFMM(K3, D3, p=6, precision="fp32", p2p_poly=1)


def test_poly_pair_value_several_vectors():
    """The one-sided FP32 kernel (several charge vectors, 8 per pair value) with the
    quadratic pair value against the hardware sine and cosine."""
    from paper_1902_05875_amd import inputs
    xyz, q = inputs.workload("c2", n=60_000, n_rhs=4)
    q = np.ascontiguousarray(q.T)  # (vectors, N)
    a, sa = _run(xyz, q, p=6, precision="fp32", depth=4)
    b, sb = _run(xyz, q, p=6, precision="fp32", depth=4, p2p_poly=-1)
    e = _rel(a, b)
    print(f"4 vectors: fit error {sa['p2p_poly_err']:.2e}, rel diff {e:.3e}")
    assert a.shape == (4, xyz.shape[0])
    assert 0 < sa["p2p_poly_err"] <= 3e-7 and sb["p2p_poly_err"] == 0
    assert e < 1e-6

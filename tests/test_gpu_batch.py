"""Batched multi-geometry evaluation (HIP graph), graph replays and the autotuner."""
import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu

K3 = (0.8, 1.5, 2.0)
D3 = (0.0, -1.2)


def _geoms():
    from paper_1902_05875_amd import inputs
    rng = np.random.default_rng(3)
    out = []
    for g, (n, a) in enumerate([(12_000, None), (30_000, 0.1), (7_000, None), (20_000, 0.15)]):
        r = np.random.default_rng(900 + g)
        xyz = inputs.cube(r, n, inputs.MID_CENTRE) if a is None else inputs.irregular(r, n, inputs.MID_CENTRE, a)
        out.append((xyz, inputs.charges(r, n, 1 if g != 1 else 2)))
    return out


def test_batch_equals_individual_and_replays():
    import torch
    from paper_1902_05875_amd import api
    geoms = _geoms()
    hs, qs, ref = [], [], []
    for xyz, q in geoms:
        f = api.TEFMM(K3, D3, p=8)
        f.set_particles(xyz)
        qt = torch.from_numpy(np.ascontiguousarray(q.T if q.ndim == 2 else q)).cuda()
        ref.append(f.evaluate(qt).cpu().numpy())
        hs.append(f)
        qs.append(qt)
    outs = [torch.empty_like(q) for q in qs]
    for rep in range(3):
        # eager work between replays; charges change in place (the graph reads them at replay)
        scale = 1.0 + rep
        for q in qs:
            q.mul_(scale)
        api.evaluate_batch(hs, qs, outs)
        torch.cuda.synchronize()
        x = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        for g in range(len(hs)):
            expect = ref[g] * np.prod([1.0 + r for r in range(rep + 1)])
            got = outs[g].cpu().numpy()
            np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
        del x
    for f in hs:
        f.close()


def test_batch_fp32_matches_individual():
    """FP32: the batch (graph, near and far field serialised, the M2L kernel that stages
    the next offset during the current one) against single evaluations (near field beside
    the far field, the other M2L kernel): the same arithmetic in the same order."""
    import torch
    from paper_1902_05875_amd import api
    geoms = _geoms()
    hs, qs, ref = [], [], []
    for xyz, q in geoms:
        f = api.TEFMM(K3, D3, p=8, precision="fp32")
        f.set_particles(xyz)
        qt = torch.from_numpy(np.ascontiguousarray(q.T if q.ndim == 2 else q)).cuda()
        ref.append(f.evaluate(qt).cpu().numpy())
        hs.append(f)
        qs.append(qt)
    outs = [torch.empty_like(q) for q in qs]
    api.evaluate_batch(hs, qs, outs)
    torch.cuda.synchronize()
    for g in range(len(hs)):
        got = outs[g].cpu().numpy()
        e = np.linalg.norm(got - ref[g]) / np.linalg.norm(ref[g])
        print(f"geometry {g}: batch vs single rel diff {e:.3e}")
        assert e < 1e-6
    for f in hs:
        f.close()


def test_autotune_keeps_results():
    import torch
    from oracle import direct
    from oracle.medium import Medium
    from paper_1902_05875_amd import api, inputs
    xyz, q = inputs.workload("c2", n=20_000)
    f = api.TEFMM(K3, D3, p=8, precision="fp32")
    f.set_particles(xyz)
    depth, ncb = f.autotune()
    assert 2 <= depth <= 7 and ncb in (1, 2)
    assert f.tree()["depth"] == depth
    phi = f.evaluate(torch.from_numpy(q).cuda()).cpu().numpy()
    f.close()
    idx = np.loadtxt(__import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                                 "expected_n20k.txt"))
    tg = idx[:, 0].astype(int)
    ref = idx[:, 1] + 1j * idx[:, 2]
    check(f"autotune depth {depth} ncb {ncb}", phi[tg], ref, 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_queue_equals_graph_batch(precision):
    """The near fields of all geometries in one persistent launch (work queue of pair items,
    then gather items waiting on their geometry) give the graph batch's result bit for bit,
    over three replays with the charges changed in place and eager work between them."""
    import torch
    from paper_1902_05875_amd import api, inputs
    hs, qs = [], []
    for g, (n, a) in enumerate([(12_000, None), (30_000, 0.1), (7_000, None), (20_000, 0.15), (2_000, None)]):
        r = np.random.default_rng(950 + g)
        xyz = inputs.cube(r, n, inputs.MID_CENTRE) if a is None else inputs.irregular(r, n, inputs.MID_CENTRE, a)
        f = api.TEFMM(K3, D3, p=8, precision=precision)
        f.set_particles(xyz)
        hs.append(f)
        qs.append(torch.from_numpy(inputs.charges(r, n)).cuda())
    outs_g = [torch.empty_like(q) for q in qs]
    outs_q = [torch.empty_like(q) for q in qs]
    for rep in range(3):
        for q in qs:
            q.mul_(1.0 + 0.5 * rep)
        api.evaluate_batch(hs, qs, outs_g)
        torch.cuda.synchronize()
        api.evaluate_batch(hs, qs, outs_q, queue=True)
        api.batch_check(hs[0])
        x = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        for g in range(len(hs)):
            a, b = outs_g[g].cpu().numpy(), outs_q[g].cpu().numpy()
            assert np.array_equal(a, b), (precision, rep, g, np.max(np.abs(a - b)))
        del x
    for f in hs:
        f.close()


def test_batch_queue_rejects_several_vectors():
    import torch
    from paper_1902_05875_amd import api, inputs
    r = np.random.default_rng(5)
    xyz = inputs.cube(r, 3000, inputs.MID_CENTRE)
    f = api.TEFMM(K3, D3, p=6)
    f.set_particles(xyz)
    q = torch.from_numpy(np.ascontiguousarray(inputs.charges(r, 3000, 2).T)).cuda()
    with pytest.raises(api.TefmmError):
        api.evaluate_batch([f], [q], queue=True)
    f.close()

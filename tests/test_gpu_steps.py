"""GPU parity of individual steps (through the C ABI) against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K3 = (0.8, 1.5, 2.0)
D3 = (0.0, -1.2)


def _api():
    from paper_1902_05875_amd import api
    api.lib()
    return api


def test_mfma_lane_layout():
    """The 16x16x4 FP64/FP32 MFMA operand/result layout the M2L kernel assumes."""
    assert _api().selftest_mfma() == 0


@pytest.mark.parametrize("pt", [(2.0, 0.0, 0.0), (1.0, -2.0, 3.0), (0.3, 0.4, 2.5 - 1.2j), (2.0, 2.0, -2.0)])
def test_taylor_recurrence_vs_series(pt):
    """GPU derivative recurrence vs the oracle's power-series Taylor coefficients (orders <= 16)."""
    from oracle.taylor import coefficient_list
    api = _api()
    k, h, order = 1.5, 0.25, 16
    x, y, z = pt
    got = api.taylor_coefficients([x * h], [y * h], [complex(z) * h], k, h, order)[0]
    ref = coefficient_list(x * h, y * h, complex(z) * h, k, order)
    # scaled coefficients h^{|g|} D^g f / g!
    n = 0
    for m in range(order + 1):
        cnt = (m + 1) * (m + 2) // 2
        r = ref[n:n + cnt] * h ** m
        g = got[n:n + cnt]
        scale = np.max(np.abs(r))
        assert np.max(np.abs(g - r)) <= 1e-11 * scale, (m, np.max(np.abs(g - r)) / scale)
        n += cnt


def _p2m_ref(xyz, q, lo, side, depth, p, box):
    nb = 2 ** depth
    h = side / nb
    idx = np.floor((xyz - lo) / side * nb).astype(int).clip(0, nb - 1)
    lin = (idx[:, 0] * nb + idx[:, 1]) * nb + idx[:, 2]
    sel = lin == box
    ix, iy, iz = box // (nb * nb), (box // nb) % nb, box % nb
    c = lo + (np.array([ix, iy, iz]) + 0.5) * h
    u = (xyz[sel] - c) / h
    out = []
    for m in range(p + 1):
        for a in range(m, -1, -1):
            for b in range(m - a, -1, -1):
                cc = m - a - b
                out.append(np.sum(q[sel] * u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** cc))
    return np.array(out)


def test_p2m_and_m2m_moments():
    """Leaf moments equal their definition; parent moments (after M2M) equal the definition
    over the parent's particles (the shift is exact)."""
    import torch
    from paper_1902_05875_amd import inputs
    api = _api()
    xyz, q = inputs.workload("c2", n=20_000)
    f = api.TEFMM(K3, D3, p=6, depth=3)
    f.set_particles(xyz)
    f.evaluate(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    t = f.tree(0)
    lo = t["centre"] - 0.5 * t["side"]
    for level in (3, 2):
        mom = f.moments(0, level)
        for box in (0, 5, 8 ** level - 1, 8 ** level // 2 + 3):
            ref = _p2m_ref(xyz, q, lo, t["side"], level, 6, box)
            np.testing.assert_allclose(mom[box], ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))
    f.close()


@pytest.mark.parametrize("p", [7, 8])
@pytest.mark.parametrize("tile", [1, 2])
def test_m2l_fp32_matches_fp64(p, tile):
    """Mixed FP32 against FP64 at the same order, depth and M2L tile width: only rounding
    differs.  p = 7 (an even number of reduced moments) stages the source moments in runs
    of 4 (16 targets per workgroup) or 8 (32) entries per thread, p = 8 element by element;
    depth 3 leaves the coarse levels' tiles partly filled."""
    import torch
    from paper_1902_05875_amd import inputs
    api = _api()
    xyz, q = inputs.workload("c2", n=20_000)
    out = []
    for prec in ("fp64", "fp32"):
        f = api.TEFMM(K3, D3, p=p, depth=3, precision=prec, m2l_tile=tile)
        f.set_particles(xyz)
        out.append(f.evaluate(torch.from_numpy(q).cuda()).cpu().numpy())
        f.close()
    e = np.linalg.norm(out[1] - out[0]) / np.linalg.norm(out[0])
    print(f"p={p} tile={tile}: FP32 vs FP64 rel diff {e:.3e}")
    assert e < 1e-5

"""Media other than the three-layer one of the workloads, against the oracle's direct sum:
one layer (free space, no interface), two layers (one interface; particles in one layer, and in
both, which takes the cross-layer translations), four layers (three interfaces), five and
eight layers (the most the library takes) with particles in two of them."""
import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu

# name: (wave numbers, interfaces, [(cube centre z, particles)])
CASES = {
    "one": ((1.5,), (), [(-0.6, 1500)]),
    "two": ((1.0, 2.0), (0.0,), [(-0.6, 1500)]),
    "two_both": ((1.0, 2.0), (0.0,), [(0.6, 800), (-0.6, 800)]),
    "four": ((0.8, 1.5, 2.0, 1.2), (0.0, -1.2, -2.0), [(-0.6, 1500)]),
    "five_both": ((0.8, 1.5, 2.0, 1.2, 0.9), (0.0, -1.2, -2.0, -2.6), [(-0.6, 900), (-2.3, 500, 0.4)]),
    "eight_both": ((0.8, 1.5, 2.0, 1.2, 0.9, 1.7, 1.1, 1.4), (0.0, -1.2, -2.0, -2.6, -3.4, -4.0, -4.8),
                   [(-0.6, 900), (-3.0, 500, 0.5)]),
}


def _case(name):
    k, d, cubes = CASES[name]
    rng = np.random.default_rng(600 + list(CASES).index(name))
    # cubes of side 1 unless a side is given (a thin layer holds a smaller cube)
    xyz = np.concatenate([rng.uniform(-0.5, 0.5, (c[1], 3)) * (c[2] if len(c) > 2 else 1.0) + [0.0, 0.0, c[0]]
                          for c in cubes])
    q = rng.uniform(-1, 1, len(xyz)) + 1j * rng.uniform(-1, 1, len(xyz))
    return k, d, xyz, q


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision,p,tol", [("fp64", 8, 3e-5), ("fp64", 12, 2e-6), ("fp32", 8, 1e-4)])
def test_media(name, precision, p, tol):
    import torch
    from oracle import direct
    from oracle.medium import Medium
    from paper_1902_05875_amd import api
    k, d, xyz, q = _case(name)
    f = api.TEFMM(k, d, p=p, precision=precision)
    f.set_particles(xyz)
    phi = f.evaluate(torch.from_numpy(q).cuda()).cpu().numpy()
    st = f.stats()
    f.close()
    tg = np.arange(0, len(xyz), len(xyz) // 40)
    ref = direct.potential(Medium(k, d), xyz, q, tg)
    check(f"{name} {precision} p={p} depth {st['depth']}", phi[tg], ref, tol)

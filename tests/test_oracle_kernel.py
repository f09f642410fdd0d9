"""Oracle reaction kernel: exact special cases and invariants of the layered Green's function."""
import numpy as np
import pytest

from oracle.medium import Medium
from oracle.sommerfeld import reaction_pair
from oracle import direct

K = (0.8, 1.5, 2.0)
D = (0.0, -1.2)
ZS = {0: 0.35, 1: -0.55, 2: -1.7}


def _full_g(med, l, lp, r, rp):
    rho = np.hypot(r[0] - rp[0], r[1] - rp[1])
    g = reaction_pair(med, l, lp, rho, r[2], rp[2])[0]
    if l == lp:
        R = np.linalg.norm(np.subtract(r, rp))
        g += np.exp(1j * med.k[l] * R) / (4 * np.pi * R)
    return g


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("lp", [0, 1, 2])
def test_equal_k_is_free_space(l, lp):
    """One wave number everywhere: G is exp(ikR)/(4 pi R) for every layer pair."""
    med = Medium((1.5, 1.5, 1.5), D)
    r = (0.1, -0.2, ZS[l] + 0.05)
    rp = (-0.3, 0.25, ZS[lp])
    R = np.linalg.norm(np.subtract(r, rp))
    np.testing.assert_allclose(_full_g(med, l, lp, r, rp), np.exp(1.5j * R) / (4 * np.pi * R), rtol=1e-11)


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("lp", [0, 1, 2])
def test_weighted_reciprocity(l, lp):
    """The flux condition k du/dz continuous (Sec. 2.1) gives k_l G_{l,lp}(r, r') = k_lp G_{lp,l}(r', r)."""
    med = Medium(K, D)
    r = (0.1, -0.2, ZS[l] + 0.07)
    rp = (-0.3, 0.25, ZS[lp] - 0.04)
    a = med.k[l] * _full_g(med, l, lp, r, rp)
    b = med.k[lp] * _full_g(med, lp, l, rp, r)
    np.testing.assert_allclose(a, b, rtol=1e-11)


@pytest.mark.parametrize("j", [0, 1])
@pytest.mark.parametrize("lp", [0, 1, 2])
def test_interface_conditions(j, lp):
    """G continuous and k dG/dz continuous across interface d_j (Sec. 2.1)."""
    med = Medium(K, D)
    rp = (0.2, -0.1, ZS[lp] + 0.03)
    x, y = -0.15, 0.3
    h = 1e-3
    up, lo = j, j + 1
    zi = med.d[j]

    def g(l, z):
        return _full_g(med, l, lp, (x, y, z), rp)

    # one-sided values and slopes (second-order one-sided differences)
    va = g(up, zi + 1e-9)
    vb = g(lo, zi - 1e-9)
    sa = (-3 * g(up, zi) + 4 * g(up, zi + h) - g(up, zi + 2 * h)) / (2 * h)
    sb = (3 * g(lo, zi) - 4 * g(lo, zi - h) + g(lo, zi - 2 * h)) / (2 * h)
    np.testing.assert_allclose(va, vb, rtol=1e-7)
    np.testing.assert_allclose(med.k[up] * sa, med.k[lo] * sb, rtol=2e-5)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_helmholtz_residual(l):
    """The reaction part solves the homogeneous Helmholtz equation in the target layer."""
    med = Medium(K, D)
    rp = (0.1, 0.05, ZS[1])
    c = np.array([-0.2, 0.15, ZS[l] + 0.02])
    h = 2e-2
    lap = 0
    val = reaction_pair(med, l, 1, np.hypot(*(c[:2] - rp[:2])), c[2], rp[2])[0]
    for ax in range(3):
        acc = 0
        for m, w in [(-2, -1 / 12), (-1, 4 / 3), (0, -5 / 2), (1, 4 / 3), (2, -1 / 12)]:
            p = c.copy()
            p[ax] += m * h
            acc += w * reaction_pair(med, l, 1, np.hypot(*(p[:2] - rp[:2])), p[2], rp[2])[0]
        lap += acc / h**2
    assert abs(lap + med.k[l] ** 2 * val) < 1e-6 * abs(med.k[l] ** 2 * val)


def test_sum_integral_swap_matches_pairwise():
    """The direct sum (sum over sources inside the integral) equals the sum of pairwise kernels."""
    med = Medium(K, D)
    rng = np.random.default_rng(7)
    xyz = np.concatenate([rng.random((20, 3)) * [1, 1, 0.6] + [-.5, -.5, 0.2],
                          rng.random((20, 3)) * [1, 1, 0.8] + [-.5, -.5, -1.0],
                          rng.random((20, 3)) * [1, 1, 0.5] + [-.5, -.5, -2.0]])
    q = rng.uniform(-1, 1, 60) + 1j * rng.uniform(-1, 1, 60)
    tg = np.array([3, 25, 50])
    got = direct.reaction_part(med, xyz, q, tg)
    lay = med.layer_of(xyz[:, 2])
    for i, t in enumerate(tg):
        ref = 0
        for lp in range(3):
            s = lay == lp
            rho = np.hypot(xyz[t, 0] - xyz[s, 0], xyz[t, 1] - xyz[s, 1])
            ref += np.sum(q[s] * reaction_pair(med, lay[t], lp, rho, xyz[t, 2], xyz[s, 2]))
        np.testing.assert_allclose(got[i], ref, rtol=1e-11)


def test_free_part_excludes_self():
    med = Medium(K, D)
    xyz = np.array([[0, 0, -0.5], [0.3, 0, -0.5], [0, 0, 0.5]])
    q = np.array([1.0, 2.0, 5.0]) + 0j
    got = direct.free_part(med, xyz, q, np.array([0]))
    np.testing.assert_allclose(got[0], 2.0 * np.exp(1.5j * 0.3) / (4 * np.pi * 0.3), rtol=1e-14)


# Media other than the three-layer one of the workloads: two layers (one interface) and
# four layers (three interfaces).  Points per layer for each.
MEDIA = {
    "two": (Medium((1.0, 2.0), (0.0,)), {0: 0.4, 1: -0.6}),
    "four": (Medium((0.8, 1.5, 2.0, 1.2), (0.0, -1.2, -2.0)), {0: 0.35, 1: -0.55, 2: -1.6, 3: -2.5}),
    "five": (Medium((0.8, 1.5, 2.0, 1.2, 0.9), (0.0, -1.2, -2.0, -2.6)),
             {0: 0.35, 1: -0.55, 2: -1.6, 3: -2.3, 4: -3.0}),
    "eight": (Medium((0.8, 1.5, 2.0, 1.2, 0.9, 1.7, 1.1, 1.4), (0.0, -1.2, -2.0, -2.6, -3.4, -4.0, -4.8)),
              {0: 0.35, 1: -0.55, 2: -1.6, 3: -2.3, 4: -3.0, 5: -3.7, 6: -4.4, 7: -5.2}),
}


@pytest.mark.parametrize("name", ["two", "four", "five", "eight"])
def test_weighted_reciprocity_other_media(name):
    """k_l G_{l,lp}(r, r') = k_lp G_{lp,l}(r', r) for every layer pair (the flux condition of Sec. 2.1)."""
    med, zs = MEDIA[name]
    for l in zs:
        for lp in zs:
            r = (0.1, -0.2, zs[l] + 0.07)
            rp = (-0.3, 0.25, zs[lp] - 0.04)
            a = med.k[l] * _full_g(med, l, lp, r, rp)
            b = med.k[lp] * _full_g(med, lp, l, rp, r)
            np.testing.assert_allclose(a, b, rtol=1e-10)


@pytest.mark.parametrize("name", ["two", "four", "five"])
def test_interface_conditions_other_media(name):
    """G and k dG/dz continuous across every interface, for a source in every layer."""
    med, zs = MEDIA[name]
    h = 1e-3
    for j, zi in enumerate(med.d):
        for lp in zs:
            rp = (0.2, -0.1, zs[lp] + 0.03)

            def g(l, z):
                return _full_g(med, l, lp, (-0.15, 0.3, z), rp)

            va, vb = g(j, zi + 1e-9), g(j + 1, zi - 1e-9)
            sa = (-3 * g(j, zi) + 4 * g(j, zi + h) - g(j, zi + 2 * h)) / (2 * h)
            sb = (3 * g(j + 1, zi) - 4 * g(j + 1, zi - h) + g(j + 1, zi - 2 * h)) / (2 * h)
            np.testing.assert_allclose(va, vb, rtol=1e-7)
            np.testing.assert_allclose(med.k[j] * sa, med.k[j + 1] * sb, rtol=2e-5)


def test_four_layers_reduce_to_three():
    """A fourth layer with the third layer's wave number is no interface at all: the four-layer
    kernel equals the three-layer one for points in the first three layers (and in the merged
    bottom layer)."""
    m4 = Medium((0.8, 1.5, 2.0, 2.0), (0.0, -1.2, -2.0))
    m3 = Medium((0.8, 1.5, 2.0), (0.0, -1.2))
    pts = {0: 0.35, 1: -0.55, 2: -1.6}
    for l, z in pts.items():
        for lp, zp in pts.items():
            r, rp = (0.1, -0.2, z + 0.05), (-0.3, 0.25, zp - 0.03)
            np.testing.assert_allclose(_full_g(m4, l, lp, r, rp), _full_g(m3, l, lp, r, rp), rtol=1e-9)
    # below the removed interface: layer 3 of the four-layer medium is layer 2 of the three-layer one
    r, rp = (0.1, -0.2, -2.4), (-0.3, 0.25, -0.6)
    np.testing.assert_allclose(_full_g(m4, 3, 1, r, rp), _full_g(m3, 2, 1, r, rp), rtol=1e-9)


def test_eight_layers_reduce_to_three():
    """Five extra layers below the third, all with its wave number, are no interfaces at all: the
    eight-layer kernel equals the three-layer one (the interface solve of Sec. 2.1 with seven
    interfaces against the one with two)."""
    m8 = Medium((0.8, 1.5, 2.0, 2.0, 2.0, 2.0, 2.0, 2.0), (0.0, -1.2, -2.0, -2.6, -3.4, -4.0, -4.8))
    m3 = Medium((0.8, 1.5, 2.0), (0.0, -1.2))
    pts = {0: 0.35, 1: -0.55, 2: -1.6}
    for l, z in pts.items():
        for lp, zp in pts.items():
            r, rp = (0.1, -0.2, z + 0.05), (-0.3, 0.25, zp - 0.03)
            np.testing.assert_allclose(_full_g(m8, l, lp, r, rp), _full_g(m3, l, lp, r, rp), rtol=1e-9)
    r, rp = (0.1, -0.2, -3.7), (-0.3, 0.25, -0.6)  # layer 5 of the eight is layer 2 of the three
    np.testing.assert_allclose(_full_g(m8, 5, 1, r, rp), _full_g(m3, 2, 1, r, rp), rtol=1e-9)


def test_reaction_part_converged_next_to_interfaces():
    """Sources and targets 0.01-0.02 from an interface (decay lengths 0.02-0.04): the direct
    sum's fixed quadrature rule agrees with a refined rule (order 24, panels a third and a
    half as wide) and with the pairwise kernel of sommerfeld.reaction_pair (its own rule)."""
    med = Medium(K, D)
    rng = np.random.default_rng(11)
    m = 12
    xyz = np.column_stack([rng.uniform(-0.5, 0.5, (2 * m, 2)),
                           np.concatenate([-rng.uniform(0.01, 0.02, m), -1.2 + rng.uniform(0.01, 0.02, m)])])
    q = rng.uniform(-1, 1, 2 * m) + 1j * rng.uniform(-1, 1, 2 * m)
    tg = np.array([0, 5, m, m + 7])
    got = direct.reaction_part(med, xyz, q, tg)
    saved = (direct.QUAD_ORDER, direct.HEAD_WIDTH, direct.TAIL_WIDTH)
    try:
        direct.QUAD_ORDER, direct.HEAD_WIDTH, direct.TAIL_WIDTH = 24, saved[1] / 3, saved[2] / 2
        fine = direct.reaction_part(med, xyz, q, tg)
    finally:
        direct.QUAD_ORDER, direct.HEAD_WIDTH, direct.TAIL_WIDTH = saved
    np.testing.assert_allclose(got, fine, rtol=1e-11)
    lay = med.layer_of(xyz[:, 2])
    ref = np.array([np.sum(q * reaction_pair(med, lay[t], 1, np.hypot(xyz[t, 0] - xyz[:, 0], xyz[t, 1] - xyz[:, 1]),
                                             xyz[t, 2], xyz[:, 2])) for t in tg])
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_kernel_matrix_matches_the_direct_sum():
    """The dense kernel matrix (pairwise quadrature) applied to charges equals the direct sum
    with the sum over sources inside the integral, three layers, every layer pair."""
    med = Medium(K, D)
    rng = np.random.default_rng(21)
    xyz = np.concatenate([rng.random((12, 3)) * [1, 1, 0.6] + [-.5, -.5, 0.2],
                          rng.random((14, 3)) * [1, 1, 0.8] + [-.5, -.5, -1.0],
                          rng.random((10, 3)) * [1, 1, 0.5] + [-.5, -.5, -2.0]])
    q = rng.uniform(-1, 1, 36) + 1j * rng.uniform(-1, 1, 36)
    G = direct.kernel_matrix(med, xyz)
    np.testing.assert_allclose(G @ q, direct.potential(med, xyz, q), rtol=1e-10)
    # weighted reciprocity of the matrix: k_l G[i, j] = k_lp G[j, i]
    kl = np.asarray(med.k)[med.layer_of(xyz[:, 2])]
    np.testing.assert_allclose(kl[:, None] * G, (kl[:, None] * G).T, rtol=1e-9, atol=1e-14)

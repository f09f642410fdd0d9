"""Oracle densities: direct interface solve vs the closed forms of Appendix A."""
import numpy as np
import pytest

from oracle.medium import Medium, densities, kz, to_paper_reference

K = (0.8, 1.5, 2.0)
KR = np.array([0.3, 1.2 + 0.1j, 2.5 - 0.5j, 4.0 - 1.0j, 0.9 - 1.0j, 7.0])


def _appendix_three_layer(d, kr):
    """Appendix A, three layers with interfaces 0 and -d: Eq. densitythreelayer1-3,
    kappa_11, kappa_12 (Eq. kappa1112), kappa_31, kappa_32."""
    k0, k1, k2 = K
    K0, K1, K2 = kz(k0, kr), kz(k1, kr), kz(k2, kr)
    a0, a1, a2 = k0 * K0, k1 * K1, k2 * K2
    e = lambda x: np.exp(1j * x)
    k11 = (a1 - a2) / 2 * e(2 * d * K1) + (a1 + a2) / 2
    k12 = 1j * ((a2 - a1) / 2 * e(2 * d * K1) + (a1 + a2) / 2)
    den = a0 * k11 - 1j * a1 * k12
    k31 = (a1 - a0) / 2 * e(2 * d * K1) + (a1 + a0) / 2
    k32 = 1j * ((a0 - a1) / 2 * e(2 * d * K1) + (a0 + a1) / 2)
    den3 = a2 * k31 - 1j * a1 * k32
    app = {
        (0, 0, "u", "u"): (a0 * k11 + 1j * a1 * k12) / den,
        (1, 0, "u", "u"): k0 * K1 * (a1 - a2) * e(d * K1) / den,
        (1, 0, "d", "u"): k0 * K1 * (a1 + a2) * e(d * K1) / den,
        (2, 0, "d", "u"): 2 * k0 * k1 * K1 * K2 * e(d * K1) / den,
        (0, 1, "u", "u"): k1 * K0 * (a1 - a2) * e(d * K1) / den,
        (0, 1, "u", "d"): k1 * K0 * (a1 + a2) / den,
        (1, 1, "u", "u"): (a1 - a2) / den * (a1 + a0) / 2,
        (1, 1, "u", "d"): (a1 - a2) / den * (a1 - a0) / 2 * e(d * K1),
        (1, 1, "d", "u"): (a1 - a0) * e(d * K1) / den * (a1 - a2) / 2 * e(d * K1),
        (1, 1, "d", "d"): (a1 - a0) * e(d * K1) / den * (a1 + a2) / 2,
        (2, 1, "d", "u"): k1 * K2 * e(-d * K2) / den * (a1 + a0),
        (2, 1, "d", "d"): k1 * K2 * e(-d * K2) / den * (a1 - a0) * e(d * K1),
        (0, 2, "u", "d"): 2 * a1 * k2 * K0 * e(d * K1) / den3,
        (1, 2, "u", "d"): k2 * K1 * (a1 + a0) / den3,
        (1, 2, "d", "d"): k2 * K1 * (a1 - a0) * e(2 * d * K1) / den3,
        (2, 2, "d", "d"): (a2 * k31 + 1j * a1 * k32) / den3,
    }
    return app, den, den3, (k11, k12)


@pytest.mark.parametrize("d", [1.2, 2.0])
def test_three_layer_appendix(d):
    med = Medium(K, (0.0, -d))
    app, den, den3, _ = _appendix_three_layer(d, KR)
    # the two forms of the common denominator agree (end of Appendix A)
    np.testing.assert_allclose(den, den3, rtol=1e-13)
    sig = {lp: densities(med, lp, KR) for lp in range(3)}
    for (m, lp, a, b), v in app.items():
        mine = sig[lp][(m, a, b)]
        if a == "d" and m == 1:
            # Appendix A writes the middle layer's down-wave relative to z = -d
            mine = to_paper_reference(med, m, KR, mine, -d)
        if a == "d" and m == 2 and lp == 1:
            # ... and the bottom layer's down-wave, for a middle-layer source, relative to z = 0
            mine = to_paper_reference(med, m, KR, mine, 0.0)
        np.testing.assert_allclose(mine, v, rtol=1e-12, atol=1e-14, err_msg=str((m, lp, a, b)))


def test_two_layer_appendix():
    """Eq. densitytwolayer1 and densitytwolayer2 (one interface at z = 0)."""
    k0, k1 = 0.8, 1.5
    med = Medium((k0, k1), (0.0,))
    K0, K1 = kz(k0, KR), kz(k1, KR)
    a0, a1 = k0 * K0, k1 * K1
    s0 = densities(med, 0, KR)
    s1 = densities(med, 1, KR)
    np.testing.assert_allclose(s0[(0, "u", "u")], (a0 - a1) / (a0 + a1), rtol=1e-13)
    np.testing.assert_allclose(s0[(1, "d", "u")], 2 * k0 * K1 / (a0 + a1), rtol=1e-13)
    np.testing.assert_allclose(s1[(0, "u", "d")], 2 * k1 * K0 / (a0 + a1), rtol=1e-13)
    np.testing.assert_allclose(s1[(1, "d", "d")], (a1 - a0) / (a0 + a1), rtol=1e-13)


def test_equal_wavenumbers_transparent():
    """With one wave number everywhere nothing reflects and everything transmits."""
    med = Medium((1.5, 1.5, 1.5), (0.0, -1.2))
    for lp in range(3):
        s = densities(med, lp, KR)
        for (m, a, b), v in s.items():
            transmitted = (m < lp and a == "u" and b == "d") or (m > lp and a == "d" and b == "u")
            # the free wave crosses every layer strictly between source and target
            between = sum(med.thickness(i) for i in range(min(m, lp) + 1, max(m, lp)))
            expect = np.exp(1j * kz(1.5, KR) * between) if transmitted else 0.0
            np.testing.assert_allclose(v, expect, atol=1e-13)


def test_layer_of():
    med = Medium(K, (0.0, -1.2))
    assert list(med.layer_of(np.array([0.5, -0.1, -1.19, -1.21, -3.0]))) == [0, 1, 1, 2, 2]

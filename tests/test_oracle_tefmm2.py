"""Pins of the TEFMM-II oracle (Sec. 4): symmetric derivatives, expansions,
translations and the layered-media integrals, each against something other
than itself: Cartesian Taylor coefficients from power-series composition,
closed forms, polynomial identities, direct sums, the Helmholtz equation and
the values printed in Tables 3.1 and 3.2."""
import math
import os

import numpy as np
import pytest

from oracle import taylor
from oracle import tefmm2 as T
from oracle.medium import Medium
from oracle.sommerfeld import reaction_pair

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table_3_1_3_2.txt")
PAIRS = {1: ((0.5, 1.0, -0.5), (0.3, 1.3, -0.5)), 2: ((0.6, 0.3, -1.2), (0.5, 1.0, -0.5))}
K = 1.3


def h0(x):
    return np.exp(1j * x) / (1j * x)


def _sym_from_cartesian(r, k, N):
    """D^s_{nm} h0 at r from the Cartesian derivatives of exp(ikR)/R (series composition,
    no recurrence): (d_x - i d_y)^s (d_x + i d_y)^(m-s) expanded by the binomial theorem."""
    cube = taylor.coefficients(r[0], r[1], r[2], k, N) / (1j * k)
    f = math.factorial
    out = []
    for (n, m, s) in T.index_set(N):
        acc = 0j
        for a in range(s + 1):
            for b in range(m - s + 1):
                gx, gy, gz = a + b, m - a - b, n - m
                acc += (math.comb(s, a) * math.comb(m - s, b) * (-1j) ** (s - a) * (1j) ** (m - s - b)
                        * cube[gx, gy, gz] * f(gx) * f(gy) * f(gz))
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("r", [(0.7, -0.4, 1.1), (-1.3, 0.2, -0.6), (0.05, 0.9, 0.3)])
def test_symmetric_derivatives_match_cartesian_series(r):
    """Theorem 4.2 (with the readings in the oracle's header) against an independent
    Cartesian route; a wrong sign in any ladder coefficient fails here."""
    r = np.array(r)
    got = T.symmetric_derivatives(r, K, 8)
    ref = _sym_from_cartesian(r, K, 8)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13 * np.max(np.abs(ref)))


def test_ladder_special_case():
    """The theorem's special case D0 Omega^{+-n}_n = Omega^{+-n}_{n+1} / sqrt(2n+3)."""
    for n in range(12):
        for m in (n, -n):
            a, b = T._ladder("0", n, m)
            assert abs(a - 1 / math.sqrt(2 * n + 3)) < 1e-15 and b == 0.0


def test_theorem41_and_corollary_converge():
    r = np.array([0.9, -0.5, 1.2])
    rp = np.array([0.1, 0.15, -0.12])
    exact = h0(K * np.linalg.norm(r - rp))
    e41 = [abs(T.theorem41(r, rp, K, p) - exact) for p in (4, 8, 12, 16)]
    ec = [abs(T.corollary41(rp, r, K, p) - exact) for p in (4, 8, 12, 16)]
    for e in (e41, ec):
        assert all(b < 0.01 * a for a, b in zip(e, e[1:3]))
        assert e[-1] < 1e-13


def _cluster(seed=0, n=20, side=0.3):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)) * side, rng.random(n) - 0.5 + 1j * (rng.random(n) - 0.5)


def test_m2m_is_exact():
    """Moments re-centred by the B coefficients equal the moments about the new centre."""
    xyz, q = _cluster()
    c, c2, p = np.array([0.15, 0.15, 0.15]), np.array([0.4, -0.1, 0.3]), 6
    a2 = T.moments(xyz, q, c2, p)
    got = T.m2m(T.moments(xyz, q, c, p), c - c2, p)
    assert np.max(np.abs(got - a2)) < 1e-14 * np.max(np.abs(a2))


def test_l2l_is_exact():
    """A local expansion re-centred by the C coefficients is the same polynomial."""
    p = 6
    rng = np.random.default_rng(1)
    beta = rng.random(len(T.index_set(p))) + 1j * rng.random(len(T.index_set(p)))
    tl, tn = np.zeros(3), np.array([0.05, -0.07, 0.02])
    pts = rng.random((5, 3)) * 0.1
    lam = T.l2l(beta, tn - tl, p)
    ref = T.evaluate_local(beta, pts - tl, p)
    assert np.max(np.abs(T.evaluate_local(lam, pts - tn, p) - ref)) < 1e-14 * np.max(np.abs(ref))


def _free_setup():
    xyz, q = _cluster()
    sc, tc = np.array([0.15, 0.15, 0.15]), np.array([1.2, 0.3, 0.9])
    rng = np.random.default_rng(2)
    tg = tc + (rng.random((6, 3)) - 0.5) * 0.3
    return xyz, q, sc, tc, tg


def test_m2l_converges_to_direct_sum():
    xyz, q, sc, tc, tg = _free_setup()
    direct = np.array([np.sum(q * h0(K * np.linalg.norm(t - xyz, axis=1))) for t in tg])
    errs = []
    for p in (4, 8, 12):
        b = T.m2l_matrix(tc - sc, K, p) @ T.moments(xyz, q, sc, p)
        errs.append(np.max(np.abs(T.evaluate_local(b, tg - tc, p) - direct)) / np.max(np.abs(direct)))
    assert errs[1] < 1e-2 * errs[0] and errs[2] < 1e-2 * errs[1] and errs[2] < 1e-10


def test_m2l_equals_cartesian_double_taylor():
    """Truncated at the same total degree on each side, the symmetric basis spans the same
    polynomials as the Cartesian one, so TEFMM-II's M2L gives the Cartesian TEFMM-I result
    to rounding, at any p."""
    xyz, q, sc, tc, tg = _free_setup()
    p = 5
    R = tc - sc
    cube = taylor.coefficients(R[0], R[1], R[2], K, 2 * p) / (1j * K)
    f = math.factorial
    multi = [(a, b, n - a - b) for n in range(p + 1) for a in range(n + 1) for b in range(n - a + 1)]
    ref = np.zeros(len(tg), np.complex128)
    for kk in multi:
        tpow = np.prod((tg - tc) ** np.array(kk), axis=1)
        for kp in multi:
            g = tuple(np.add(kk, kp))
            coef = (-1) ** sum(kp) * cube[g] * np.prod([f(x) for x in g]) / np.prod(
                [f(x) for x in kk + kp])
            ref += tpow * coef * np.sum(q * np.prod((xyz - sc) ** np.array(kp), axis=1))
    b = T.m2l_matrix(R, K, p) @ T.moments(xyz, q, sc, p)
    got = T.evaluate_local(b, tg - tc, p)
    np.testing.assert_allclose(got, ref, rtol=1e-11)


@pytest.mark.parametrize("row", list(range(10)))
def test_s_integrals_reproduce_tables_3_1_3_2(row):
    """Tables 3.1/3.2 print (d_x + i d_y)^s d_z^k3 d_z'^k3' u^up_11 / (s! k3! k3'!); from the
    integrals of Eq. symmetricdetable it is 2^s (-1)^s e^{i s phi} S^{s,0}_{k3,k3'}."""
    r = np.loadtxt(GOLD)[row]
    pr, k3, k3p, s = map(int, r[:4])
    ref = r[4] + 1j * r[5]
    t, sp = map(np.array, PAIRS[pr])
    med = Medium((0.8, 1.5, 2.0), (0.0, -2.0))
    rho = math.hypot(t[0] - sp[0], t[1] - sp[1])
    phi = math.atan2(t[1] - sp[1], t[0] - sp[0])
    p = max(k3, k3p, (s + 1) // 2, 1)
    S = T.s_integrals(med, 1, 1, "u", rho, t[2], sp[2], p)
    v = 2 ** s * (-1) ** s * np.exp(1j * s * phi) * S[s, 0, k3, k3p]
    assert abs(v - ref) <= 2e-11 * abs(ref) + 1e-22, (row, v, ref)


@pytest.mark.parametrize("comp", ["u", "d"])
def test_layered_m2l_entries_solve_helmholtz(comp):
    """The reaction component solves the Helmholtz equation in the target variables, so
    (d_x^2 + d_y^2) = -(d_z^2 + k^2):  F(n,2,1) L[(n,2,1)] = -F(n,0,0) L[(n,0,0)]
    - k^2 F(n-2,0,0) L[(n-2,0,0)] for every source index.  This fixes the Bessel order
    M - 2S, the phase and the signs of the assembly."""
    med = Medium((0.8, 1.5, 2.0), (0.0, -1.2))
    p = 4
    tc, sc = np.array([0.5, 0.25, -0.8]), np.array([0.0, 0.1, -0.4])
    L = T.layered_m2l_matrix(med, 1, 1, comp, tc, sc, p)
    im = T.index_map(p)
    kl = med.k[1]
    for n in range(2, p + 1):
        lhs = T.factor(n, 2, 1) * L[im[(n, 2, 1)]]
        rhs = -T.factor(n, 0, 0) * L[im[(n, 0, 0)]] - kl ** 2 * T.factor(n - 2, 0, 0) * L[im[(n - 2, 0, 0)]]
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-12 * np.max(np.abs(rhs)))


@pytest.mark.parametrize("lp,sc", [(1, (0.0, 0.0, -0.4)), (0, (0.1, 0.0, 0.35))])
def test_layered_m2l_converges_to_direct_reaction_sum(lp, sc):
    """Moments -> layered M2L (both target-side components) -> local evaluation against the
    reaction sum by plain J0 quadrature (Eq. greenfuncomponent), same layer and cross layer."""
    med = Medium((0.8, 1.5, 2.0), (0.0, -1.2))
    rng = np.random.default_rng(3)
    hb = 0.125
    sc = np.array(sc)
    tc = np.array([0.5, 0.25, -0.8])
    xyz = sc + (rng.random((12, 3)) - 0.5) * hb
    q = rng.random(12) - 0.5 + 1j * (rng.random(12) - 0.5)
    tg = tc + (rng.random((5, 3)) - 0.5) * hb
    direct = np.array([np.sum(q * reaction_pair(med, 1, lp, np.hypot(t[0] - xyz[:, 0], t[1] - xyz[:, 1]),
                                                t[2], xyz[:, 2], normalization="paper")) for t in tg])
    errs = []
    for p in (3, 5, 7):
        a = T.moments(xyz, q, sc, p)
        b = sum(T.layered_m2l_matrix(med, 1, lp, c, tc, sc, p) @ a for c in ("u", "d"))
        errs.append(np.max(np.abs(T.evaluate_local(b, tg - tc, p) - direct)) / np.max(np.abs(direct)))
    assert errs[1] < 0.05 * errs[0] and errs[2] < 0.05 * errs[1] and errs[2] < 1e-9, errs


def test_delta_terms_depend_on_difference_and_complete_the_reaction():
    """The two cross terms of Eq. symmetricdetable in one layer (target wave up with the
    source's down-going part, and the reverse: the Delta family) depend on z - z' alone,
    which is what lets the GPU tabulate them by offset; with the two Sigma terms they give
    the whole same-layer reaction kernel of the plain J0 quadrature."""
    med = Medium((0.8, 1.5, 2.0), (0.0, -1.2))

    def s00(comp, src, rho, z, zp):
        return T.s_integrals(med, 1, 1, comp, rho, z, zp, 2, src=src)[0, 0, 0, 0]

    for rho, z, zp in [(0.4, -0.3, -0.8), (0.9, -1.0, -0.15)]:
        delta = s00("u", ("d",), rho, z, zp) + s00("d", ("u",), rho, z, zp)
        a = 0.1 if z < -0.5 else -0.1
        shifted = s00("u", ("d",), rho, z + a, zp + a) + s00("d", ("u",), rho, z + a, zp + a)
        other = s00("u", ("d",), rho, z, zp + a)
        sigma = s00("u", ("u",), rho, z, zp) + s00("d", ("d",), rho, z, zp)
        full = reaction_pair(med, 1, 1, np.array([rho]), z, np.array([zp]), normalization="paper")[0]
        assert abs(delta - shifted) <= 1e-12 * abs(delta)
        assert abs(other - s00("u", ("d",), rho, z, zp)) > 1e-3 * abs(delta)  # not constant in z'
        assert abs(sigma + delta - full) <= 1e-10 * abs(full)

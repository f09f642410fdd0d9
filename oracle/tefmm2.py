"""TEFMM-II (Sec. 4): Taylor expansions in the symmetric derivatives, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Index set: (n, m, s) with 0 <= s <= m <= n <= p, ordered by n, then m, then s
(C(p+3, 3) entries).  With u = x + i y:

  alpha~^s_{nm}(r) = u^s conj(u)^(m-s) z^(n-m)                        (Eq. coefMExyz)
  D^s_{nm} = (d_x - i d_y)^s (d_x + i d_y)^(m-s) d_z^(n-m)            (Eq. sysdifferential)
  F(n, m, s) = 2^m (n-m)! s! (m-s)!

Free space (Sec. 4.1):
  source expansion   sum_j q_j h0(k|r - r_j|) ~ sum alpha^s_{nm} D^s_{nm}^ H(r, r_c) / F      (Theorem 4.1)
  moments            alpha^s_{nm} = sum_j q_j alpha~^s_{nm}(r_j - r_c)                        (Eq. mecoefficients)
  local expansion    ~ sum beta^s_{nm} alpha~^s_{nm}(r - r_c^l)                               (Corollary 4.1)
  local coefficients beta^s_{nm} = sum_j q_j D^s_{nm} H(r_c^l, r_j) / F                       (Eq. localexpcoeff2)
  M2L                beta = sum alpha' D^s_{nm} D^{s'}_{n'm'}^ H(r_c^l, r_c) / (F F')        (Eq. M2Ltransop)
                     with D^s_{nm} D^{s'}_{n'm'}^ H = (-1)^n' D^{s+s'}_{n+n', m+m'} H
  M2M                binomial re-centring of the moments                                     (Eq. me2mesymmetricte)
  L2L                re-centring of the local expansion                                      (Eq. le2lesymmetricte)

The derivatives D^s_{nm} h0(k|r|) come from Theorem 4.2: Omega^m_n = h_n(k r) Y^m_n,
D+- = (d_x +- i d_y)/k and D0 = -d_z/k map Omega^m_n to combinations of
Omega^{m+-1}_{n+-1} and Omega^m_{n+-1}, so that
  D^s_{nm} h0(k|r|) = sqrt(4 pi) k^n (-1)^(n-m) (D-)^s (D+)^(m-s) (D0)^(n-m) Omega^0_0(r).
Readings (the printed theorem is not self-consistent; each reading is fixed by
the Cartesian derivatives of h0 in the tests):
  * Y^m_n are the complex spherical harmonics with the Condon-Shortley phase,
    Y^{-m}_n = (-1)^m conj(Y^m_n), m >= 0 as printed (the (-1)^m in front of a
    Ferrers function without that phase);
  * A0, B0 carry the signs opposite to the printed table: A0 = +sqrt(...),
    B0 = -sqrt(...), which is what the theorem's own special case
    D0 Omega^{+-n}_n = Omega^{+-n}_{n+1} / sqrt(2n+3) and D0 = -d_z/k give;
  * the prefactor above (printed as (-1/k)^n sqrt(1/4pi)) is the one that
    follows from h0 = sqrt(4 pi) Omega^0_0 and the definitions of D+-, D0.

Layered media (Sec. 4.2): for a reaction component u (target-side wave a:
'u' = e^{ik_lz (z - d_l)}, 'd' = e^{ik_lz (d_{l-1} - z)}), the M2L entry
  D^s_{nm} D^{s'}_{n'm'}^ u / (F F') = (-1)^(m+s+s') (m+m')! / (s!(m-s)! s'!(m'-s')!)
        e^{i(m+m'-2(s+s'))phi} S^{m+m', s+s'}_{n-m, n'-m'}(rho, z_c^l, z_c)
with the integrals of Eq. symmetricdetable
  S^{M,S}_{a,b}(rho, z, z') = (1/k_l) int k_rho^(M+1) J_{M-2S}(k_rho rho) (+-i k_lz)^a / (2^M M! a! b!)
        P_a(z) / k_lz  d^b sigma~(k_rho, z') / dz'^b  dk_rho,
  d^b sigma~ / dz'^b = (i k_l'z)^b (E_u(z') sigma^{a u} + (-1)^b E_d(z') sigma^{a d}),
(the sign + for the up-going target wave, - for the down-going one), evaluated on
the deformed contour of oracle/sommerfeld.py.  The paper's normalisation is used
(u = G / (i k_l / 4 pi)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .medium import Medium, densities, kz
from .sommerfeld import contour, tail_length, bessel_j, B_CONTOUR


def index_set(p):
    return [(n, m, s) for n in range(p + 1) for m in range(n + 1) for s in range(m + 1)]


def index_map(p):
    return {t: i for i, t in enumerate(index_set(p))}


def factor(n, m, s):
    return 2.0 ** m * math.factorial(n - m) * math.factorial(s) * math.factorial(m - s)


def alpha_tilde(d, p):
    """alpha~^s_{nm}(d) over the index set; d: (3,) or (N, 3) -> (C,) or (N, C)."""
    d = np.asarray(d, np.float64)
    one = d.ndim == 1
    d2 = d.reshape(-1, 3)
    u = d2[:, 0] + 1j * d2[:, 1]
    ub = np.conj(u)
    z = d2[:, 2] + 0j
    out = np.empty((d2.shape[0], len(index_set(p))), np.complex128)
    for i, (n, m, s) in enumerate(index_set(p)):
        out[:, i] = u ** s * ub ** (m - s) * z ** (n - m)
    return out[0] if one else out


def moments(xyz, q, centre, p):
    """alpha^s_{nm} = sum_j q_j alpha~^s_{nm}(r_j - r_c) (Eq. mecoefficients)."""
    A = alpha_tilde(np.asarray(xyz) - np.asarray(centre)[None, :], p)
    return np.asarray(q, np.complex128) @ A


# --- Theorem 4.2 -----------------------------------------------------------------

def _ladder(op, n, m):
    """Coefficients (A, B) of op Omega^m_n = A Omega^{m'}_{n+1} + B Omega^{m'}_{n-1}."""
    if op == "+":
        a = math.sqrt((n + m + 2) * (n + m + 1) / ((2 * n + 1) * (2 * n + 3)))
        b2 = (n - m) * (n - m - 1) / (4 * n * n - 1) if n > 0 else 0.0
        return a, math.sqrt(max(b2, 0.0))
    if op == "-":
        a = -math.sqrt((n - m + 2) * (n - m + 1) / ((2 * n + 1) * (2 * n + 3)))
        b2 = (n + m) * (n + m - 1) / (4 * n * n - 1) if n > 0 else 0.0
        return a, -math.sqrt(max(b2, 0.0))
    a = math.sqrt(((n + 1) ** 2 - m * m) / ((2 * n + 1) * (2 * n + 3)))
    b2 = (n * n - m * m) / (4 * n * n - 1) if n > 0 else 0.0
    return a, -math.sqrt(max(b2, 0.0))


def _apply(E, op, N):
    """op applied to the expansion E[n, m + N] = coefficient of Omega^m_n."""
    dm = {"+": 1, "-": -1, "0": 0}[op]
    out = np.zeros_like(E)
    for n, mi in zip(*np.nonzero(E)):
        m = mi - N
        a, b = _ladder(op, n, m)
        c = E[n, mi]
        if n + 1 < E.shape[0] and abs(m + dm) <= n + 1:
            out[n + 1, mi + dm] += a * c
        if n >= 1 and abs(m + dm) <= n - 1 and b != 0.0:
            out[n - 1, mi + dm] += b * c
    return out


def harmonics(nmax, theta, phi):
    """Y[n, m + nmax] for 0 <= n <= nmax, |m| <= n (Condon-Shortley phase)."""
    Y = np.zeros((nmax + 1, 2 * nmax + 1), np.complex128)
    x = math.cos(theta)
    for n in range(nmax + 1):
        for m in range(n + 1):
            # scipy's Ferrers function already carries (-1)^m
            norm = math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - m) / math.factorial(n + m))
            Y[n, m + nmax] = norm * special.lpmv(m, n, x) * np.exp(1j * m * phi)
            if m:
                Y[n, -m + nmax] = (-1) ** m * np.conj(Y[n, m + nmax])
    return Y


def omega(nmax, d, k):
    """Omega[n, m + nmax] = h_n(k|d|) Y^m_n at the point d (free space, real k)."""
    d = np.asarray(d, np.float64)
    r = float(np.linalg.norm(d))
    theta = math.acos(max(-1.0, min(1.0, d[2] / r)))
    phi = math.atan2(d[1], d[0])
    h = np.array([special.spherical_jn(n, k * r) + 1j * special.spherical_yn(n, k * r) for n in range(nmax + 1)])
    return h[:, None] * harmonics(nmax, theta, phi)


def symmetric_derivatives(d, k, N):
    """D^s_{nm} h0(k|r|) at r = d for all (n, m, s) with n <= N (index_set order),
    from the Theorem 4.2 recurrences applied to Omega^0_0."""
    Om = omega(N, d, k)
    im = index_map(N)
    out = np.empty(len(im), np.complex128)
    E = np.zeros((N + 1, 2 * N + 1))
    E[0, N] = 1.0
    for c in range(N + 1):  # c = n - m applications of D0
        # T[(a, b)] = (D+)^a (D-)^b (D0)^c Omega^0_0 (the operators commute)
        T = {(0, 0): E}
        for tot in range(1, N - c + 1):
            for bb in range(tot + 1):
                a = tot - bb
                T[(a, bb)] = _apply(T[(a - 1, bb)], "+", N) if a > 0 else _apply(T[(a, bb - 1)], "-", N)
        for (a, bb), Eab in T.items():
            m, s = a + bb, bb
            n = c + m
            out[im[(n, m, s)]] = math.sqrt(4 * math.pi) * k ** n * (-1) ** c * np.sum(Eab * Om)
        if c < N:
            E = _apply(E, "0", N)
    return out


# --- free-space expansions and translations -------------------------------------

def theorem41(r, rp, k, p):
    """Truncated Eq. teatrc: sum_{n<=p} alpha~(r') (-1)^n D^s_{nm} H(r, 0) / F."""
    D = symmetric_derivatives(r, k, p)
    A = alpha_tilde(rp, p)
    return sum(A[i] * (-1) ** n * D[i] / factor(n, m, s) for i, (n, m, s) in enumerate(index_set(p)))


def corollary41(r, rp, k, p):
    """Truncated Eq. taylorexploc: sum beta(r') alpha~(r), beta = D^s_{nm} H(0, r') / F."""
    D = symmetric_derivatives(-np.asarray(rp, np.float64), k, p)
    A = alpha_tilde(r, p)
    return sum(A[i] * D[i] / factor(n, m, s) for i, (n, m, s) in enumerate(index_set(p)))


def local_from_sources(tc, xyz, q, k, p):
    """beta^s_{nm} = sum_j q_j D^s_{nm} H(r_c^l, r_j) / F (Eq. localexpcoeff2)."""
    tc = np.asarray(tc, np.float64)
    out = np.zeros(len(index_set(p)), np.complex128)
    F = np.array([factor(*t) for t in index_set(p)])
    for xj, qj in zip(np.asarray(xyz), np.asarray(q)):
        out += qj * symmetric_derivatives(tc - xj, k, p) / F
    return out


def m2l_matrix(R, k, p):
    """L[(n,m,s), (n',m',s')] of Eq. M2Ltransop at R = r_c^l - r_c (free space)."""
    D = symmetric_derivatives(R, k, 2 * p)
    big = index_map(2 * p)
    idx = index_set(p)
    L = np.empty((len(idx), len(idx)), np.complex128)
    for i, (n, m, s) in enumerate(idx):
        for j, (n2, m2, s2) in enumerate(idx):
            L[i, j] = (-1) ** n2 * D[big[(n + n2, m + m2, s + s2)]] / (factor(n, m, s) * factor(n2, m2, s2))
    return L


def m2m(alpha, d, p):
    """Moments about r_c' from moments about r_c, d = r_c - r_c' (Eq. me2mesymmetricte)."""
    im = index_map(p)
    u = d[0] + 1j * d[1]
    ub = np.conj(u)
    dz = d[2]
    f = math.factorial
    out = np.zeros(len(im), np.complex128)
    for (n, m, s), i in im.items():
        acc = 0j
        for s1 in range(s + 1):
            for m1 in range(m - s + 1):
                for n1 in range(n - m + 1):
                    B = (f(s) * f(m - s) * f(n - m) / (f(s1) * f(s - s1) * f(m1) * f(m - s - m1) * f(n1) * f(n - m - n1))
                         * u ** (s - s1) * ub ** (m - s - m1) * dz ** (n - m - n1))
                    acc += B * alpha[im[(n1 + m1 + s1, m1 + s1, s1)]]
        out[i] = acc
    return out


def l2l(beta, d, p):
    """Local coefficients about r~_c^l from those about r_c^l, d = r~_c^l - r_c^l
    (Eq. le2lesymmetricte)."""
    im = index_map(p)
    f = math.factorial
    out = np.zeros(len(im), np.complex128)
    for (n, m, s), i in im.items():
        acc = 0j
        for n1 in range(n, p + 1):
            for m1 in range(m, m + n1 - n + 1):
                if m1 > n1:
                    continue
                for s1 in range(s, s + m1 - m + 1):
                    if s1 > m1 or (m1 - s1) < (m - s) or (n1 - m1) < (n - m):
                        continue
                    C = (f(m1 - s1) * f(s1) * f(n1 - m1)
                         / (f(m1 - s1 - m + s) * f(s1 - s) * f(n1 - m1 - (n - m))))
                    at = (d[0] + 1j * d[1]) ** (s1 - s) * (d[0] - 1j * d[1]) ** ((m1 - m) - (s1 - s)) \
                        * d[2] ** ((n1 - n) - (m1 - m))
                    acc += beta[im[(n1, m1, s1)]] * C * at
        out[i] = acc / (f(n - m) * f(s) * f(m - s))
    return out


def evaluate_local(beta, d, p):
    """sum beta^s_{nm} alpha~^s_{nm}(d) at the points d (Eq. taylorexplocxclfree2)."""
    return alpha_tilde(d, p) @ beta


# --- layered media -----------------------------------------------------------------

def s_integrals(med: Medium, l: int, lp: int, comp: str, rho, z, zp, p, b=B_CONTOUR, src=("u", "d")):
    """S[M, S, a, bb] = S^{M,S}_{a,bb}(rho, z, z') of Eq. symmetricdetable for
    M <= 2p, S <= M, a, bb <= p (zero-filled elsewhere), target-side wave comp;
    src selects the source-side waves kept in sigma~ (both by default)."""
    dt = (z - med.bottom(l)) if comp == "u" else (med.top(l) - z)
    ds = min((zp - med.bottom(lp)) if lp < med.L else np.inf, (med.top(lp) - zp) if lp > 0 else np.inf)
    kmax = float(np.max(med.k))
    t_max = tail_length(dt + ds, 4 * p, kmax)
    nodes, wts, _ = contour(kmax, t_max, b)
    sig = densities(med, lp, nodes)
    kl = kz(med.k[l], nodes)
    klp = kz(med.k[lp], nodes)
    P = np.exp(1j * kl * (z - med.d[l])) if comp == "u" else np.exp(1j * kl * (med.top(l) - z))
    su = sig.get((l, comp, "u"))
    sd = sig.get((l, comp, "d"))
    Eu = np.exp(1j * klp * (zp - med.d[lp])) if lp < med.L else None
    Ed = np.exp(1j * klp * (med.top(lp) - zp)) if lp > 0 else None
    tsign = 1.0 if comp == "u" else -1.0
    J = np.array([bessel_j(nu, nodes * rho) for nu in range(2 * p + 1)])
    out = np.zeros((2 * p + 1, 2 * p + 1, p + 1, p + 1), np.complex128)
    f = math.factorial
    for bb in range(p + 1):
        sv = 0
        if Eu is not None and su is not None and "u" in src:
            sv = sv + Eu * su
        if Ed is not None and sd is not None and "d" in src:
            sv = sv + (-1) ** bb * Ed * sd
        sv = sv * (1j * klp) ** bb
        for a in range(p + 1):
            vert = (tsign * 1j * kl) ** a * P / kl * sv
            for M in range(2 * p + 1):
                base = nodes ** (M + 1) * vert / (2.0 ** M * f(M) * f(a) * f(bb))
                for S in range(M + 1):
                    nu = M - 2 * S
                    Jn = J[nu] if nu >= 0 else (-1) ** (-nu) * J[-nu]
                    out[M, S, a, bb] = np.sum(wts * base * Jn) / med.k[l]
    return out


def layered_m2l_matrix(med: Medium, l: int, lp: int, comp: str, tc, sc, p, b=B_CONTOUR):
    """M2L matrix of Eq. layerm2ltrans for one reaction component, from the S integrals."""
    tc = np.asarray(tc, np.float64)
    sc = np.asarray(sc, np.float64)
    dx, dy = tc[0] - sc[0], tc[1] - sc[1]
    rho = math.hypot(dx, dy)
    phi = math.atan2(dy, dx)
    Sv = s_integrals(med, l, lp, comp, rho, tc[2], sc[2], p, b)
    idx = index_set(p)
    f = math.factorial
    L = np.empty((len(idx), len(idx)), np.complex128)
    for i, (n, m, s) in enumerate(idx):
        for j, (n2, m2, s2) in enumerate(idx):
            M, S = m + m2, s + s2
            L[i, j] = ((-1) ** (m + s + s2) * f(M) / (f(s) * f(m - s) * f(s2) * f(m2 - s2))
                       * np.exp(1j * (M - 2 * S) * phi) * Sv[M, S, n - m, n2 - m2])
    return L

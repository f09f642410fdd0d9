"""Sommerfeld-integral evaluation of the reaction components by contour quadrature.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The reaction part of the layered Green's function (Eq. greenfuncomponent and
Eq. totaldensity, Sec. 2.1) is, for a target at height z in layer l and a
source at z' in layer lp,

    G^r(rho, z, z') = (i/4pi) int_0^inf k_rho J0(k_rho rho) (1/k_lz)
                      sum_{a,b} P_a(z) sigma^{ab}_{l,lp}(k_rho) E_b(z') dk_rho

with P_u(z) = exp(i k_lz (z - d_l)), P_d(z) = exp(i k_lz (d_{l-1} - z)) (this
package references down-going waves at the layer's upper interface, see
oracle/medium.py), E_u(z') = exp(i k_lpz (z' - d_lp)),
E_d(z') = exp(i k_lpz (d_{lp-1} - z')).  The paper's normalisation drops the
factor i k_l / 4pi (Sec. 3.1 and Sec. 3.2), i.e. u = G / (i k_l / 4pi).

Quadrature path (Sec. 4.2, contour deformation): the real k_rho axis is
replaced by  Gamma1: 0 -> -ib,  Gamma2: -ib -> T - ib,  then the vertical
segment T - ib -> T and the real axis T -> t_max.  The paper leaves b and the
truncation unspecified; we take b = 1, T = max(k) + 2 (beyond every branch
point), and t_max from the exponential decay of the integrand.  The integrand is
analytic in the fourth quadrant on the radiation sheet (Im k_z >= 0), so the
deformed path gives the same integral.  Every segment uses composite
Gauss-Legendre panels.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .medium import Medium, densities, kz

B_CONTOUR = 1.0


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w  # on [0, 1]


def tail_length(z_min: float, n_deriv: int = 0, k_max: float = 0.0, tol_log: float = 41.0) -> float:
    """Smallest t with t^n exp(-t Z) below exp(-tol_log) of its peak (Z = z_min > 0)."""
    Z = max(z_min, 1e-3)
    tpk = max(n_deriv / Z, 1.0)
    t = tpk + 1.0
    for _ in range(200):
        val = n_deriv * math.log(t / tpk) - Z * (t - tpk) if n_deriv else -Z * t
        if val < -tol_log:
            break
        t *= 1.1
    return t + k_max


def contour(k_max: float, t_max: float, b: float = B_CONTOUR, order: int = 16,
            width_head: float = 0.5, width_tail: float = 1.0):
    """Nodes and weights (dk_rho included) of the deformed Sommerfeld path.

    Returns (nodes, weights, is_real_tail) where is_real_tail marks nodes on the
    real axis (real k_rho)."""
    T = k_max + 2.0
    u, w = _gl(order)
    nodes, wts, real = [], [], []
    # Gamma1: k = -i s, s in [0, b]
    nodes.append(-1j * b * u); wts.append(-1j * b * w); real.append(np.zeros(order, bool))
    # Gamma2: k = t - i b, t in [0, T]
    npan = int(math.ceil(T / width_head))
    hpan = T / npan
    for p in range(npan):
        t = p * hpan + hpan * u
        nodes.append(t - 1j * b); wts.append(hpan * w + 0j); real.append(np.zeros(order, bool))
    # Gamma3: k = T - i b (1 - u), u in [0,1]
    nodes.append(T - 1j * b * (1.0 - u)); wts.append(1j * b * w); real.append(np.zeros(order, bool))
    # real tail
    if t_max > T:
        npan = int(math.ceil((t_max - T) / width_tail))
        hpan = (t_max - T) / npan
        for p in range(npan):
            t = T + p * hpan + hpan * u
            nodes.append(t + 0j); wts.append(hpan * w + 0j); real.append(np.ones(order, bool))
    return np.concatenate(nodes), np.concatenate(wts), np.concatenate(real)


def bessel_j(n: int, x):
    """J_n(x) for complex x; exact real/imag special cases routed to real routines."""
    x = np.asarray(x, dtype=np.complex128)
    out = np.empty(x.shape, np.complex128)
    re = x.imag == 0
    im = (x.real == 0) & ~re
    gen = ~(re | im)
    if np.any(re):
        xr = x.real[re]
        out[re] = special.j0(xr) if n == 0 else special.jv(n, xr)
    if np.any(im):
        # J_n(i y) = i^n I_n(y)
        yi = x.imag[im]
        out[im] = (1j ** n) * (special.i0(yi) if n == 0 else special.iv(n, yi))
    if np.any(gen):
        out[gen] = special.jv(n, x[gen])
    return out


def _wave_factors(med: Medium, l: int, lp: int, krho, z, zp):
    """Target factors P_a(z) and source factors E_b(z') at the given nodes.

    krho: (K,); z, zp: scalars or arrays broadcastable against (K,)."""
    kl = kz(med.k[l], krho)
    klp = kz(med.k[lp], krho)
    P = {}
    if l < med.L:
        P["u"] = np.exp(1j * kl * (z - med.d[l]))
    if l > 0:
        P["d"] = np.exp(1j * kl * (med.top(l) - z))
    E = {}
    if lp < med.L:
        E["u"] = np.exp(1j * klp * (zp - med.d[lp]))
    if lp > 0:
        E["d"] = np.exp(1j * klp * (med.top(lp) - zp))
    return kl, klp, P, E


def reaction_pair(med: Medium, l: int, lp: int, rho, z, zp, *, normalization="physical",
                  components=("u", "d"), b=B_CONTOUR):
    """Reaction kernel G^r_{l,lp}(rho, z, z') for arrays of pairs (one quadrature per call,
    vectorised over pairs).  ``components`` selects the target-side waves (u: the paper's
    u-up, d: u-down)."""
    rho = np.atleast_1d(np.asarray(rho, np.float64))
    z = np.broadcast_to(np.asarray(z, np.float64), rho.shape)
    zp = np.broadcast_to(np.asarray(zp, np.float64), rho.shape)
    zmin = _min_decay_length(med, l, lp, z, zp)
    t_max = tail_length(zmin, 0, float(np.max(med.k)))
    nodes, wts, _ = contour(float(np.max(med.k)), t_max, b)
    sig = densities(med, lp, nodes)
    kl, klp, P, E = _wave_factors(med, l, lp, nodes[:, None], z[None, :], zp[None, :])
    J = bessel_j(0, nodes[:, None] * rho[None, :])
    acc = np.zeros(J.shape, np.complex128)
    for a in components:
        if a not in P:
            continue
        for bb in E:
            acc += P[a] * sig[(l, a, bb)][:, None] * E[bb]
    integrand = nodes[:, None] * J * acc / kl
    val = np.sum(wts[:, None] * integrand, axis=0)
    if normalization == "physical":
        return 1j / (4.0 * np.pi) * val
    return val / med.k[l]  # paper normalisation (Sec. 3.2): drop i k_l / 4pi


def _min_decay_length(med: Medium, l, lp, z, zp):
    """Smallest total distance to the interfaces that the reaction waves travel
    (sets the exponential decay of the integrand along the real tail)."""
    dz = np.inf
    zt = np.asarray(z)
    zs = np.asarray(zp)
    dist_t = np.minimum(np.where(l < med.L, zt - med.bottom(l), np.inf),
                        np.where(l > 0, med.top(l) - zt, np.inf))
    dist_s = np.minimum(np.where(lp < med.L, zs - med.bottom(lp), np.inf),
                        np.where(lp > 0, med.top(lp) - zs, np.inf))
    dz = float(np.min(dist_t + dist_s))
    return dz


def reaction_derivative_table(med: Medium, l: int, lp: int, r, rp, k3: int, k3p: int, s: int,
                              *, component="u", b=B_CONTOUR):
    """(d/dx + i d/dy)^s d_z^k3 d_z'^k3' u^{component}_{l,lp}(r, r') / (s! k3! k3'!)
    in the paper's normalisation (the quantity of Eq. testderi, Sec. 3.3).

    Uses (d_x + i d_y)^s J0(k rho) = (-k)^s J_s(k rho) e^{i s theta}, theta the
    polar angle of (x - x', y - y') (Sec. 4.1, the Bessel ladder), and moves
    the z' derivative onto the source exponentials (Eq. layermediumdensity)."""
    r = np.asarray(r, np.float64)
    rp = np.asarray(rp, np.float64)
    dx, dy = r[0] - rp[0], r[1] - rp[1]
    rho = math.hypot(dx, dy)
    theta = math.atan2(dy, dx)
    z, zp = float(r[2]), float(rp[2])
    zmin = _min_decay_length(med, l, lp, z, zp)
    t_max = tail_length(zmin, s + k3 + k3p, float(np.max(med.k)))
    nodes, wts, _ = contour(float(np.max(med.k)), t_max, b)
    sig = densities(med, lp, nodes)
    kl, klp, P, E = _wave_factors(med, l, lp, nodes, z, zp)
    a = component
    tgt = P[a] * (1j * kl * (1 if a == "u" else -1)) ** k3
    src = 0
    for bb in E:
        sgn = 1 if bb == "u" else -1
        src = src + sig[(l, a, bb)] * E[bb] * (1j * klp * sgn) ** k3p
    J = bessel_j(s, nodes * rho)
    integrand = nodes * (-nodes) ** s * J * tgt * src / kl
    val = np.sum(wts * integrand) * np.exp(1j * s * theta)
    val /= med.k[l]
    return val / (math.factorial(s) * math.factorial(k3) * math.factorial(k3p))

"""Layered-medium reflection/transmission densities, by a direct interface solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain CPU oracle that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does.

What is computed (Sec. 2.1, the spectral problem and the up/down form of the
solution, Eq. updownspectraldoamin):

  * L+1 horizontal layers, interfaces d_0 > d_1 > ... > d_{L-1}, real wave
    numbers k_0..k_L, layer 0 on top (Sec. 2.1).
  * In the partial Fourier domain the Green's function obeys an ODE in z with
    the transmission conditions  u continuous  and  k * du/dz continuous
    across every interface (Sec. 2.1), plus decay/outgoing behaviour at
    z -> +-inf.
  * The reaction field in target layer m, for a unit source in layer lp, is
        (1/k_mz) [ b_m exp(i k_mz (z - d_m)) + a_m exp(i k_mz (d_{m-1} - z)) ]
    (the common factor  theta = (i/2) exp(-i(kx x' + ky y'))  is dropped).
    b_m is the up-going amplitude, referenced at the layer's lower interface
    exactly as the paper does; a_m is the down-going amplitude, referenced here
    at the layer's UPPER interface so that every exponential stays bounded by 1
    (the paper references it at the lower interface; convert with
    ``to_paper_reference``).
  * The amplitudes are linear in the two incident waves of the source layer,
        E_up = exp(i k_lpz (z' - d_lp))       (wave reaching the lower interface)
        E_dn = exp(i k_lpz (d_{lp-1} - z'))   (wave reaching the upper interface)
    and the densities sigma^{ab}_{m,lp} are the coefficients:
        b_m = sigma^{uu} E_up + sigma^{ud} E_dn,  a_m = sigma^{du} E_up + sigma^{dd} E_dn
    (first letter: target-side wave, second: incident wave), which is the
    paper's sigma notation in Eq. updownspectraldoamin.

The densities are obtained by solving the 2L x 2L linear system of interface
conditions for every k_rho, independently of the closed forms of Appendix A
(those serve as a cross-check in the tests).
"""
from __future__ import annotations

import numpy as np


class Medium:
    """Horizontally layered medium (Sec. 2.1).

    k: wave numbers of layers 0..L (top to bottom), real and positive.
    d: interface heights d_0 > d_1 > ... > d_{L-1}.
    """

    def __init__(self, k, d):
        self.k = np.asarray(k, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.L = len(self.k) - 1
        if len(self.d) != self.L:
            raise ValueError("need len(d) == len(k) - 1")
        if np.any(np.diff(self.d) >= 0):
            raise ValueError("interfaces must be strictly decreasing")
        if np.any(self.k <= 0):
            raise ValueError("wave numbers must be positive")

    def top(self, m):
        """Upper interface of layer m (+inf for the top layer)."""
        return np.inf if m == 0 else self.d[m - 1]

    def bottom(self, m):
        """Lower interface of layer m (-inf for the bottom layer)."""
        return -np.inf if m == self.L else self.d[m]

    def thickness(self, m):
        return self.top(m) - self.bottom(m)

    def layer_of(self, z):
        """Layer index of each height z (Sec. 2.1: d_l < z < d_{l-1})."""
        z = np.asarray(z, dtype=np.float64)
        # number of interfaces strictly above z
        return np.sum(z[..., None] < self.d[None, :], axis=-1) if self.L else np.zeros(z.shape, int)


def kz(k, krho):
    """Vertical wave number sqrt(k^2 - krho^2) on the radiation branch, Im >= 0.

    (Sec. 2.1: k_lz = sqrt(k_l^2 - k_rho^2).)"""
    krho = np.asarray(krho, dtype=np.complex128)
    v = np.sqrt(k * k - krho * krho)
    return np.where(v.imag < 0, -v, v)


def _unknown_index(L):
    """Map (layer, 'b'|'a') -> column of the interface system."""
    idx = {}
    c = 0
    for m in range(L + 1):
        if m < L:
            idx[(m, "b")] = c
            c += 1
        if m > 0:
            idx[(m, "a")] = c
            c += 1
    return idx, c


def densities(med: Medium, lp: int, krho):
    """Reaction densities for a source in layer ``lp``.

    Returns a dict keyed by (m, a, b) with m the target layer, a in 'u','d'
    (target-side wave) and b in 'u','d' (incident wave of the source layer),
    each an array over ``krho``.  Entries that the geometry does not have (no
    up-wave in the bottom layer, no down-wave in the top layer, no E_up for a
    bottom-layer source, no E_dn for a top-layer source) are absent.
    """
    krho = np.atleast_1d(np.asarray(krho, dtype=np.complex128))
    L = med.L
    kk = med.k
    KZ = [kz(kk[m], krho) for m in range(L + 1)]
    idx, n = _unknown_index(L)
    P = krho.shape[0]
    A = np.zeros((P, n, n), dtype=np.complex128)
    incident = []
    if lp < L:
        incident.append("u")
    if lp > 0:
        incident.append("d")
    rhs = np.zeros((P, n, len(incident)), dtype=np.complex128)

    for j in range(L):  # interface z = d_j between layer j (above) and j+1 (below)
        r_val, r_flx = 2 * j, 2 * j + 1
        up, lo = j, j + 1
        # layer above, evaluated at its lower interface
        A[:, r_val, idx[(up, "b")]] += 1.0 / KZ[up]
        A[:, r_flx, idx[(up, "b")]] += kk[up] * 1j
        if up > 0:
            e = np.exp(1j * KZ[up] * med.thickness(up))
            A[:, r_val, idx[(up, "a")]] += e / KZ[up]
            A[:, r_flx, idx[(up, "a")]] += -kk[up] * 1j * e
        # layer below, evaluated at its upper interface (enters with a minus sign)
        A[:, r_val, idx[(lo, "a")]] -= 1.0 / KZ[lo]
        A[:, r_flx, idx[(lo, "a")]] -= -kk[lo] * 1j
        if lo < L:
            e = np.exp(1j * KZ[lo] * med.thickness(lo))
            A[:, r_val, idx[(lo, "b")]] -= e / KZ[lo]
            A[:, r_flx, idx[(lo, "b")]] -= kk[lo] * 1j * e
        # incident wave of the source layer:  value_above - value_below = inc_below - inc_above
        for c, inc in enumerate(incident):
            if inc == "u" and lp == up:      # interface below the source: value E/kz, slope -iE
                rhs[:, r_val, c] -= 1.0 / KZ[lp]
                rhs[:, r_flx, c] -= kk[up] * (-1j)
            if inc == "d" and lp == lo:      # interface above the source: value E/kz, slope +iE
                rhs[:, r_val, c] += 1.0 / KZ[lp]
                rhs[:, r_flx, c] += kk[lo] * (1j)
    sol = np.linalg.solve(A, rhs)
    out = {}
    for m in range(L + 1):
        for c, inc in enumerate(incident):
            if m < L:
                out[(m, "u", inc)] = sol[:, idx[(m, "b")], c]
            if m > 0:
                out[(m, "d", inc)] = sol[:, idx[(m, "a")], c]
    return out


def to_paper_reference(med: Medium, m: int, krho, value, ref: float):
    """Convert a down-going density of target layer m from this module's
    reference (upper interface of layer m) to a down-wave referenced at height
    ``ref``:  a e^{i kz (d_{m-1} - z)} = a' e^{i kz (ref - z)}."""
    k_z = kz(med.k[m], krho)
    return value * np.exp(1j * k_z * (med.top(m) - ref))

"""Taylor coefficients of exp(i k R)/R by truncated multivariate power series.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The Taylor-expansion FMM needs c_g = D^g f(x) / g!  for all multi-indices
|g| <= n, f(x) = exp(i k R)/R, R = |x| (Sec. 3.1, the local expansion
coefficients and the M2L operator), also at points whose third coordinate is
complex (the complex images of Eq. closedformgreen, Sec. 3.3; principal
square root, Re R > 0).  By definition c_g is the coefficient of h^g in the
expansion of f(x + h).  This module computes those coefficients by plain
power-series arithmetic on dense coefficient cubes truncated at total degree
n:  R^2(x + h) is a quadratic polynomial in h, and 1/R, R and exp(i k R) are
univariate series composed with it.  No recurrence is involved, so this is
independent of the derivative recurrence used by the GPU library.
"""
from __future__ import annotations

import math

import numpy as np


def _mask(n):
    i, j, l = np.indices((n + 1, n + 1, n + 1))
    return (i + j + l) <= n


def _mul(A, B, n, mask):
    C = np.zeros_like(A)
    nz = np.argwhere((A != 0) & mask)
    for (i, j, l) in nz:
        C[i:, j:, l:] += A[i, j, l] * B[: n + 1 - i, : n + 1 - j, : n + 1 - l]
    C[~mask] = 0
    return C


def _compose(coef, U, n, mask):
    """sum_m coef[m] U^m, with U of zero constant term."""
    out = np.zeros_like(U)
    out[0, 0, 0] = coef[0]
    P = np.zeros_like(U)
    P[0, 0, 0] = 1.0
    for m in range(1, n + 1):
        P = _mul(P, U, n, mask)
        if coef[m] != 0:
            out += coef[m] * P
    return out


def _binom(alpha, m):
    v = 1.0
    for i in range(m):
        v *= (alpha - i) / (i + 1)
    return v


def coefficients(x, y, zeta, k, n):
    """Dense cube c[a, b, c] = D^(a,b,c) f / (a! b! c!) at (x, y, zeta), entries with
    a + b + c > n set to zero.  f = exp(i k R)/R."""
    mask = _mask(n)
    zeta = complex(zeta)
    R02 = x * x + y * y + zeta * zeta
    R0 = np.sqrt(R02 + 0j)
    if R0.real < 0:
        R0 = -R0
    U = np.zeros((n + 1,) * 3, np.complex128)
    if n >= 1:
        U[1, 0, 0] = 2 * x
        U[0, 1, 0] = 2 * y
        U[0, 0, 1] = 2 * zeta
    if n >= 2:
        U[2, 0, 0] = 1.0
        U[0, 2, 0] = 1.0
        U[0, 0, 2] = 1.0
    V = U / R02  # R^2 = R0^2 (1 + V)
    inv_r = _compose([_binom(-0.5, m) / R0 for m in range(n + 1)], V, n, mask)
    r = _compose([_binom(0.5, m) * R0 for m in range(n + 1)], V, n, mask)
    dr = r.copy()
    dr[0, 0, 0] = 0.0
    e = _compose([np.exp(1j * k * R0) * (1j * k) ** m / math.factorial(m) for m in range(n + 1)],
                 dr, n, mask)
    f = _mul(e, inv_r, n, mask)
    f[~mask] = 0
    return f


def coefficient_list(x, y, zeta, k, n):
    """Coefficients in graded order: |g| = 0, 1, ..., n; within an order by
    decreasing g1, then decreasing g2 (g = (g1, g2, n - g1 - g2))."""
    c = coefficients(x, y, zeta, k, n)
    out = []
    for m in range(n + 1):
        for a in range(m, -1, -1):
            for b in range(m - a, -1, -1):
                out.append(c[a, b, m - a - b])
    return np.array(out)

"""Oracle Taylor coefficients of exp(ikR)/R: closed forms, finite differences, Helmholtz."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.taylor import coefficients


def test_laplace_axis_closed_form():
    """k = 0 on the z axis: D_z^n (1/z) / n! = (-1)^n / z^(n+1)."""
    z = 0.8
    c = coefficients(0.0, 0.0, z, 0.0, 12)
    for n in range(13):
        np.testing.assert_allclose(c[0, 0, n], (-1) ** n / z ** (n + 1), rtol=1e-12)


def test_helmholtz_invariant():
    """sum_i (g_i+1)(g_i+2) c_{g+2e_i} + k^2 c_g = 0 for every |g| <= n-2."""
    k = 1.5
    n = 10
    for pt in [(0.7, -0.4, 1.1), (0.2, 0.3, 0.9 - 0.6j)]:
        c = coefficients(*pt, k, n)
        worst = 0
        for a in range(n - 1):
            for b in range(n - 1 - a):
                for g in range(n - 1 - a - b):
                    lap = ((a + 1) * (a + 2) * c[a + 2, b, g] + (b + 1) * (b + 2) * c[a, b + 2, g]
                           + (g + 1) * (g + 2) * c[a, b, g + 2])
                    scale = max(abs(c[a + 2, b, g]), abs(c[a, b + 2, g]), abs(c[a, b, g + 2]), 1e-300)
                    worst = max(worst, abs(lap + k * k * c[a, b, g]) / scale / (n * n))
        assert worst < 1e-12


@pytest.mark.parametrize("pt", [(0.7, -0.4, 1.1), (0.3, 0.2, 0.6 - 0.5j)])
def test_against_mpmath_derivatives(pt):
    """A few mixed derivatives by mpmath's high-precision numerical differentiation."""
    mp.mp.dps = 40
    k = 1.5
    x0, y0, z0 = pt

    def f(x, y, z):
        R = mp.sqrt(x * x + y * y + z * z)
        if mp.re(R) < 0:
            R = -R
        return mp.exp(1j * k * R) / R

    c = coefficients(x0, y0, z0, k, 7)
    for g in [(1, 0, 0), (0, 2, 1), (3, 1, 2), (2, 2, 3), (0, 0, 7)]:
        d = mp.diff(lambda x, y, z: f(x, y, z), (mp.mpf(x0), mp.mpf(y0), mp.mpc(z0)), g)
        ref = complex(d) / (math.factorial(g[0]) * math.factorial(g[1]) * math.factorial(g[2]))
        np.testing.assert_allclose(c[g], ref, rtol=1e-11)

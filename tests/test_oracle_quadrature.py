"""Oracle quadrature vs the reference values printed in Tables 3.1 and 3.2."""
import os

import numpy as np
import pytest

from oracle.medium import Medium
from oracle.sommerfeld import reaction_derivative_table, reaction_pair

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table_3_1_3_2.txt")
PAIRS = {1: ((0.5, 1.0, -0.5), (0.3, 1.3, -0.5)), 2: ((0.6, 0.3, -1.2), (0.5, 1.0, -0.5))}


def _rows():
    return np.loadtxt(GOLD)


@pytest.mark.parametrize("row", list(range(10)))
def test_table_quadrature_values(row):
    """Sec. 3.3: three layers k = (0.8, 1.5, 2.0), d = 2, the derivatives of u^up_11."""
    r = _rows()[row]
    p, k3, k3p, s = map(int, r[:4])
    ref = r[4] + 1j * r[5]
    med = Medium((0.8, 1.5, 2.0), (0.0, -2.0))
    v = reaction_derivative_table(med, 1, 1, *PAIRS[p], k3, k3p, s)
    # printed values carry 15 significant digits; compare on the complex modulus
    assert abs(v - ref) <= 2e-11 * abs(ref) + 1e-22, (row, v, ref)


def test_derivative_kernel_consistency():
    """(k3, k3', s) = (0, 0, 0) of the derivative routine equals the plain kernel."""
    med = Medium((0.8, 1.5, 2.0), (0.0, -2.0))
    r, rp = PAIRS[2]
    rho = np.hypot(r[0] - rp[0], r[1] - rp[1])
    a = reaction_derivative_table(med, 1, 1, r, rp, 0, 0, 0)
    b = reaction_pair(med, 1, 1, rho, r[2], rp[2], normalization="paper", components=("u",))
    np.testing.assert_allclose(b[0], a, rtol=1e-12)

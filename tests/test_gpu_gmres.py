"""The integral-equation driver: GMRES on (I - tau G) x = b with the FMM as the operator,
through the C ABI (tefmm_gmres), against the oracle's dense solve and by its own residual."""
import os

import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu

K3 = (0.8, 1.5, 2.0)
D3 = (0.0, -1.2)
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TAU = 0.1 * complex(np.cos(np.pi / 4), np.sin(np.pi / 4))


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "expected_gmres.txt")), reason="no stored values")
@pytest.mark.parametrize("precision,p,restart,tol", [("fp64", 16, 30, 1e-6), ("fp64", 16, 5, 1e-6),
                                                     ("fp32", 8, 30, 1e-4)])
def test_gmres_matches_dense_oracle_solve(precision, p, restart, tol):
    """400 point scatterers in the middle layer (Foldy-Lax, tau = 0.1 e^{i pi/4}, condition
    number 9.3), plane-wave right-hand side: GMRES with the FMM operator against the dense
    LAPACK solve of the oracle's kernel matrix; restart 5 exercises the restarts."""
    import torch
    from paper_1902_05875_amd import api, inputs
    rng = np.random.default_rng(180)
    xyz = inputs.cube(rng, 400, inputs.MID_CENTRE)
    b = np.exp(1j * inputs.MEDIUM_K[1] * xyz[:, 0])
    a = np.loadtxt(os.path.join(GOLD, "expected_gmres.txt"))
    xref = a[:, 1] + 1j * a[:, 2]
    f = api.TEFMM(K3, D3, p=p, precision=precision)
    f.set_particles(xyz)
    x, info = f.gmres(torch.from_numpy(b).cuda(), TAU, tol=1e-11 if precision == "fp64" else 1e-7,
                      restart=restart, max_iter=400)
    f.close()
    print(f"{precision} p={p} restart {restart}: {info}")
    assert info["converged"] and info["iterations"] < 400
    check(f"GMRES solution {precision} p={p} restart {restart}", x.cpu().numpy(), xref, tol)


def test_gmres_large_geometry_residual():
    """200,000 scatterers (tau scaled by 400 / N, the same density of scattering), the mixed
    mode: converged to 1e-6 in the FMM's own operator, the residual recomputed by a separate
    evaluation, and an initial guess (the converged x) accepted without steps."""
    import torch
    from paper_1902_05875_amd import api, inputs
    xyz, _ = inputs.workload("c2")
    n = xyz.shape[0]
    b = torch.from_numpy(np.exp(1j * inputs.MEDIUM_K[1] * xyz[:, 0])).cuda()
    tau = TAU * 400 / n
    f = api.TEFMM(K3, D3, p=8, precision="fp32")
    f.set_particles(xyz)
    x, info = f.gmres(b, tau, tol=1e-6, restart=30, max_iter=200)
    r = b - (x - tau * f.evaluate(x))
    res = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    print(f"N = {n}: {info}; residual by a separate evaluation {res:.2e}")
    assert info["converged"] and res < 2e-6
    x2, info2 = f.gmres(b, tau, tol=1e-6, x0=x)
    assert info2["converged"] and info2["iterations"] == 0
    f.close()

"""Write the oracle's expected potentials for the parity tests.

Calls only oracle/ (and the seeded input generators).  Usage:
    python tests/golden/make_expected.py [case ...]
Cases: c1 (N=1000, all targets), c2s (N=200,000, 64 sampled targets),
c4s (N=1,000,000, 16 sampled targets), c4m (the same geometry, 64 sampled targets: 48 uniform + the
16 closest to an interface), c5r (the 500,000-particle geometry with 32 charge vectors, 8 sampled
targets, every vector), c5g (the 16 geometries of the batched workload, 16 sampled targets each), n20k (N=20,000, 128 sampled targets),
c3small (three layers, N=3000, 300 targets), c3s (three layers, N=1,000,000, 6 targets per layer),
c1ns (c1 plus 24 particles at distance 1e-6 from existing ones; the 48 particles of those pairs),
nearif_top, nearif_bottom (N=2000 with 100 particles 0.01-0.02 from one interface; 50 targets),
gmres (the solution of the Foldy-Lax system (I - tau G) x = b for 400 particles, dense solve), ex2small (the Example-2 domain, N=20,000, 64 sampled targets), ex2s (the same domain, N=1,000,000,
16 sampled targets).
Output: tests/golden/expected_<case>.txt with columns  index  re  im  (c5r: index  vector  re  im;
c5g: geometry  index  re  im).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

# one BLAS thread per worker process (the workers already use every core)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.medium import Medium  # noqa: E402
from oracle import direct  # noqa: E402
from paper_1902_05875_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def case_spec(name):
    """(workload name, N, targets) of a parity case."""
    if name == "c1":
        xyz, q = inputs.workload("c1")
        return xyz, q, np.arange(xyz.shape[0])
    if name == "c2s":
        xyz, q = inputs.workload("c2")
        return xyz, q, inputs.sample_targets(xyz, 48, 16, seed=102)
    if name == "c4s":
        xyz, q = inputs.workload("c4")
        return xyz, q, inputs.sample_targets(xyz, 12, 4, seed=104)
    if name == "c4m":
        xyz, q = inputs.workload("c4")
        return xyz, q, inputs.sample_targets(xyz, 48, 16, seed=1040)
    if name == "c5r":
        xyz, q = inputs.workload("c5")
        return xyz, q, inputs.sample_targets(xyz, 6, 2, seed=105)
    if name in ("nearif_top", "nearif_bottom"):
        xyz, q = inputs.near_interface(name.split("_")[1])
        rng = np.random.default_rng(171)
        n = xyz.shape[0]
        near = np.arange(n - 100, n)
        return xyz, q, np.sort(np.concatenate([rng.choice(n - 100, 24, replace=False), near[::4], [n - 1]]))
    if name == "c3small":
        xyz, q = inputs.workload("c3", n=3000)
        rng = np.random.default_rng(130)
        return xyz, q, np.sort(rng.choice(3000, size=300, replace=False))
    if name == "c3s":
        xyz, q = inputs.workload("c3")
        med_d = np.asarray(inputs.MEDIUM_D)
        lay = np.sum(xyz[:, 2:3] < med_d[None, :], axis=1)
        rng = np.random.default_rng(103)
        tg = np.concatenate([rng.choice(np.nonzero(lay == l)[0], size=6, replace=False) for l in range(3)])
        return xyz, q, np.sort(tg)
    if name == "c1ns":
        xyz, q = inputs.workload("c1")
        xyz, q, pairs = inputs.with_close_pairs(xyz, q, 24, 1e-6, seed=140)
        return xyz, q, np.sort(pairs.ravel())
    if name == "n20k":
        xyz, q = inputs.workload("c2", n=20_000)
        return xyz, q, inputs.sample_targets(xyz, 96, 32, seed=120)
    if name == "ex2small":
        xyz, q = inputs.workload("ex2", n=20_000)
        return xyz, q, inputs.sample_targets(xyz, 48, 16, seed=160)
    if name == "ex2s":
        xyz, q = inputs.workload("ex2")
        return xyz, q, inputs.sample_targets(xyz, 12, 4, seed=106)
    raise ValueError(name)


_G = {}


def _work(chunk):
    med = Medium(inputs.MEDIUM_K, inputs.MEDIUM_D)
    xyz, q = _G["xyz"], _G["q"]
    return direct.potential(med, xyz, q, chunk)


def _init(name):
    xyz, q, _ = case_spec(name)
    _G["xyz"], _G["q"] = xyz, q


def _init_geom(g):
    xyz, q = inputs.c5_geometries()[g]
    _G["xyz"], _G["q"] = xyz, q


def run_c5g(procs=None):
    """The 16 batched geometries, 16 targets each (12 uniform + the 4 closest to an interface)."""
    procs = procs or min(8, os.cpu_count() or 1)
    geoms = inputs.c5_geometries()
    rows = []
    t0 = time.time()
    for g, (xyz, q) in enumerate(geoms):
        targets = inputs.sample_targets(xyz, 12, 4, seed=1050 + g)
        chunks = np.array_split(targets, min(len(targets), procs))
        with mp.get_context("fork").Pool(procs, initializer=_init_geom, initargs=(g,)) as pool:
            phi = np.concatenate(pool.map(_work, chunks))
        rows.append(np.column_stack([np.full(len(targets), g), targets, phi.real, phi.imag]))
        print(f"c5g: geometry {g} (N={xyz.shape[0]}) done at {time.time() - t0:.1f} s", flush=True)
    out = os.path.join(HERE, "expected_c5g.txt")
    np.savetxt(out, np.concatenate(rows), fmt=["%d", "%d", "%.17e", "%.17e"],
               header="oracle direct sum (oracle/direct.py), case c5g: the 16 geometries of the batched "
                      "workload; columns: geometry, target index, Re phi, Im phi (physical normalisation)")
    print(f"c5g: {sum(len(r) for r in rows)} targets in {time.time() - t0:.1f} s -> {out}", flush=True)


GMRES_TAU = 0.1 * complex(np.cos(np.pi / 4), np.sin(np.pi / 4))


def gmres_case():
    """400 particles in the mid-layer cube (seed 180) and the plane wave b = e^{i k_1 x}."""
    rng = np.random.default_rng(180)
    xyz = inputs.cube(rng, 400, inputs.MID_CENTRE)
    b = np.exp(1j * inputs.MEDIUM_K[1] * xyz[:, 0])
    return xyz, b


def run_gmres():
    """x = (I - tau G)^-1 b with G the oracle's dense kernel matrix (LAPACK solve)."""
    t0 = time.time()
    xyz, b = gmres_case()
    G = direct.kernel_matrix(Medium(inputs.MEDIUM_K, inputs.MEDIUM_D), xyz)
    A = np.eye(len(b)) - GMRES_TAU * G
    x = np.linalg.solve(A, b)
    out = os.path.join(HERE, "expected_gmres.txt")
    np.savetxt(out, np.column_stack([np.arange(len(b)), x.real, x.imag]), fmt=["%d", "%.17e", "%.17e"],
               header=f"oracle dense solve of (I - tau G) x = b, G = oracle/direct.kernel_matrix, tau = {GMRES_TAU!r}, "
                      f"400 particles (seed 180, mid-layer cube), b = exp(i k_1 x); condition number "
                      f"{np.linalg.cond(A):.3e}; columns: index, Re x, Im x")
    print(f"gmres: dense solve in {time.time() - t0:.1f} s -> {out}", flush=True)


def run(name, procs=None):
    if name == "c5g":
        return run_c5g(procs)
    if name == "gmres":
        return run_gmres()
    xyz, q, targets = case_spec(name)
    procs = procs or min(8, os.cpu_count() or 1)
    chunks = np.array_split(targets, max(1, min(len(targets), procs * 4)))
    t0 = time.time()
    with mp.get_context("fork").Pool(procs, initializer=_init, initargs=(name,)) as pool:
        parts = pool.map(_work, chunks)
    phi = np.concatenate(parts)
    out = os.path.join(HERE, f"expected_{name}.txt")
    if phi.ndim == 2:  # several charge vectors: one row per (target, vector)
        R = phi.shape[1]
        np.savetxt(out, np.column_stack([np.repeat(targets, R), np.tile(np.arange(R), len(targets)),
                                         phi.real.ravel(), phi.imag.ravel()]),
                   fmt=["%d", "%d", "%.17e", "%.17e"],
                   header=f"oracle direct sum (oracle/direct.py), case {name}, N={xyz.shape[0]}, {R} charge "
                          f"vectors; columns: target index, vector, Re phi, Im phi (physical normalisation)")
        print(f"{name}: {len(targets)} targets x {R} vectors in {time.time() - t0:.1f} s -> {out}", flush=True)
        return
    np.savetxt(out, np.column_stack([targets, phi.real, phi.imag]), fmt=["%d", "%.17e", "%.17e"],
               header=f"oracle direct sum (oracle/direct.py), case {name}, N={xyz.shape[0]}; "
                      f"columns: target index, Re phi, Im phi (physical normalisation)")
    print(f"{name}: {len(targets)} targets in {time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["c1", "n20k", "c2s", "c4s"]):
        run(c)

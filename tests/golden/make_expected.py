"""Write the oracle's expected potentials for the parity tests.

Calls only oracle/ (and the seeded input generators).  Usage:
    python tests/golden/make_expected.py [case ...]
Cases: c1 (N=1000, all targets), c2s (N=200,000, 64 sampled targets),
c4s (N=1,000,000, 16 sampled targets), n20k (N=20,000, 128 sampled targets),
c3small (three layers, N=3000, 300 targets), c3s (three layers, N=1,000,000, 6 targets per layer),
c1ns (c1 plus 24 particles at distance 1e-6 from existing ones; the 48 particles of those pairs),
ex2small (the Example-2 domain, N=20,000, 64 sampled targets), ex2s (the same domain, N=1,000,000,
16 sampled targets).
Output: tests/golden/expected_<case>.txt with columns  index  re  im.
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


def run(name, procs=None):
    xyz, q, targets = case_spec(name)
    procs = procs or min(8, os.cpu_count() or 1)
    chunks = np.array_split(targets, max(1, min(len(targets), procs * 4)))
    t0 = time.time()
    with mp.get_context("fork").Pool(procs, initializer=_init, initargs=(name,)) as pool:
        parts = pool.map(_work, chunks)
    phi = np.concatenate(parts)
    out = os.path.join(HERE, f"expected_{name}.txt")
    np.savetxt(out, np.column_stack([targets, phi.real, phi.imag]), fmt=["%d", "%.17e", "%.17e"],
               header=f"oracle direct sum (oracle/direct.py), case {name}, N={xyz.shape[0]}; "
                      f"columns: target index, Re phi, Im phi (physical normalisation)")
    print(f"{name}: {len(targets)} targets in {time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["c1", "n20k", "c2s", "c4s"]):
        run(c)

"""Seeded synthetic workloads (particle positions, charges, target samples).

This module only draws random numbers; it holds none of the method's
arithmetic, so both the GPU path and the CPU oracle tests may use it.

Workload shapes follow the paper's experiments (Sec. 5, Example 1: particles
uniform in unit cubes, one cube per layer; Example 2: an irregular domain
r = 1/2 - a + (a/8)(35 cos^4 t - 30 cos^2 t + 3) filled by rejection from its
bounding cube), re-centred inside the three-layer medium used throughout:
interfaces z = 0 and z = -1.2, wave numbers k = (0.8, 1.5, 2.0) top to bottom.
RNG: numpy default_rng (PCG64); positions are drawn first (N x 3), then the
charges (N x 2 -> real, imaginary), all float64.
"""
from __future__ import annotations

import numpy as np

MEDIUM_K = (0.8, 1.5, 2.0)
MEDIUM_D = (0.0, -1.2)

MID_CENTRE = (0.0, 0.0, -0.6)
TOP_CENTRE = (0.0, 0.0, 0.6)
BOT_CENTRE = (0.0, 0.0, -1.8)


def cube(rng, n, centre, side=1.0):
    c = np.asarray(centre, np.float64)
    return c + side * (rng.random((n, 3)) - 0.5)


def charges(rng, n, n_rhs=1):
    """Complex charges, real and imaginary parts U[-1, 1]."""
    u = rng.uniform(-1.0, 1.0, size=(n, n_rhs, 2))
    q = u[..., 0] + 1j * u[..., 1]
    return q[:, 0] if n_rhs == 1 else q


def irregular(rng, n, centre, a):
    """Example-2 domain r(theta) = 1/2 - a + (a/8)(35 c^4 - 30 c^2 + 3), c = cos(theta),
    sampled by keeping uniform points of the bounding cube that fall inside."""
    out = np.empty((0, 3))
    while out.shape[0] < n:
        p = rng.random((max(2 * n, 1024), 3)) - 0.5
        r = np.linalg.norm(p, axis=1)
        c = np.where(r > 0, p[:, 2] / np.maximum(r, 1e-300), 1.0)
        rb = 0.5 - a + (a / 8.0) * (35 * c**4 - 30 * c**2 + 3)
        out = np.concatenate([out, p[r < rb]])
    return out[:n] + np.asarray(centre, np.float64)


def workload(name: str, n: int | None = None, n_rhs: int | None = None):
    """Return (xyz (N,3), q (N,) or (N,R)) for a named configuration.

    c1: N=1000 mid-layer cube, seed 1.
    c2: N=200,000 mid-layer cube, seed 2.
    c3: N=1,000,000 over three cubes (one per layer), seed 3.
    c4: N=1,000,000 mid-layer cube, seed 4.
    c5: N=500,000 mid-layer cube with 32 charge vectors, seed 5.
    ex2: N=1,000,000 in the Example-2 domain (a = 0.15) centred in the middle layer, seed 6.
    ``n`` overrides the size (same recipe, smaller or larger)."""
    name = name.lower()
    if name == "c1":
        rng = np.random.default_rng(1)
        n = n or 1000
        xyz = cube(rng, n, MID_CENTRE)
        return xyz, charges(rng, n, n_rhs or 1)
    if name == "c2":
        rng = np.random.default_rng(2)
        n = n or 200_000
        xyz = cube(rng, n, MID_CENTRE)
        return xyz, charges(rng, n, n_rhs or 1)
    if name == "c3":
        rng = np.random.default_rng(3)
        n = n or 1_000_000
        n0 = n - 2 * (n // 3)
        n1 = n // 3
        xyz = np.concatenate([cube(rng, n0, TOP_CENTRE), cube(rng, n1, MID_CENTRE),
                              cube(rng, n1, BOT_CENTRE)])
        return xyz, charges(rng, n, n_rhs or 1)
    if name == "c4":
        rng = np.random.default_rng(4)
        n = n or 1_000_000
        xyz = cube(rng, n, MID_CENTRE)
        return xyz, charges(rng, n, n_rhs or 1)
    if name == "c5":
        rng = np.random.default_rng(5)
        n = n or 500_000
        xyz = cube(rng, n, MID_CENTRE)
        return xyz, charges(rng, n, n_rhs or 32)
    if name == "ex2":
        rng = np.random.default_rng(6)
        n = n or 1_000_000
        xyz = irregular(rng, n, MID_CENTRE, 0.15)
        return xyz, charges(rng, n, n_rhs or 1)
    raise ValueError(name)


def near_interface(side, n=2000, n_near=100, seed=170, gap=(0.01, 0.02)):
    """Particles next to one interface of the middle layer: n - n_near uniform in the
    mid-layer cube, n_near with heights gap[0]-gap[1] from the interface (side "top":
    below z = 0; "bottom": above z = -1.2), x and y uniform in [-1/2, 1/2]; then complex
    U[-1, 1] charges.  Returns (xyz, q); the near particles are the last n_near."""
    rng = np.random.default_rng(seed + (side == "bottom"))
    bulk = cube(rng, n - n_near, MID_CENTRE)
    dz = rng.uniform(gap[0], gap[1], n_near)
    z = -dz if side == "top" else -1.2 + dz
    near = np.column_stack([rng.random((n_near, 2)) - 0.5, z])
    return np.concatenate([bulk, near]), charges(rng, n)


def with_close_pairs(xyz, q, n_pairs, dist, seed):
    """Append n_pairs particles, each at distance `dist` (random direction) from a
    randomly chosen existing particle, with fresh U[-1,1] complex charges.  Returns
    (xyz, q, partners): partners[i] = (existing index, new index)."""
    rng = np.random.default_rng(seed)
    n = xyz.shape[0]
    base = rng.choice(n, size=n_pairs, replace=False)
    v = rng.normal(size=(n_pairs, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    new = xyz[base] + dist * v
    qn = charges(rng, n_pairs)
    pairs = np.column_stack([base, n + np.arange(n_pairs)])
    return np.concatenate([xyz, new]), np.concatenate([q, qn]), pairs


def c5_geometries(count=16, seed=50):
    """The 16 independent geometries of the batched workload: sizes log-uniform in
    [1e4, 3e5]; even entries are unit cubes, odd ones Example-2 domains with
    a cycling through 0.05, 0.1, 0.15, all centred at (0, 0, -0.6)."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(1e4), np.log(3e5), size=count))).astype(int)
    geoms = []
    for g, n in enumerate(sizes):
        r = np.random.default_rng(500 + g)
        if g % 2 == 0:
            xyz = cube(r, int(n), MID_CENTRE)
        else:
            a = (0.05, 0.1, 0.15)[(g // 2) % 3]
            xyz = irregular(r, int(n), MID_CENTRE, a)
        geoms.append((xyz, charges(r, int(n), 1)))
    return geoms


def sample_targets(xyz, n_uniform, n_near, seed, interfaces=MEDIUM_D):
    """Fixed target sample: n_uniform indices uniformly at random plus the n_near
    particles closest to any interface (stresses the reaction part)."""
    rng = np.random.default_rng(seed)
    N = xyz.shape[0]
    uni = rng.choice(N, size=min(n_uniform, N), replace=False)
    dist = np.min(np.abs(xyz[:, 2:3] - np.asarray(interfaces)[None, :]), axis=1)
    near = np.argsort(dist, kind="stable")
    near = near[~np.isin(near, uni)][:n_near]
    return np.sort(np.concatenate([uni, near]))

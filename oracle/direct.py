"""Direct O(N^2) evaluation of the layered-media potential, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For every target i in layer l (Eq. totalinteraction, Sec. 3.2):

    phi_i = sum_{j in l, j != i} q_j exp(i k_l R_ij) / (4 pi R_ij)          (free part)
          + sum_{lp} sum_{j in lp} q_j G^r_{l,lp}(rho_ij, z_i, z_j)         (reaction part)

in physical normalisation (the paper's kernels times i k_l / 4pi).  The free
part excludes j = i and the reaction part includes it, as in
Eq. totalinteraction.  The reaction kernel is the Sommerfeld integral of
oracle/sommerfeld.py; for many sources the sum over sources is taken inside
the integral (exact up to rounding, since the quadrature rule does not depend
on the source):

    sum_j q_j G^r = (i/4pi) sum_nodes w k_rho / k_lz sum_{a,b} P_a(z_i)
                    sigma^{ab}(k_rho) [ sum_j q_j J0(k_rho rho_ij) E_b(z_j) ].

The quadrature is the fixed composite Gauss-Legendre rule of
oracle/sommerfeld.contour, with the real tail long enough for the closest
target/source pair of each (l, lp) block.  Sums over sources use numpy's
pairwise summation.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .medium import Medium, densities, kz
from .sommerfeld import contour, tail_length, bessel_j

QUAD_ORDER = 12
HEAD_WIDTH = 1.0
TAIL_WIDTH = 1.5


def free_part(med: Medium, xyz, q, targets, layer=None):
    """Free-space part (k of the common layer), j != i excluded.  q: (N,) or (N, R)."""
    xyz = np.asarray(xyz, np.float64)
    q = np.asarray(q, np.complex128)
    q2 = q.reshape(q.shape[0], -1)
    targets = np.asarray(targets)
    if layer is None:
        layer = med.layer_of(xyz[:, 2])
    out = np.zeros((len(targets), q2.shape[1]), np.complex128)
    for l in range(med.L + 1):
        src = np.nonzero(layer == l)[0]
        tsel = np.nonzero(layer[targets] == l)[0]
        if len(src) == 0 or len(tsel) == 0:
            continue
        k = med.k[l]
        for c0 in range(0, len(tsel), 64):
            tt = tsel[c0:c0 + 64]
            ti = targets[tt]
            d = xyz[ti][:, None, :] - xyz[src][None, :, :]
            R = np.sqrt(np.sum(d * d, axis=-1))
            self_mask = ti[:, None] == src[None, :]
            R = np.where(self_mask, 1.0, R)
            K = np.exp(1j * k * R) / (4.0 * np.pi * R)
            K = np.where(self_mask, 0.0, K)
            out[tt] = K @ q2[src]
    return out.reshape((len(targets),) + q.shape[1:])


def _decay(med: Medium, l, z):
    z = np.asarray(z)
    a = z - med.bottom(l) if l < med.L else np.full(z.shape, np.inf)
    b = med.top(l) - z if l > 0 else np.full(z.shape, np.inf)
    return np.minimum(a, b)


def reaction_part(med: Medium, xyz, q, targets, layer=None, *, target_batch=16,
                  source_chunk=16384, node_block=16, b=1.0):
    """Reaction part, physical normalisation, j = i included.  q: (N,) or (N, R)."""
    xyz = np.asarray(xyz, np.float64)
    q = np.asarray(q, np.complex128)
    q2 = q.reshape(q.shape[0], -1)
    R = q2.shape[1]
    targets = np.asarray(targets)
    if layer is None:
        layer = med.layer_of(xyz[:, 2])
    kmax = float(np.max(med.k))
    out = np.zeros((len(targets), R), np.complex128)
    for l in range(med.L + 1):
        tsel_all = np.nonzero(layer[targets] == l)[0]
        if len(tsel_all) == 0:
            continue
        for lp in range(med.L + 1):
            src = np.nonzero(layer == lp)[0]
            if len(src) == 0:
                continue
            zs = xyz[src, 2]
            min_src = float(np.min(_decay(med, lp, zs)))
            for c0 in range(0, len(tsel_all), target_batch):
                tt = tsel_all[c0:c0 + target_batch]
                ti = targets[tt]
                zt = xyz[ti, 2]
                zmin = float(np.min(_decay(med, l, zt))) + min_src
                t_max = tail_length(zmin, 0, kmax)
                nodes, wts, real = contour(kmax, t_max, b, QUAD_ORDER, HEAD_WIDTH, TAIL_WIDTH)
                sig = densities(med, lp, nodes)
                kl = kz(med.k[l], nodes)
                klp = kz(med.k[lp], nodes)
                P = {}
                if l < med.L:
                    P["u"] = np.exp(1j * kl[:, None] * (zt[None, :] - med.d[l]))
                if l > 0:
                    P["d"] = np.exp(1j * kl[:, None] * (med.top(l) - zt[None, :]))
                bset = (["u"] if lp < med.L else []) + (["d"] if lp > 0 else [])
                # S[b][node, target, rhs] = sum_j q_j J0(k rho_ij) E_b(z_j)
                S = {bb: np.zeros((len(nodes), len(tt), R), np.complex128) for bb in bset}
                for s0 in range(0, len(src), source_chunk):
                    sj = src[s0:s0 + source_chunk]
                    dx = xyz[ti, 0][:, None] - xyz[sj, 0][None, :]
                    dy = xyz[ti, 1][:, None] - xyz[sj, 1][None, :]
                    rho = np.sqrt(dx * dx + dy * dy)
                    zj = xyz[sj, 2]
                    for n0 in range(0, len(nodes), node_block):
                        nn = slice(n0, n0 + node_block)
                        kn = nodes[nn]
                        if np.all(real[nn]):
                            J = special.j0(kn.real[:, None, None] * rho[None, :, :])
                        else:
                            J = bessel_j(0, kn[:, None, None] * rho[None, :, :])
                        for bb in bset:
                            if bb == "u":
                                E = np.exp(1j * klp[nn, None] * (zj[None, :] - med.d[lp]))
                            else:
                                E = np.exp(1j * klp[nn, None] * (med.top(lp) - zj[None, :]))
                            W = E[:, :, None] * q2[sj][None, :, :]          # (n, j, R)
                            if np.isrealobj(J):
                                S[bb][nn] += (np.matmul(J, W.real) + 1j * np.matmul(J, W.imag))
                            else:
                                S[bb][nn] += np.matmul(J, W)
                acc = np.zeros((len(nodes), len(tt), R), np.complex128)
                for a in P:
                    for bb in bset:
                        acc += (P[a] * sig[(l, a, bb)][:, None])[:, :, None] * S[bb]
                integrand = (wts * nodes / kl)[:, None, None] * acc
                out[tt] += 1j / (4.0 * np.pi) * np.sum(integrand, axis=0)
    return out.reshape((len(targets),) + q.shape[1:])


def potential(med: Medium, xyz, q, targets=None, layer=None, **kw):
    """Total physical potential phi at the targets (free + reaction)."""
    xyz = np.asarray(xyz, np.float64)
    if targets is None:
        targets = np.arange(xyz.shape[0])
    if layer is None:
        layer = med.layer_of(xyz[:, 2])
    return free_part(med, xyz, q, targets, layer) + reaction_part(med, xyz, q, targets, layer, **kw)


def rel_l2(approx, exact):
    """Relative 2-norm error, Err_2 of Sec. 5 restricted to the given targets."""
    a = np.asarray(approx).ravel()
    e = np.asarray(exact).ravel()
    return float(np.linalg.norm(a - e) / np.linalg.norm(e))


def rel_max(approx, exact):
    """Err_max of Sec. 5: max_i |phi_i - phi~_i| / |phi_i|."""
    a = np.asarray(approx).ravel()
    e = np.asarray(exact).ravel()
    return float(np.max(np.abs(a - e) / np.abs(e)))


def kernel_matrix(med: Medium, xyz, layer=None):
    """The dense matrix G of the sum (Eq. totalinteraction): G[i, j] = free-space kernel
    e^{ik_l R}/(4 pi R) for j != i in the same layer (0 on the diagonal) plus the reaction
    kernel G^r_{l_i l_j} (the diagonal included), physical normalisation, from the pairwise
    Sommerfeld quadrature of sommerfeld.reaction_pair.  For small N (N^2 pairs)."""
    from .sommerfeld import reaction_pair
    xyz = np.asarray(xyz, np.float64)
    if layer is None:
        layer = med.layer_of(xyz[:, 2])
    N = xyz.shape[0]
    G = np.zeros((N, N), np.complex128)
    for l in range(med.L + 1):
        ti = np.nonzero(layer == l)[0]
        for lp in range(med.L + 1):
            sj = np.nonzero(layer == lp)[0]
            if len(ti) == 0 or len(sj) == 0:
                continue
            T, S = np.meshgrid(ti, sj, indexing="ij")
            T, S = T.ravel(), S.ravel()
            rho = np.hypot(xyz[T, 0] - xyz[S, 0], xyz[T, 1] - xyz[S, 1])
            for c0 in range(0, len(T), 2048):  # pairs in chunks (nodes x pairs arrays)
                c = slice(c0, c0 + 2048)
                G[T[c], S[c]] = reaction_pair(med, l, lp, rho[c], xyz[T[c], 2], xyz[S[c], 2])
            T, S = np.meshgrid(ti, sj, indexing="ij")
            if l == lp:
                R = np.linalg.norm(xyz[T] - xyz[S], axis=-1)
                free = np.exp(1j * med.k[l] * np.where(R > 0, R, 1.0)) / (4 * np.pi * np.where(R > 0, R, 1.0))
                G[T, S] += np.where(T == S, 0.0, free)
    return G

"""Seeded Bloch orbitals for Brillouin-zone sampling.

psi_{jk}(x) = exp(i 2 pi sum_a k_a x_a / (n_a h_a)) u_{jk}(x) on the grid nodes
x_a = i_a h_a, with u_{jk} a periodic sum of Gaussians with complex N(0, 1)
weights (a pool of shared centres, minimum-image distance on periodic axes),
orthonormal per k under (u, v)_h = h1 h2 h3 sum conj(u) v.  k is given in
reduced coordinates (fractions of the reciprocal lattice vectors); Dirichlet
axes take k_a = 0.  Layout: psi[k, j, i3, i2, i1].
"""
from __future__ import annotations

import math

import numpy as np

from .orbitals import _axis_profile


def orthonormalise_cgs2_complex(Q, dV):
    """Classical Gram-Schmidt applied twice, in index order, under
    (u, v)_h = dV sum conj(u) v (rows of Q, modified in place and returned)."""
    m = Q.shape[0]
    for i in range(m):
        for _ in range(2):
            if i > 0:
                c = dV * (np.conj(Q[:i]) @ Q[i])
                Q[i] -= c @ Q[:i]
        Q[i] /= math.sqrt(dV * float(np.real(np.vdot(Q[i], Q[i]))))
    return Q


def bloch_orbitals(n, h, bc, kpts, norb, seed, n_centres):
    n1, n2, n3 = n
    N = n1 * n2 * n3
    rng = np.random.default_rng(seed)
    K = n_centres
    u = rng.random((K, 3))
    widths = rng.uniform(0.8, 1.5, K)
    centres = np.empty((K, 3))
    for ax in range(3):
        length = (n[ax] - 1) * h[ax]
        if bc[ax] == "periodic":
            centres[:, ax] = u[:, ax] * n[ax] * h[ax]
        else:
            lo, hi = 4.0, length - 4.0
            if hi <= lo:
                lo = hi = 0.5 * length
            centres[:, ax] = lo + u[:, ax] * (hi - lo)
    G = np.empty((K, N))
    for k in range(K):
        gx = _axis_profile(n1, h[0], bc[0], centres[k, 0], widths[k])
        gy = _axis_profile(n2, h[1], bc[1], centres[k, 1], widths[k])
        gz = _axis_profile(n3, h[2], bc[2], centres[k, 2], widths[k])
        G[k] = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).ravel()
    dV = h[0] * h[1] * h[2]
    out = np.empty((len(kpts), norb, n3, n2, n1), dtype=np.complex128)
    i1 = np.arange(n1)
    i2 = np.arange(n2)
    i3 = np.arange(n3)
    for kk, kv in enumerate(kpts):
        for a in range(3):
            if bc[a] != "periodic" and float(kv[a]) != 0.0:
                raise ValueError("a Dirichlet axis takes no wavevector component")
        A = rng.standard_normal((norb, K)) + 1j * rng.standard_normal((norb, K))
        U = orthonormalise_cgs2_complex(A @ G, dV)
        ramp = (np.exp(2j * math.pi * kv[2] * i3 / n3)[:, None, None] *
                np.exp(2j * math.pi * kv[1] * i2 / n2)[None, :, None] *
                np.exp(2j * math.pi * kv[0] * i1 / n1)[None, None, :])
        out[kk] = U.reshape(norb, n3, n2, n1) * ramp
    return out

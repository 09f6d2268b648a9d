"""Seeded Gaussian-sum orbitals on a uniform finite-difference grid.

The paper's own systems (a silicon nanocluster, bulk LiH and MnO2, liquid
water) need structures, pseudopotentials and converged orbitals that are not
available here.  These synthetic orbitals stand in for them: smooth,
localised-to-delocalised fields with the grid sizes and orbital counts of the
paper's workloads, orthonormal under the grid inner product
(u, v)_h = h1 h2 h3 sum_r u(r) v(r).

Array layout: ``psi[j, i3, i2, i1]`` (C order), i.e. flat index
``j*N + i1 + n1*(i2 + n2*i3)`` with axis 1 fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: tuple            # (n1, n2, n3) grid points per axis
    h: tuple            # (h1, h2, h3) spacing in bohr
    order: int          # FD order of the second-derivative stencil
    bc: tuple           # per axis: "dirichlet" | "periodic"
    kernel: str         # "coulomb" | "erfc"
    omega: float        # screening parameter (bohr^-1); ignored for coulomb
    norb: int
    occ: float          # occupation of every orbital
    seed: int
    n_centres: int      # Gaussians in the pool
    shared: bool        # True: every orbital mixes the whole pool (N(0,1) weights)
                        # False: each orbital owns n_centres//norb Gaussians (U(-1,1) weights)
    storage: str = "f64"

    @property
    def N(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def npairs(self) -> int:
        return self.norb * (self.norb + 1) // 2

    @property
    def dV(self) -> float:
        return self.h[0] * self.h[1] * self.h[2]

    def flops_per_pair(self) -> int:
        """Six mode products, 2*N*n_k flops each (forward and inverse)."""
        return 4 * self.N * sum(self.n)


D, P = "dirichlet", "periodic"

WORKLOADS = {
    # 8 orbitals, 32^3 all-Dirichlet, h=0.3, unscreened kernel, 36 pair solves.
    "dirichlet32_coulomb": Workload("dirichlet32_coulomb", (32, 32, 32), (0.3,) * 3, 12,
                                    (D, D, D), "coulomb", 0.0, 8, 2.0, 1, 32, False),
    # 128 orbitals, 96^3 periodic, h=0.35, erfc omega=0.106, 8256 pair solves.
    "periodic96_erfc": Workload("periodic96_erfc", (96, 96, 96), (0.35,) * 3, 12,
                                (P, P, P), "erfc", 0.106, 128, 2.0, 2, 256, True),
    # 256 orbitals, 144^3 periodic, h=0.3, erfc, FP32 orbital storage.
    "periodic144_erfc_f32": Workload("periodic144_erfc_f32", (144, 144, 144), (0.3,) * 3, 12,
                                     (P, P, P), "erfc", 0.106, 256, 2.0, 5, 512, True, "f32"),
    # Ragged batch of six systems (h=0.3, order 12).
    "ragged_a_dirichlet48": Workload("ragged_a_dirichlet48", (48, 48, 48), (0.3,) * 3, 12,
                                     (D, D, D), "coulomb", 0.0, 16, 2.0, 41, 32, True),
    "ragged_b_periodic60x60x72": Workload("ragged_b_periodic60x60x72", (60, 60, 72), (0.3,) * 3, 12,
                                          (P, P, P), "erfc", 0.106, 32, 2.0, 42, 64, True),
    "ragged_c_dirichlet80": Workload("ragged_c_dirichlet80", (80, 80, 80), (0.3,) * 3, 12,
                                     (D, D, D), "coulomb", 0.0, 48, 2.0, 43, 96, True),
    "ragged_d_periodic96": Workload("ragged_d_periodic96", (96, 96, 96), (0.3,) * 3, 12,
                                    (P, P, P), "erfc", 0.106, 64, 2.0, 44, 128, True),
    "ragged_e_slab120x120x60": Workload("ragged_e_slab120x120x60", (120, 120, 60), (0.3,) * 3, 12,
                                        (P, P, D), "erfc", 0.106, 96, 2.0, 45, 192, True),
    "ragged_f_periodic112": Workload("ragged_f_periodic112", (112, 112, 112), (0.3,) * 3, 12,
                                     (P, P, P), "erfc", 0.106, 128, 2.0, 46, 256, True),
    # Small cases that still span several 16-point tiles with ragged tails on
    # every axis; used by the parity tests.
    "mixed40x36x44_erfc": Workload("mixed40x36x44_erfc", (40, 36, 44), (0.35, 0.3, 0.4), 12,
                                   (P, D, P), "erfc", 0.106, 6, 2.0, 7, 24, True),
    "dirichlet20x27x34_coulomb": Workload("dirichlet20x27x34_coulomb", (20, 27, 34), (0.4, 0.35, 0.3), 8,
                                          (D, D, D), "coulomb", 0.0, 5, 2.0, 8, 20, False),
}

RAGGED_BATCH = tuple(k for k in WORKLOADS if k.startswith("ragged_"))


def _axis_profile(n, h, bc, centre, width):
    """exp(-d^2 / (2 s^2)) along one axis, minimum image on periodic axes."""
    x = np.arange(n, dtype=np.float64) * h
    d = x - centre
    if bc == "periodic":
        period = n * h
        d = d - period * np.round(d / period)
    return np.exp(-(d * d) / (2.0 * width * width))


def gaussian_orbitals(n, h, bc, norb, seed, n_centres, shared, chunk=32):
    """Draw norb Gaussian-sum orbitals (not yet orthonormal).

    Random draws, in this order, from ``numpy.random.default_rng(seed)``:
    centres U(0,1)^(K x 3) mapped per axis, widths U(0.8, 1.5)^K, then the
    weights: N(0,1)^(norb x K) when ``shared``, else U(-1,1)^(norb x K/norb)
    with orbital j owning Gaussians j*K/norb .. (j+1)*K/norb - 1.
    Dirichlet axes keep centres at least 4 bohr inside the grid.
    """
    n1, n2, n3 = n
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
    if shared:
        A = rng.standard_normal((norb, K))
    else:
        per = K // norb
        if per * norb != K:
            raise ValueError("n_centres must be a multiple of norb when not shared")
        A = np.zeros((norb, K))
        w = rng.uniform(-1.0, 1.0, (norb, per))
        for j in range(norb):
            A[j, j * per:(j + 1) * per] = w[j]
    N = n1 * n2 * n3
    psi = np.zeros((norb, N))
    for k0 in range(0, K, chunk):
        k1 = min(K, k0 + chunk)
        G = np.empty((k1 - k0, N))
        for k in range(k0, k1):
            gx = _axis_profile(n1, h[0], bc[0], centres[k, 0], widths[k])
            gy = _axis_profile(n2, h[1], bc[1], centres[k, 1], widths[k])
            gz = _axis_profile(n3, h[2], bc[2], centres[k, 2], widths[k])
            G[k - k0] = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).ravel()
        psi += A[:, k0:k1] @ G
    return psi.reshape(norb, n3, n2, n1)


def orthonormalise_cgs2(psi, dV, block=16):
    """Classical Gram-Schmidt with one re-orthogonalisation pass, in index
    order, under (u, v)_h = dV * sum(u v).  Earlier blocks are projected out
    with matrix products; inside a block it runs one vector at a time."""
    shape = psi.shape
    Q = np.array(psi.reshape(shape[0], -1), dtype=np.float64, copy=True)
    m = Q.shape[0]
    for b0 in range(0, m, block):
        b1 = min(m, b0 + block)
        if b0 > 0:
            for _ in range(2):
                C = dV * (Q[:b0] @ Q[b0:b1].T)
                Q[b0:b1] -= C.T @ Q[:b0]
        for i in range(b0, b1):
            if i > b0:
                for _ in range(2):
                    c = dV * (Q[b0:i] @ Q[i])
                    Q[i] -= c @ Q[b0:i]
            nrm = math.sqrt(dV * float(Q[i] @ Q[i]))
            Q[i] /= nrm
    return Q.reshape(shape)


def make_workload(w: Workload | str):
    """Return (workload, psi, occ) with psi orthonormal, stored as w.storage."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    psi = gaussian_orbitals(w.n, w.h, w.bc, w.norb, w.seed, w.n_centres, w.shared)
    psi = orthonormalise_cgs2(psi, w.dV)
    if w.storage == "f32":
        psi = psi.astype(np.float32)
    occ = np.full(w.norb, w.occ, dtype=np.float64)
    return w, psi, occ


def random_fields(n, batch, seed, dtype=np.float64):
    """Batch of N(0,1) fields of shape (batch, n3, n2, n1)."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    return rng.standard_normal((batch, n3, n2, n1)).astype(dtype)

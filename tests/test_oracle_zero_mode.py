"""Pins of the zero-mode value of the unscreened kernel on all-periodic grids
(Sec. IV: for 3D bulk systems the k = q problem has the constant mode, whose
value the paper takes from auxiliary functions; here it is an input chi).

  * Exactly one mode (the constant) is replaced, and the result is the
    zero-mean Poisson solution plus chi times the mean of rho: the sparse
    residual (-L) phi = 4 pi (rho - mean rho) holds, mean(phi) = chi mean(rho).
  * phi is affine in chi with slope mean(rho) at every node.
  * The exchange energy is affine in chi with the slope written from the
    definition: dE/dchi = -1/4 sum_{ij} occ_i occ_j dV N mean(rho_ij)^2.
  * k-points: only the k = q pairs see chi (k-points distinct modulo the
    reciprocal lattice); time reversal and the energy identity still hold;
    k - q a reciprocal lattice vector is the zero mode again.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as orc
from synth import bloch_orbitals, make_workload

P3 = ("periodic",) * 3


def _sparse_L(n, h, order):
    L = [sp.csr_matrix(orc.laplacian_1d(n[a], h[a], order, "periodic")) for a in range(3)]
    I = [sp.identity(n[a], format="csr") for a in range(3)]
    return (sp.kron(I[2], sp.kron(I[1], L[0])) + sp.kron(I[2], sp.kron(L[1], I[0]))
            + sp.kron(L[2], sp.kron(I[1], I[0]))).tocsr()


@pytest.mark.parametrize("order", [2, 8, 12])
def test_zero_mode_solve(order):
    n, h = (9, 8, 10), (0.5, 0.45, 0.4)
    grid = orc.make_grid(n, h, order, P3)
    F = orc.kernel_values_zero_mode(grid.lam_sum(), "coulomb", 0.0, 3.7)
    assert np.sum(F == 3.7) == 1 and np.all(np.isfinite(F))
    rng = np.random.default_rng(order)
    rho = rng.standard_normal((n[2], n[1], n[0])) + 0.3
    phi = orc.apply_fL(rho, grid, "coulomb", F=F)
    res = -(_sparse_L(n, h, order) @ phi.ravel()) - 4 * math.pi * (rho - rho.mean()).ravel()
    assert np.max(np.abs(res)) <= 1e-10 * 4 * math.pi * np.max(np.abs(rho))
    assert abs(phi.mean() - 3.7 * rho.mean()) <= 1e-12 * np.max(np.abs(phi))
    # affine in chi, slope mean(rho)
    F2 = orc.kernel_values_zero_mode(grid.lam_sum(), "coulomb", 0.0, -1.2)
    phi2 = orc.apply_fL(rho, grid, "coulomb", F=F2)
    assert np.allclose(phi - phi2, (3.7 + 1.2) * rho.mean(), atol=1e-12 * np.max(np.abs(phi)))


def test_zero_mode_exchange_energy_slope():
    w, psi, occ = make_workload("dirichlet20x27x34_coulomb")
    n, h = (10, 9, 8), (0.5, 0.5, 0.5)
    psi = np.array([np.resize(p, (n[2], n[1], n[0])) for p in psi[:3]])
    occ = np.array([2.0, 1.0, 0.5])
    grid = orc.make_grid(n, h, 4, P3)
    _, e1 = orc.exchange(psi, occ, grid, "coulomb", zero_mode=1.0)
    _, e2 = orc.exchange(psi, occ, grid, "coulomb", zero_mode=3.0)
    N = n[0] * n[1] * n[2]
    dV = grid.dV
    slope = -0.25 * sum(occ[i] * occ[j] * dV * N * float(np.mean(psi[i] * psi[j])) ** 2
                        for i in range(3) for j in range(3))
    assert abs((e2 - e1) / 2.0 - slope) <= 1e-10 * abs(slope)
    with pytest.raises(ZeroDivisionError):
        orc.exchange(psi, occ, grid, "coulomb")


def test_zero_mode_with_k_points():
    n, h, order = (8, 7, 6), (0.5, 0.5, 0.5), 4
    # distinct modulo the reciprocal lattice (0.5 and -0.5 would be one point,
    # whose pairs also carry the zero mode)
    kpts = [(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)]
    wk = [0.5, 0.5]
    occ = [[0.9, 0.6], [0.9, 0.6]]
    psi = bloch_orbitals(n, h, P3, kpts[:1], 2, seed=9, n_centres=4)
    psi = np.concatenate([psi, np.conj(psi)])  # psi_{-k} = conj(psi_k)
    vx1, e1 = orc.exchange_bloch(psi, kpts, wk, occ, n, h, order, P3, "coulomb", zero_mode=2.0)
    vx2, e2 = orc.exchange_bloch(psi, kpts, wk, occ, n, h, order, P3, "coulomb", zero_mode=5.0)
    dV = h[0] * h[1] * h[2]
    N = n[0] * n[1] * n[2]
    # only the k = q pairs see chi: slope from the definition
    assert orc.bloch_phases(np.subtract(kpts[0], kpts[1]), P3)[0] != 0.0
    slope = 0.0
    for k in range(2):
        for a in range(2):
            for b in range(2):
                m = np.mean(np.conj(psi[k, b]) * psi[k, a])
                slope -= 0.25 * wk[k] ** 2 * occ[k][a] * occ[k][b] * dV * N * abs(m) ** 2
    assert abs((e2 - e1) / 3.0 - slope) <= 1e-10 * abs(slope)
    # k - q = (1, 0, 0): the same operator as k = q, zero mode included
    g0 = orc.make_grid_bloch(n, h, order, P3, (0.0, 0.0, 0.0))
    g1 = orc.make_grid_bloch(n, h, order, P3, (2 * math.pi, 0.0, 0.0))
    rho = np.conj(psi[0, 0]) * psi[0, 1]
    a = orc.apply_fL_bloch(rho, g0, "coulomb", zero_mode=2.0)
    b = orc.apply_fL_bloch(rho, g1, "coulomb", zero_mode=2.0)
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(a))
    # time reversal and the energy identity
    assert np.max(np.abs(vx1[1] - np.conj(vx1[0]))) <= 1e-12 * np.max(np.abs(vx1[0]))
    ev = 0.25 * sum(wk[k] * occ[k][b] * dV * np.vdot(psi[k, b], vx1[k, b]).real
                    for k in range(2) for b in range(2))
    assert abs(ev - e1) <= 1e-12 * abs(e1)

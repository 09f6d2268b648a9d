"""Pins of the oracle's non-orthogonal cells (Sec. III, closing remark: with
periodic or Bloch-periodic conditions on every axis the Laplacian with mixed
derivatives keeps a shared 1-D eigenbasis).

  * First-derivative weights: Fornberg's published table, the closed form
    d_p = (-1)^(p+1) (m!)^2 / (p (m-p)! (m+p)!), exactness on polynomials.
  * D_k(theta) is anti-Hermitian and its Bloch plane waves are eigenvectors
    with eigenvalue i s(kappa) / h, s(kappa) = 2 sum_p d_p sin(p kappa).
  * The metric of a hexagonal cell has the closed form g = [[4/3, 2/3, 0],
    [2/3, 4/3, 0], [0, 0, 1]], |det E| = sqrt(3)/2; rotations give g = I.
  * The dense lattice-coordinate Laplacian acts on plane waves with the
    closed-form symbol, approaches -|G|^2 of the Cartesian reciprocal vector
    as the order grows, is Hermitian and negative semidefinite, and reduces
    to the Kronecker route of apply_fL_bloch for an orthogonal cell.
  * Exchange: reduces to exchange_bloch on an orthogonal cell;
    E_x = 1/4 sum_k w_k sum_n occ <psi_nk, Vx psi_nk>_h with the cell's
    volume element; the unscreened solve satisfies (-L) phi = 4 pi rho.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc
from synth import bloch_orbitals

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P3 = ("periodic",) * 3
HEX = [[1.0, 0.0, 0.0], [-0.5, math.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.0]]
SKEW = [[1.0, 0.0, 0.0], [0.3, 1.0, 0.0], [0.2, -0.25, 1.0]]


def _golden_d1():
    out = {}
    with open(os.path.join(GOLDEN, "fd_weights_centred_d1.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                order, vals = line.split(":")
                out[int(order)] = [Fraction(v) for v in vals.split()]
    return out


def test_d1_weights_match_textbook_table():
    for order, ref in _golden_d1().items():
        assert orc.fd_weights_d1(order) == ref, order


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 16, 24])
def test_d1_weights_closed_form_and_polynomial_exactness(order):
    m = order // 2
    d = orc.fd_weights_d1(order)
    for p in range(1, m + 1):
        ref = Fraction((-1) ** (p + 1) * math.factorial(m) ** 2,
                       p * math.factorial(m - p) * math.factorial(m + p))
        assert d[p - 1] == ref
    # exact derivative of x^k at x = 0 for k <= order (h = 1)
    for k in range(order + 1):
        val = sum(d[p - 1] * (Fraction(p) ** k - Fraction(-p) ** k) for p in range(1, m + 1))
        assert val == (1 if k == 1 else 0), k
    # and not for k = order + 1 (the order is exact, not higher)
    k = order + 1
    assert sum(d[p - 1] * (Fraction(p) ** k - Fraction(-p) ** k) for p in range(1, m + 1)) != 0


@pytest.mark.parametrize("n,order,theta", [(9, 4, 0.7), (12, 12, -2.2), (6, 2, math.pi), (16, 8, 0.0)])
def test_bloch_derivative_spectrum(n, order, theta):
    h = 0.4
    D = orc.derivative_1d_bloch(n, h, order, theta)
    assert np.allclose(D, -D.conj().T, atol=1e-14)
    d = [float(x) for x in orc.fd_weights_d1(order)]
    x = np.arange(n)
    for j in range(n):
        kappa = (2 * math.pi * j + theta) / n
        v = np.exp(1j * kappa * x)
        s = 2.0 * sum(d[p - 1] * math.sin(p * kappa) for p in range(1, order // 2 + 1))
        assert np.allclose(D @ v, 1j * s / h * v, atol=1e-12)


def test_cell_metric_closed_forms():
    g, jac = orc.cell_metric(HEX)
    assert np.allclose(g, [[4 / 3, 2 / 3, 0], [2 / 3, 4 / 3, 0], [0, 0, 1]], atol=1e-14)
    assert abs(jac - math.sqrt(3) / 2) < 1e-14
    # any length of the direction rows
    g2, jac2 = orc.cell_metric(np.array(HEX) * np.array([[2.0], [0.5], [3.0]]))
    assert np.allclose(g2, g) and abs(jac2 - jac) < 1e-14
    # a rotated orthonormal frame is an orthogonal cell
    c, s = math.cos(0.4), math.sin(0.4)
    R = [[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]]
    g3, jac3 = orc.cell_metric(R)
    assert np.allclose(g3, np.eye(3), atol=1e-14) and abs(jac3 - 1.0) < 1e-14


def _symbol_cell(n, h, order, lattice, theta, m3):
    g, _ = orc.cell_metric(lattice)
    w = [float(x) for x in orc.fd_weights(order)]
    d = [float(x) for x in orc.fd_weights_d1(order)]
    M = order // 2
    kap = [(2 * math.pi * m3[a] + theta[a]) / n[a] for a in range(3)]
    s2 = [(w[0] + 2 * sum(w[p] * math.cos(p * kap[a]) for p in range(1, M + 1))) / h[a] ** 2
          for a in range(3)]
    s1 = [2 * sum(d[p - 1] * math.sin(p * kap[a]) for p in range(1, M + 1)) / h[a] for a in range(3)]
    # L e^{i kappa.i} = [sum g_aa s2_a + sum_{a != b} g_ab (i s1_a)(i s1_b)] e^{i kappa.i}
    val = sum(g[a, a] * s2[a] for a in range(3))
    val -= sum(g[a, b] * s1[a] * s1[b] for a in range(3) for b in range(3) if a != b)
    return val, kap


@pytest.mark.parametrize("lattice", [HEX, SKEW])
def test_cell_laplacian_symbol_on_plane_waves(lattice):
    n, h, order = (5, 4, 6), (0.5, 0.45, 0.4), 4
    theta = (0.6, -1.1, 2.0)
    L = orc.laplacian_cell(n, h, order, lattice, theta)
    assert np.allclose(L, L.conj().T, atol=1e-12)
    ev = np.linalg.eigvalsh(-L)
    assert ev.min() >= -1e-10 * ev.max()
    i1, i2, i3 = np.arange(n[0]), np.arange(n[1]), np.arange(n[2])
    for m3 in [(0, 0, 0), (1, 0, 0), (2, 3, 1), (4, 1, 5), (3, 2, 2)]:
        val, kap = _symbol_cell(n, h, order, lattice, theta, m3)
        v = (np.exp(1j * kap[2] * i3)[:, None, None] * np.exp(1j * kap[1] * i2)[None, :, None]
             * np.exp(1j * kap[0] * i1)[None, None, :]).ravel()
        assert np.allclose(L @ v, val * v, atol=1e-10 * abs(L).max())


def test_cell_laplacian_approaches_the_continuum_on_reciprocal_vectors():
    # a plane wave e^{i G.r} with G a reciprocal lattice vector of the cell
    # spanned by the rows n_a h_a e_a: the discrete eigenvalue tends to
    # -|G|^2 (G from the Cartesian lattice matrix) as the order grows
    n, h = (40, 36, 44), (0.3, 0.35, 0.28)
    A = np.array(SKEW) / np.linalg.norm(SKEW, axis=1)[:, None] * (np.array(n) * np.array(h))[:, None]
    B = 2 * math.pi * np.linalg.inv(A).T  # rows b_a with a_a . b_b = 2 pi delta
    m3 = (1, -2, 1)
    G = sum(m3[a] * B[a] for a in range(3))
    exact = -float(G @ G)
    errs = []
    for order in (2, 4, 8, 12):
        val, _ = _symbol_cell(n, h, order, SKEW, (0.0, 0.0, 0.0), m3)
        errs.append(abs(val - exact) / abs(exact))
    assert all(errs[k + 1] < errs[k] for k in range(3))
    assert errs[0] > 1e-4 and errs[-1] < 1e-9


def test_orthogonal_cell_reduces_to_the_kronecker_route():
    n, h, order = (6, 5, 7), (0.5, 0.4, 0.45), 4
    theta = (0.7, -1.9, 2.5)
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((2, n[2], n[1], n[0])) + 1j * rng.standard_normal((2, n[2], n[1], n[0]))
    c, s = math.cos(0.3), math.sin(0.3)
    R = [[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]]
    ref = orc.apply_fL_bloch(rho, orc.make_grid_bloch(n, h, order, P3, theta), "erfc", 0.3)
    got = orc.apply_fL_cell(rho, n, h, order, R, theta, "erfc", 0.3)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("lattice", [HEX, SKEW])
def test_cell_coulomb_solve_residual(lattice):
    n, h, order = (6, 7, 5), (0.5, 0.45, 0.4), 6
    theta = (0.9, 0.0, -0.4)  # no zero mode
    rng = np.random.default_rng(11)
    rho = rng.standard_normal((n[2], n[1], n[0])) + 1j * rng.standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL_cell(rho, n, h, order, lattice, theta, "coulomb")
    L = orc.laplacian_cell(n, h, order, lattice, theta)
    res = -L @ phi.ravel() - 4 * math.pi * rho.ravel()
    assert np.max(np.abs(res)) <= 1e-10 * 4 * math.pi * np.max(np.abs(rho))


def test_cell_exchange_reduces_and_satisfies_the_energy_identity():
    n, h, order = (6, 5, 6), (0.5, 0.5, 0.5), 4
    kpts = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.25)]
    wk = [0.4, 0.6]
    occ = [[1.0, 0.7], [0.9, 0.5]]
    psi = bloch_orbitals(n, h, P3, kpts, 2, seed=4, n_centres=4)
    # an orthogonal cell: the Kronecker exchange
    vx_r, ex_r = orc.exchange_bloch(psi, kpts, wk, occ, n, h, order, P3, "erfc", 0.3)
    vx_c, ex_c = orc.exchange_cell(psi, kpts, wk, occ, n, h, order, np.eye(3), "erfc", 0.3)
    assert np.max(np.abs(vx_c - vx_r)) <= 1e-12 * np.max(np.abs(vx_r))
    assert abs(ex_c - ex_r) <= 1e-12 * abs(ex_r)
    # a skewed cell: E_x from the operator (dV includes |det E|)
    vx, ex = orc.exchange_cell(psi, kpts, wk, occ, n, h, order, SKEW, "erfc", 0.3)
    _, jac = orc.cell_metric(SKEW)
    dV = h[0] * h[1] * h[2] * jac
    ev = 0.25 * sum(wk[k] * occ[k][b] * dV * np.vdot(psi[k, b], vx[k, b]).real
                    for k in range(2) for b in range(2))
    assert abs(ev - ex) <= 1e-12 * abs(ex)
    assert ex < 0 and abs(ex - ex_r) > 1e-4 * abs(ex_r)

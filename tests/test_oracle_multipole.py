"""Pins of the oracle's multipole boundary values for isolated systems
(Sec. IV: Dirichlet values from the multipole expansion of the Coulomb
kernel, enforced through the right-hand side).

  * The moment form of the expansion equals an independent formula, the
    Legendre sum  sum_src q sum_l r'^l / r^(l+1) P_l(cos gamma)  (no moments,
    no addition theorem), to rounding.
  * The truncated expansion converges to the exact direct sum q / |r - r'|.
  * The monopole and dipole moments are the total charge and the first
    moments of the density.
  * A Gaussian charge: with multipole boundary values the finite-difference
    potential matches the closed form Q erf(r / (sqrt 2 s)) / r to the
    discretisation error; with homogeneous Dirichlet values it does not.
    Off centre, the error falls as lmax grows.
  * The solve satisfies (-L_D) phi = 4 pi rho + c with the sparse stencil
    (no eigendecomposition).
"""
import math

import numpy as np
import pytest
from scipy.special import erf, eval_legendre

import oracle as orc

D3 = ("dirichlet",) * 3


def _gaussian(n, h, centre, s):
    x1, x2, x3 = orc.node_coords(n, h)
    Z, Y, X = np.meshgrid(x3 - centre[2], x2 - centre[1], x1 - centre[0], indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = np.exp(-r * r / (2 * s * s)) / ((2 * np.pi) ** 1.5 * s ** 3)
    exact = np.where(r > 0, erf(r / (math.sqrt(2) * s)) / np.where(r > 0, r, 1.0),
                     math.sqrt(2 / math.pi) / s)
    return rho, exact


def _charges(seed=3):
    rng = np.random.default_rng(seed)
    n, h = (5, 6, 7), (0.3, 0.35, 0.25)
    grid = orc.make_grid(n, h, 4, D3)
    rho = rng.standard_normal((n[2], n[1], n[0]))
    centre = ((n[0] - 1) * h[0] / 2, (n[1] - 1) * h[1] / 2, (n[2] - 1) * h[2] / 2)
    x1, x2, x3 = orc.node_coords(n, h)
    Z, Y, X = np.meshgrid(x3, x2, x1, indexing="ij")
    src = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    q = grid.dV * rho.ravel()
    # evaluation points well outside the charge, in several directions
    pts = np.array([[9.0, 0.3, -1.0], [-6.0, 7.5, 2.0], [0.4, 0.5, 11.0], [-5.0, -5.0, -5.0],
                    [3.0, -8.0, 6.0]])
    return grid, rho, centre, src, q, pts


@pytest.mark.parametrize("lmax", [0, 1, 2, 4, 6])
def test_moment_form_equals_legendre_sum(lmax):
    grid, rho, centre, src, q, pts = _charges()
    A, B = orc.multipole_moments(rho, grid, centre, lmax)
    got = orc.multipole_potential(A, B, pts, centre)
    c = np.asarray(centre)
    ref = np.zeros(len(pts))
    for k, p in enumerate(pts):
        d = p - c
        r = np.linalg.norm(d)
        s = src - c
        rs = np.linalg.norm(s, axis=1)
        cosg = np.where(rs > 0, (s @ d) / (np.where(rs > 0, rs, 1.0) * r), 1.0)
        for l in range(lmax + 1):
            ref[k] += float(np.sum(q * rs ** l * eval_legendre(l, cosg))) / r ** (l + 1)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)) + 1e-15


def test_expansion_converges_to_the_direct_coulomb_sum():
    grid, rho, centre, src, q, pts = _charges()
    exact = np.array([float(np.sum(q / np.linalg.norm(src - p, axis=1))) for p in pts])
    errs = []
    for lmax in range(0, 9):
        A, B = orc.multipole_moments(rho, grid, centre, lmax)
        errs.append(np.max(np.abs(orc.multipole_potential(A, B, pts, centre) - exact)))
    assert errs[-1] <= 1e-6 * np.max(np.abs(exact))
    assert errs[-1] < errs[4] < errs[0]


def test_low_moments_are_charge_and_dipole():
    grid, rho, centre, src, q, pts = _charges()
    A, B = orc.multipole_moments(rho, grid, centre, 1)
    s = src - np.asarray(centre)
    assert A[0, 0] == pytest.approx(float(np.sum(q)), rel=1e-13)
    assert A[1, 0] == pytest.approx(float(np.sum(q * s[:, 2])), rel=1e-12)
    # P_1^1(cos t) = -sin t (Condon-Shortley): A[1,1] = -p_x, B[1,1] = -p_y
    assert A[1, 1] == pytest.approx(-float(np.sum(q * s[:, 0])), rel=1e-12)
    assert B[1, 1] == pytest.approx(-float(np.sum(q * s[:, 1])), rel=1e-12)
    assert B[0, 0] == 0.0 and B[1, 0] == 0.0


def test_centred_gaussian_matches_its_closed_form():
    n, h = (24, 24, 24), (0.4, 0.4, 0.4)
    grid = orc.make_grid(n, h, 12, D3)
    centre = ((n[0] - 1) * h[0] / 2,) * 3
    rho, exact = _gaussian(n, h, centre, 0.8)
    phi = orc.apply_coulomb_multipole(rho, grid, centre, 2)
    phi0 = orc.apply_fL(rho, grid, "coulomb")
    scale = np.max(exact)
    assert np.max(np.abs(phi - exact)) <= 1e-5 * scale
    assert np.max(np.abs(phi0 - exact)) >= 0.1 * scale


def test_off_centre_gaussian_error_falls_with_lmax():
    # the box holds the whole charge (to 2e-12), so the closed form is exact;
    # what remains at high lmax is the finite-difference error (~6e-6 here)
    n, h = (30, 30, 30), (0.4, 0.4, 0.4)
    grid = orc.make_grid(n, h, 12, D3)
    box_centre = ((n[0] - 1) * h[0] / 2, (n[1] - 1) * h[1] / 2, (n[2] - 1) * h[2] / 2)
    charge = (box_centre[0] + 1.2, box_centre[1] - 0.8, box_centre[2] + 0.6)
    rho, exact = _gaussian(n, h, charge, 0.7)
    scale = np.max(exact)
    errs = [np.max(np.abs(orc.apply_coulomb_multipole(rho, grid, box_centre, l) - exact)) / scale
            for l in (0, 2, 4, 6)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[0] >= 1e-2 and errs[3] <= 1e-5


def test_multipole_solve_satisfies_the_modified_stencil_equation():
    import scipy.sparse as sp
    n, h = (14, 12, 10), (0.35, 0.3, 0.4)
    grid = orc.make_grid(n, h, 8, D3)
    rng = np.random.default_rng(9)
    rho = rng.standard_normal((n[2], n[1], n[0]))
    centre = (2.0, 1.5, 1.9)
    phi = orc.apply_coulomb_multipole(rho, grid, centre, 3)
    c = orc.multipole_rhs_correction(rho, grid, centre, 3)
    L = [sp.csr_matrix(orc.laplacian_1d(n[k], h[k], 8, "dirichlet")) for k in range(3)]
    I = [sp.identity(n[k], format="csr") for k in range(3)]
    Lfull = (sp.kron(sp.kron(I[2], I[1]), L[0]) + sp.kron(sp.kron(I[2], L[1]), I[0]) +
             sp.kron(sp.kron(L[2], I[1]), I[0]))
    lhs = -(Lfull @ phi.ravel())
    rhs = 4 * np.pi * rho.ravel() + c.ravel()
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * np.max(np.abs(rhs))


def test_correction_touches_only_the_boundary_layers():
    n, h = (16, 15, 17), (0.3, 0.3, 0.3)
    grid = orc.make_grid(n, h, 12, D3)
    rho, _ = _gaussian(n, h, (2.2, 2.1, 2.4), 0.6)
    c = orc.multipole_rhs_correction(rho, grid, (2.2, 2.1, 2.4), 2)
    m = 6
    inner = c[m:n[2] - m, m:n[1] - m, m:n[0] - m]
    assert np.all(inner == 0.0)
    assert np.all(c[0, m:-m, m:-m] != 0.0)


def test_rejects_periodic_axes():
    grid = orc.make_grid((6, 6, 6), (0.4,) * 3, 4, ("periodic", "dirichlet", "dirichlet"))
    with pytest.raises(ValueError):
        orc.multipole_rhs_correction(np.ones((6, 6, 6)), grid, (1.0, 1.0, 1.0), 1)


def _gaussian_orbitals(n, h, centres, alphas):
    x1, x2, x3 = orc.node_coords(n, h)
    Z, Y, X = np.meshgrid(x3, x2, x1, indexing="ij")
    out = []
    for c, a in zip(centres, alphas):
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        out.append((2 * a / math.pi) ** 0.75 * np.exp(-a * r2))  # unit norm in the continuum
    return np.array(out)


def test_isolated_exchange_matches_the_gaussian_closed_form():
    # s-type Gaussians psi_i ~ exp(-a_i |r - A_i|^2): every pair density is a
    # Gaussian charge of exponent p = a_i + a_j and charge Q_ij = int psi_i psi_j,
    # whose Coulomb self-energy in free space is Q^2 sqrt(2 p / pi).  The
    # exchange with multipole boundary values approaches the free-space value;
    # with homogeneous ends it does not.
    n, h = (36, 34, 38), (0.3, 0.3, 0.3)
    L = [(n[k] - 1) * h[k] for k in range(3)]
    mid = [L[k] / 2 for k in range(3)]
    centres = [(mid[0] - 0.7, mid[1] + 0.2, mid[2] - 0.4), (mid[0] + 0.6, mid[1] - 0.5, mid[2] + 0.3),
               (mid[0] + 0.1, mid[1] + 0.6, mid[2] + 0.8)]
    alphas = [0.9, 1.3, 1.1]
    psi = _gaussian_orbitals(n, h, centres, alphas)
    occ = np.array([2.0, 1.5, 1.0])
    exact = 0.0
    for i in range(3):
        for j in range(3):
            p = alphas[i] + alphas[j]
            mu = alphas[i] * alphas[j] / p
            d2 = sum((centres[i][k] - centres[j][k]) ** 2 for k in range(3))
            Q = ((2 * alphas[i] / math.pi) * (2 * alphas[j] / math.pi)) ** 0.75 * (math.pi / p) ** 1.5 \
                * math.exp(-mu * d2)
            exact -= 0.25 * occ[i] * occ[j] * Q * Q * math.sqrt(2 * p / math.pi)
    grid = orc.make_grid(n, h, 12, D3)
    errs = []
    for lmax in (0, 2):
        errs.append(abs(orc.exchange_multipole(psi, occ, grid, mid, lmax)[1] - exact) / abs(exact))
    vx, ex = orc.exchange_multipole(psi, occ, grid, mid, 6)
    errs.append(abs(ex - exact) / abs(exact))
    _, ex0 = orc.exchange(psi, occ, grid, "coulomb")
    # the error falls as the expansion grows, to the discretisation level
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 2e-6
    assert abs(ex0 - exact) >= 1e-2 * abs(exact)
    # E_x = 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h
    ev = 0.25 * sum(occ[j] * grid.dV * float(np.sum(psi[j] * vx[j])) for j in range(3))
    assert abs(ev - ex) <= 1e-12 * abs(ex)

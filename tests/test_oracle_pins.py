"""Pins for the FP64 oracle: each test checks it against something other than
itself (textbook constants, closed forms, brute force, an FFT route, sparse
residuals, a Krylov matrix exponential, invariants of the exchange operator).

Every test here runs on the CPU only.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.special
from scipy.sparse.linalg import expm_multiply

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D, P = "dirichlet", "periodic"


# ---------------------------------------------------------------- P1: FD weights
def _golden_weights():
    out = {}
    with open(os.path.join(GOLDEN, "fd_weights_centred_d2.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            order, vals = line.split(":")
            out[int(order)] = [Fraction(v) for v in vals.split()]
    return out


def test_fd_weights_match_textbook_table():
    for order, ref in _golden_weights().items():
        assert orc.fd_weights(order) == ref, order


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 16, 24])
def test_fd_weights_match_closed_form(order):
    # w_p = 2 (-1)^(p+1) (m!)^2 / (p^2 (m-p)! (m+p)!),  w_0 = -2 sum_p w_p
    m = order // 2
    fm = math.factorial(m)
    wp = [Fraction(2 * (-1) ** (p + 1) * fm * fm,
                   p * p * math.factorial(m - p) * math.factorial(m + p)) for p in range(1, m + 1)]
    ref = [-2 * sum(wp)] + wp
    assert orc.fd_weights(order) == ref


@pytest.mark.parametrize("order", [2, 4, 8, 12])
def test_fd_stencil_exact_on_polynomials(order):
    # A centred stencil of order 2m differentiates x^q exactly for q <= 2m+1.
    n, h = 40, 0.25
    L = orc.laplacian_1d(n, h, order, D)
    m = order // 2
    x = np.arange(n) * h - 4.0
    for q in range(order + 2):
        f = x ** q
        d2 = q * (q - 1) * x ** (q - 2) if q >= 2 else np.zeros(n)
        interior = slice(m, n - m)
        scale = max(1.0, np.max(np.abs(f)) / h ** 2)
        assert np.max(np.abs((L @ f)[interior] - d2[interior])) < 1e-9 * scale, q


def test_fd_convergence_order():
    # error on sin(x) falls like h^order (periodic grid, 12th order)
    errs = []
    for n in (10, 20):
        h = 2 * np.pi / n
        x = np.arange(n) * h
        L = orc.laplacian_1d(n, h, 12, P)
        errs.append(np.max(np.abs(L @ np.sin(x) + np.sin(x))))
    rate = math.log(errs[0] / errs[1], 2)
    assert rate > 11.0


# ---------------------------------------------------------------- P2: 1-D spectra
@pytest.mark.parametrize("n,h,order", [(96, 0.35, 12), (60, 0.3, 12), (7, 0.4, 12), (33, 0.5, 4)])
def test_periodic_eigenvalues_match_circulant_symbol(n, h, order):
    w = [float(x) for x in _closed_form(order)]
    q = np.arange(n)
    sym = -(w[0] + 2 * sum(w[p] * np.cos(2 * np.pi * q * p / n) for p in range(1, len(w)))) / h ** 2
    g = orc.make_grid((n, 5, 5), (h, 1.0, 1.0), order, (P, D, D))
    assert np.max(np.abs(np.sort(sym) - g.lam[0])) < 1e-12 * np.max(sym)


def _closed_form(order):
    m = order // 2
    fm = math.factorial(m)
    wp = [Fraction(2 * (-1) ** (p + 1) * fm * fm,
                   p * p * math.factorial(m - p) * math.factorial(m + p)) for p in range(1, m + 1)]
    return [-2 * sum(wp)] + wp


def test_dirichlet_second_order_matches_dst():
    n, h = 37, 0.3
    g = orc.make_grid((n, 3, 3), (h, 1, 1), 2, (D, D, D))
    q = np.arange(1, n + 1)
    lam = (2 - 2 * np.cos(q * np.pi / (n + 1))) / h ** 2
    assert np.max(np.abs(lam - g.lam[0])) < 1e-12 * lam.max()
    i = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, q) * np.pi / (n + 1))
    # eigenvectors agree up to sign (spectrum is simple)
    dots = np.abs(np.sum(S * g.V[0], axis=0))
    assert np.max(np.abs(dots - 1.0)) < 1e-12


# ---------------------------------------------------------------- P3: brute force
def _dense_laplacian(n, h, order, bc):
    L1, L2, L3 = (orc.laplacian_1d(n[k], h[k], order, bc[k]) for k in range(3))
    I1, I2, I3 = (np.eye(n[k]) for k in range(3))
    # vec index i1 + n1 (i2 + n2 i3): axis 1 is the innermost Kronecker factor
    return (np.kron(I3, np.kron(I2, L1)) + np.kron(I3, np.kron(L2, I1))
            + np.kron(L3, np.kron(I2, I1)))


def _dense_f(n, h, order, bc, kernel, omega):
    L = _dense_laplacian(n, h, order, bc)
    lam, Q = np.linalg.eigh(-L)
    if kernel == "coulomb":
        f = 4 * np.pi / lam
    else:
        f = 4 * np.pi * (1 - np.exp(-lam / (4 * omega ** 2))) / np.where(lam == 0, 1, lam)
        f = np.where(np.abs(lam) < 1e-12, np.pi / omega ** 2, f)
    return (Q * f) @ Q.T


BRUTE_CASES = [
    ((4, 5, 6), (0.4, 0.3, 0.35), 12, (D, D, D), "coulomb", 0.0),
    ((4, 5, 6), (0.4, 0.3, 0.35), 12, (D, D, D), "erfc", 0.106),
    ((5, 6, 7), (0.3, 0.3, 0.3), 12, (P, P, D), "erfc", 0.106),
    ((5, 6, 7), (0.3, 0.3, 0.3), 4, (P, P, D), "coulomb", 0.0),
    ((7, 7, 9), (0.35, 0.35, 0.35), 12, (P, P, P), "erfc", 0.106),
    ((6, 5, 8), (0.5, 0.4, 0.3), 2, (D, P, D), "coulomb", 0.0),
    ((8, 6, 5), (0.3, 0.4, 0.5), 8, (D, P, D), "erfc", 0.5),
]


@pytest.mark.parametrize("n,h,order,bc,kernel,omega", BRUTE_CASES)
def test_apply_fL_matches_dense_brute_force(n, h, order, bc, kernel, omega):
    g = orc.make_grid(n, h, order, bc)
    rng = np.random.default_rng(11)
    rho = rng.standard_normal((2, n[2], n[1], n[0]))
    phi = orc.apply_fL(rho, g, kernel, omega)
    Fd = _dense_f(n, h, order, bc, kernel, omega)
    for b in range(2):
        ref = (Fd @ rho[b].ravel()).reshape(rho[b].shape)
        assert np.max(np.abs(phi[b] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_exchange_matches_dense_brute_force():
    # Vx and E_x from the dense f(-L) and a plain double loop over all (i, j)
    n, h, order, bc = (5, 4, 6), (0.4, 0.45, 0.35), 12, (D, P, D)
    g = orc.make_grid(n, h, order, bc)
    rng = np.random.default_rng(3)
    norb = 4
    psi = rng.standard_normal((norb, n[2], n[1], n[0]))
    occ = np.array([2.0, 1.5, 0.5, 1.0])
    for kernel, omega in (("coulomb", 0.0), ("erfc", 0.3)):
        Fd = _dense_f(n, h, order, bc, kernel, omega)
        vx_ref = np.zeros_like(psi)
        ex_ref = 0.0
        for j in range(norb):
            for i in range(norb):
                rho = (psi[i] * psi[j]).ravel()
                phi = Fd @ rho
                vx_ref[j] -= occ[i] * (phi * psi[i].ravel()).reshape(psi[j].shape)
                ex_ref -= 0.25 * occ[i] * occ[j] * g.dV * float(rho @ phi)
        vx, ex = orc.exchange(psi, occ, g, kernel, omega)
        assert np.max(np.abs(vx - vx_ref)) <= 1e-12 * np.max(np.abs(vx_ref))
        assert abs(ex - ex_ref) <= 1e-12 * abs(ex_ref)
        for j in range(norb):
            v1 = orc.vx_orbital(psi, occ, j, g, kernel, omega)
            assert np.max(np.abs(v1 - vx_ref[j])) <= 1e-12 * np.max(np.abs(vx_ref))


# ---------------------------------------------------------------- P4: FFT route
@pytest.mark.parametrize("n,h", [((48, 48, 48), (0.35, 0.35, 0.35)), ((20, 24, 18), (0.3, 0.35, 0.4))])
def test_periodic_apply_matches_fft(n, h):
    order = 12
    g = orc.make_grid(n, h, order, (P, P, P))
    w = [float(x) for x in _closed_form(order)]
    lam_axes = []
    for k in range(3):
        q = np.arange(n[k])
        lam_axes.append(-(w[0] + 2 * sum(w[p] * np.cos(2 * np.pi * q * p / n[k])
                                         for p in range(1, len(w)))) / h[k] ** 2)
    lam = lam_axes[2][:, None, None] + lam_axes[1][None, :, None] + lam_axes[0][None, None, :]
    omega = 0.106
    x = lam / (4 * omega ** 2)
    # the q = 0 mode of the symbol is zero up to rounding; its limit is pi/w^2
    zero = np.abs(lam) < 1e-9
    f = np.where(zero, np.pi / omega ** 2,
                 4 * np.pi * (1 - np.exp(-x)) / np.where(zero, 1, lam))
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((n[2], n[1], n[0]))
    ref = np.real(np.fft.ifftn(np.fft.fftn(rho) * f))
    phi = orc.apply_fL(rho, g, "erfc", omega)
    assert np.max(np.abs(phi - ref)) <= 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------- P5: kernel constant
def test_erfc_kernel_matches_real_space_closed_form():
    # Unit Gaussian charge of width s at the centre of a periodic box.  The
    # potential of erfc(w r)/r is [erf(r/(sqrt2 s)) - erf(r/sqrt(2 s^2 + 1/w^2))]/r.
    n, h = 48, 0.35
    s, omega = 1.2, 0.8
    g = orc.make_grid((n, n, n), (h, h, h), 12, (P, P, P))
    c = (n // 2) * h
    x = np.arange(n) * h - c
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    rho = np.exp(-r2 / (2 * s * s)) / ((2 * np.pi) ** 1.5 * s ** 3)
    phi = orc.apply_fL(rho, g, "erfc", omega)
    r = np.sqrt(r2)
    a, b = 1 / (math.sqrt(2) * s), 1 / math.sqrt(2 * s * s + 1 / omega ** 2)
    rs = np.where(r == 0, 1.0, r)
    ref = np.where(r == 0, 2 / math.sqrt(math.pi) * (a - b),
                   (scipy.special.erf(a * rs) - scipy.special.erf(b * rs)) / rs)
    err = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert err < 1e-6, err
    # the 16 pi omega^2 exponent printed in Eq. (10) would miss by far more
    wrong = orc.apply_fL(rho, g, "erfc", omega * math.sqrt(4 * math.pi))
    assert np.max(np.abs(wrong - ref)) / np.max(np.abs(ref)) > 0.1


# ---------------------------------------------------------------- P6/P7: residuals
def _sparse_L(n, h, order, bc):
    L1, L2, L3 = (sp.csr_matrix(orc.laplacian_1d(n[k], h[k], order, bc[k])) for k in range(3))
    I1, I2, I3 = (sp.identity(n[k], format="csr") for k in range(3))
    return (sp.kron(I3, sp.kron(I2, L1)) + sp.kron(I3, sp.kron(L2, I1))
            + sp.kron(L3, sp.kron(I2, I1))).tocsr()


@pytest.mark.parametrize("bc", [(D, D, D), (P, P, D), (D, P, P)])
def test_coulomb_residual(bc):
    n, h = (16, 14, 18), (0.3, 0.35, 0.3)
    g = orc.make_grid(n, h, 12, bc)
    rho = np.random.default_rng(2).standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL(rho, g, "coulomb")
    L = _sparse_L(n, h, 12, bc)
    res = -(L @ phi.ravel()) - 4 * np.pi * rho.ravel()
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(4 * np.pi * rho)


@pytest.mark.parametrize("bc,omega", [((D, D, D), 0.106), ((P, P, D), 0.106), ((D, D, D), 0.6)])
def test_erfc_residual_against_krylov_expm(bc, omega):
    # (-L) phi = 4 pi (rho - exp(L / (4 w^2)) rho)
    n, h = (12, 14, 10), (0.3, 0.3, 0.35)
    g = orc.make_grid(n, h, 12, bc)
    rho = np.random.default_rng(4).standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL(rho, g, "erfc", omega)
    L = _sparse_L(n, h, 12, bc)
    rhs = 4 * np.pi * (rho.ravel() - expm_multiply(L / (4 * omega ** 2), rho.ravel()))
    res = -(L @ phi.ravel()) - rhs
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(rhs)


# ---------------------------------------------------------------- P8: exchange invariants
def _small_orbitals(n, h, bc, norb, seed):
    from synth import gaussian_orbitals, orthonormalise_cgs2
    psi = gaussian_orbitals(n, h, bc, norb, seed, 3 * norb, True)
    return orthonormalise_cgs2(psi, h[0] * h[1] * h[2])


@pytest.mark.parametrize("kernel,omega,bc", [("coulomb", 0.0, (D, D, D)), ("erfc", 0.106, (P, P, P)),
                                             ("erfc", 0.3, (P, D, P))])
def test_vx_symmetric_negative_semidefinite(kernel, omega, bc):
    n, h = (14, 16, 12), (0.45, 0.4, 0.5)
    norb = 6
    psi = _small_orbitals(n, h, bc, norb, 9)
    occ = np.array([2.0, 2.0, 1.0, 1.5, 0.5, 2.0])
    g = orc.make_grid(n, h, 12, bc)
    vx, ex, es = orc.exchange(psi, occ, g, kernel, omega, pair_energies=True)
    M = g.dV * np.einsum("kr,jr->jk", psi.reshape(norb, -1), vx.reshape(norb, -1))
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.max(np.linalg.eigvalsh(0.5 * (M + M.T))) <= 1e-12 * np.max(np.abs(M))
    assert abs(ex - 0.25 * float(occ @ np.diag(M))) <= 1e-12 * abs(ex)
    assert ex < 0
    assert all(e > 0 for (i, j), e in es.items() if i == j)


def test_energy_bilinear_in_occupations():
    n, h, bc = (10, 12, 11), (0.45, 0.4, 0.5), (D, D, D)
    psi = _small_orbitals(n, h, bc, 3, 4)
    g = orc.make_grid(n, h, 12, bc)
    _, _, es = orc.exchange(psi, np.ones(3), g, "coulomb", pair_energies=True)
    occ = np.array([2.0, 0.7, 1.3])
    _, ex = orc.exchange(psi, occ, g, "coulomb")
    ref = -0.25 * sum(occ[i] * occ[j] * es[(min(i, j), max(i, j))] for i in range(3) for j in range(3))
    assert abs(ex - ref) <= 1e-13 * abs(ref)


# ---------------------------------------------------------------- P9: kernel limits
def test_erfc_limits():
    n, h, bc = (12, 10, 14), (0.3, 0.3, 0.3), (D, D, D)
    g = orc.make_grid(n, h, 12, bc)
    rho = np.random.default_rng(6).standard_normal((n[2], n[1], n[0]))
    coul = orc.apply_fL(rho, g, "coulomb")
    small = orc.apply_fL(rho, g, "erfc", 1e-3)
    assert np.max(np.abs(small - coul)) <= 1e-13 * np.max(np.abs(coul))
    big = 1e3
    far = orc.apply_fL(rho, g, "erfc", big) * big ** 2 / np.pi
    assert np.max(np.abs(far - rho)) <= 1e-4 * np.max(np.abs(rho))
    lam = g.lam_sum()
    w = 0.5
    fe = orc.kernel_values(lam, "erfc", w)
    fc = orc.kernel_values(lam, "coulomb")
    # 0 < f_erfc <= f_coul (equal to rounding once exp(-lam/(4 w^2)) underflows)
    assert np.all(fe > 0) and np.all(fe <= fc * (1 + 4e-16))
    soft = lam / (4 * w * w) < 30
    assert soft.any() and np.all(fe[soft] < fc[soft])
    psi = _small_orbitals(n, h, bc, 3, 5)
    _, e_c = orc.exchange(psi, np.full(3, 2.0), g, "coulomb")
    _, e_s = orc.exchange(psi, np.full(3, 2.0), g, "erfc", w)
    assert e_c < e_s < 0


def test_erfc_zero_mode_value():
    assert orc.kernel_values(np.array([0.0]), "erfc", 0.106)[0] == pytest.approx(np.pi / 0.106 ** 2, rel=1e-15)
    v = orc.kernel_values(np.array([-1e-15, 1e-15]), "erfc", 0.106)
    assert np.all(np.abs(v / (np.pi / 0.106 ** 2) - 1) < 1e-12)
    with pytest.raises(ZeroDivisionError):
        orc.kernel_values(np.array([0.0, 1.0]), "coulomb")


# ---------------------------------------------------------------- P10: energy identity
def test_pair_energy_parseval():
    n, h, bc = (16, 12, 14), (0.35, 0.35, 0.35), (P, P, D)
    g = orc.make_grid(n, h, 12, bc)
    rng = np.random.default_rng(8)
    a, b = rng.standard_normal((2, n[2], n[1], n[0]))
    rho = a * b
    F = orc.kernel_values(g.lam_sum(), "erfc", 0.106)
    Bt = orc.forward_transform(rho, g)
    e1 = g.dV * float(np.sum(F * Bt * Bt))
    e2 = orc.pair_energy(a, b, g, "erfc", 0.106)
    assert abs(e1 - e2) <= 1e-13 * abs(e2)


# ---------------------------------------------------------------- ACE form of the exchange (Sec. IV)
def _ace_case(kernel, omega, bc, norb=5, seed=11):
    n, h = (9, 8, 10), (0.5, 0.45, 0.4)
    psi = _small_orbitals(n, h, bc, norb, seed)
    occ = np.linspace(2.0, 1.0, norb)
    g = orc.make_grid(n, h, 12, bc)
    vx, _ = orc.exchange(psi, occ, g, kernel, omega)
    return g, psi, vx


@pytest.mark.parametrize("kernel,omega,bc", [("coulomb", 0.0, (D, D, D)), ("erfc", 0.106, (P, P, P)),
                                             ("erfc", 0.3, (P, D, P))])
def test_ace_reproduces_exchange_on_orbitals(kernel, omega, bc):
    # defining property of the compressed operator: V_ACE psi_j = (Vx psi)_j
    g, psi, vx = _ace_case(kernel, omega, bc)
    xi = orc.ace_build(psi, vx, g.dV)
    out = orc.ace_apply(xi, psi, g.dV)
    assert np.max(np.abs(out - vx)) <= 1e-12 * np.max(np.abs(vx))


def test_ace_equals_projector_form():
    # V_ACE = W M^{-1} W^T (h-weighted), M = (psi, W)_h: the same operator
    # written with an explicit inverse instead of the Cholesky factor
    g, psi, vx = _ace_case("erfc", 0.2, (P, P, D))
    norb = psi.shape[0]
    xi = orc.ace_build(psi, vx, g.dV)
    W = vx.reshape(norb, -1)
    M = g.dV * (psi.reshape(norb, -1) @ W.T)
    phi = np.random.default_rng(3).standard_normal((4,) + psi.shape[1:])
    ref = (W.T @ np.linalg.inv(M) @ (g.dV * (W @ phi.reshape(4, -1).T))).T.reshape(phi.shape)
    out = orc.ace_apply(xi, phi, g.dV)
    assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_ace_operator_symmetric_negative_rank():
    # as a matrix on the grid: symmetric in the h inner product, negative
    # semidefinite, of rank norb, and zero on fields h-orthogonal to every W_j
    g, psi, vx = _ace_case("coulomb", 0.0, (D, P, D), norb=4)
    xi = orc.ace_build(psi, vx, g.dV)
    N = int(np.prod(psi.shape[1:]))
    A = orc.ace_apply(xi, np.eye(N).reshape((N,) + psi.shape[1:]), g.dV).reshape(N, N)
    assert np.max(np.abs(A - A.T)) <= 1e-12 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() <= 1e-12 * np.abs(ev).max()
    assert int(np.sum(ev < -1e-9 * np.abs(ev).max())) == 4
    W = vx.reshape(4, -1)
    phi = np.random.default_rng(8).standard_normal(N)
    phi -= W.T @ np.linalg.solve(W @ W.T, W @ phi)
    out = orc.ace_apply(xi, phi.reshape((1,) + psi.shape[1:]), g.dV)
    assert np.max(np.abs(out)) <= 1e-12 * np.max(np.abs(A))


def test_ace_rejects_non_negative_definite():
    g, psi, vx = _ace_case("coulomb", 0.0, (D, D, D), norb=3)
    with pytest.raises(np.linalg.LinAlgError):
        orc.ace_build(psi, -vx, g.dV)

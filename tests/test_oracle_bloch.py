"""Pins of the oracle's Brillouin-zone sampling (Sec. II: the pair (m q, n k)
solves the Poisson problem with Bloch boundary conditions at k - q).

  * L_k(theta) is Hermitian, equals the periodic L_k at theta = 0 and is
    2 pi periodic in theta; its eigenvalues are the closed-form symbol
    (-w0 - 2 sum_p w_p cos((2 pi j + theta) p / n)) / h^2.
  * The Kronecker solve equals dense brute force (kron of the complex 1-D
    matrices, eigh, f) on tiny grids with Bloch and Dirichlet axes.
  * On all-periodic grids it equals an FFT route: remove the phase ramp,
    fftn, multiply by f of the shifted symbols, ifftn, restore the ramp.
  * The Bloch solution satisfies the Bloch condition: extended by one period
    it picks up e^{i theta} (checked through the sparse residual of the
    stencil equation with wrapped phases).
  * Exchange: at the Gamma point with real orbitals it equals the real
    exchange; the matrix <psi_m'k, Vx psi_nk> is Hermitian and negative
    semidefinite per k; E_x = 1/4 sum w_k occ <psi, Vx psi>; time reversal
    (psi_{-k} = conj psi_k) gives Vx psi_{-k} = conj(Vx psi_k).
"""
import math

import numpy as np
import pytest

import oracle as orc
from synth import bloch_orbitals, make_workload

P3 = ("periodic",) * 3


def _symbol(n, h, order, theta):
    w = [float(x) for x in orc.fd_weights(order)]
    m = order // 2
    j = np.arange(n)
    lam = -w[0] - 2.0 * sum(w[p] * np.cos((2 * math.pi * j + theta) * p / n) for p in range(1, m + 1))
    return lam / (h * h)


@pytest.mark.parametrize("n,order,theta", [(8, 4, 0.7), (11, 12, 2.9), (16, 8, math.pi),
                                           (5, 2, -1.3), (24, 12, 0.0)])
def test_bloch_laplacian_and_its_spectrum(n, order, theta):
    h = 0.35
    L = orc.laplacian_1d_bloch(n, h, order, theta)
    assert np.allclose(L, L.conj().T, rtol=0, atol=1e-13 / h ** 2)
    if theta == 0.0:
        assert np.allclose(L.real, orc.laplacian_1d(n, h, order, "periodic"), atol=1e-14)
        assert np.max(np.abs(L.imag)) == 0.0
    assert np.allclose(L, orc.laplacian_1d_bloch(n, h, order, theta + 2 * math.pi), atol=1e-12)
    lam = np.linalg.eigvalsh(-L)
    ref = np.sort(_symbol(n, h, order, theta))
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,bc,theta,kernel", [
    ((4, 5, 6), ("periodic", "periodic", "periodic"), (0.8, -2.1, 3.0), "erfc"),
    ((5, 4, 6), ("periodic", "dirichlet", "periodic"), (1.7, 0.0, -0.4), "coulomb"),
    ((6, 5, 4), ("dirichlet", "periodic", "dirichlet"), (0.0, 2.5, 0.0), "erfc"),
])
def test_bloch_solve_equals_dense_brute_force(n, bc, theta, kernel):
    h, order, omega = (0.4, 0.35, 0.3), 4, 0.3
    grid = orc.make_grid_bloch(n, h, order, bc, theta)
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((n[2], n[1], n[0])) + 1j * rng.standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL_bloch(rho, grid, kernel, omega)
    Ls = []
    for k in range(3):
        if bc[k] == "periodic":
            Ls.append(orc.laplacian_1d_bloch(n[k], h[k], order, theta[k]))
        else:
            Ls.append(orc.laplacian_1d(n[k], h[k], order, bc[k]).astype(np.complex128))
    I = [np.eye(n[k]) for k in range(3)]
    A = -(np.kron(np.kron(I[2], I[1]), Ls[0]) + np.kron(np.kron(I[2], Ls[1]), I[0]) +
          np.kron(np.kron(Ls[2], I[1]), I[0]))
    lam, V = np.linalg.eigh(A)
    f = orc.kernel_values(lam, kernel, omega)
    ref = (V @ (f * (V.conj().T @ rho.ravel()))).reshape(rho.shape)
    assert np.max(np.abs(phi - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_bloch_solve_equals_fft_route():
    n, h, theta = (12, 10, 14), (0.35, 0.3, 0.4), (0.9, -2.4, 3.1)
    grid = orc.make_grid_bloch(n, h, 12, P3, theta)
    rng = np.random.default_rng(7)
    rho = rng.standard_normal((n[2], n[1], n[0])) + 1j * rng.standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL_bloch(rho, grid, "erfc", 0.2)
    i1, i2, i3 = (np.arange(n[k]) for k in range(3))
    ramp = (np.exp(1j * theta[2] * i3 / n[2])[:, None, None] *
            np.exp(1j * theta[1] * i2 / n[1])[None, :, None] *
            np.exp(1j * theta[0] * i1 / n[0])[None, None, :])
    # the phase-free field is periodic; its Fourier mode j sees the symbol at j + theta / 2 pi
    lam = (_symbol(n[2], h[2], 12, theta[2])[:, None, None] +
           _symbol(n[1], h[1], 12, theta[1])[None, :, None] +
           _symbol(n[0], h[0], 12, theta[0])[None, None, :])
    ref = ramp * np.fft.ifftn(orc.kernel_values(lam, "erfc", 0.2) * np.fft.fftn(rho / ramp))
    assert np.max(np.abs(phi - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_bloch_solve_satisfies_the_stencil_equation():
    import scipy.sparse as sp
    n, h, theta = (9, 8, 7), (0.3, 0.35, 0.4), (1.1, -0.6, 2.2)
    grid = orc.make_grid_bloch(n, h, 8, P3, theta)
    rng = np.random.default_rng(2)
    rho = rng.standard_normal((n[2], n[1], n[0])) + 1j * rng.standard_normal((n[2], n[1], n[0]))
    phi = orc.apply_fL_bloch(rho, grid, "coulomb")
    L = [sp.csr_matrix(orc.laplacian_1d_bloch(n[k], h[k], 8, theta[k])) for k in range(3)]
    I = [sp.identity(n[k], format="csr") for k in range(3)]
    Lf = (sp.kron(sp.kron(I[2], I[1]), L[0]) + sp.kron(sp.kron(I[2], L[1]), I[0]) +
          sp.kron(sp.kron(L[2], I[1]), I[0]))
    res = -(Lf @ phi.ravel()) - 4 * np.pi * rho.ravel()
    assert np.max(np.abs(res)) <= 1e-11 * 4 * np.pi * np.max(np.abs(rho))


def test_gamma_point_real_orbitals_reduce_to_the_real_exchange():
    w, psi, occ = make_workload("dirichlet20x27x34_coulomb")
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_r, ex_r = orc.exchange(psi, occ, grid, w.kernel, w.omega)
    vx_c, ex_c = orc.exchange_bloch(psi[None].astype(np.complex128), [(0.0, 0.0, 0.0)], [1.0],
                                    occ[None], w.n, w.h, w.order, w.bc, w.kernel, w.omega)
    assert abs(ex_c - ex_r) <= 1e-12 * abs(ex_r)
    assert np.max(np.abs(vx_c[0] - vx_r)) <= 1e-12 * np.max(np.abs(vx_r))


@pytest.fixture(scope="module")
def kset():
    n, h, bc = (10, 9, 11), (0.45, 0.5, 0.4), P3
    # a time-reversal symmetric set: k1 = -k0, k3 = -k2, psi_{-k} = conj(psi_k)
    kpts = [(0.5, 0.0, 0.25), (-0.5, 0.0, -0.25), (0.25, 0.5, 0.0), (-0.25, -0.5, 0.0)]
    wk = [0.25] * 4
    psi = bloch_orbitals(n, h, bc, kpts, 3, seed=21, n_centres=12)
    psi[1] = np.conj(psi[0])
    psi[3] = np.conj(psi[2])
    occ = np.array([[2.0, 1.5, 0.5]] * 4)
    vx, ex = orc.exchange_bloch(psi, kpts, wk, occ, n, h, 12, bc, "erfc", 0.3)
    return dict(n=n, h=h, bc=bc, kpts=kpts, wk=wk, psi=psi, occ=occ, vx=vx, ex=ex)


def test_bloch_exchange_matrix_is_hermitian_negative_semidefinite(kset):
    dV = float(np.prod(kset["h"]))
    psi, vx = kset["psi"], kset["vx"]
    K, norb = psi.shape[:2]
    for k in range(K):
        P = psi[k].reshape(norb, -1)
        W = vx[k].reshape(norb, -1)
        M = dV * (P.conj() @ W.T)
        assert np.max(np.abs(M - M.conj().T)) <= 1e-12 * np.max(np.abs(M))
        assert np.max(np.linalg.eigvalsh(0.5 * (M + M.conj().T))) <= 1e-12 * np.max(np.abs(M))


def test_bloch_exchange_energy_identity_and_time_reversal(kset):
    dV = float(np.prod(kset["h"]))
    psi, vx, occ, wk = kset["psi"], kset["vx"], kset["occ"], kset["wk"]
    e = 0.25 * sum(wk[k] * occ[k][j] * dV * np.vdot(psi[k, j], vx[k, j]).real
                   for k in range(psi.shape[0]) for j in range(psi.shape[1]))
    assert kset["ex"] < 0.0
    assert abs(e - kset["ex"]) <= 1e-12 * abs(kset["ex"])
    for a, b in ((0, 1), (2, 3)):
        assert np.max(np.abs(vx[b] - np.conj(vx[a]))) <= 1e-12 * np.max(np.abs(vx[a]))


def test_bloch_orbitals_are_orthonormal_bloch_functions():
    n, h = (8, 9, 10), (0.4, 0.4, 0.4)
    kpts = [(0.25, -0.5, 0.0)]
    psi = bloch_orbitals(n, h, P3, kpts, 4, seed=3, n_centres=8)
    dV = 0.4 ** 3
    P = psi[0].reshape(4, -1)
    assert np.max(np.abs(dV * P.conj() @ P.T - np.eye(4))) <= 1e-12


def test_complex_ace_reproduces_the_kpoint_exchange():
    # the compressed exchange of one k-point (Sec. IV, with the Bloch
    # exchange of Sec. II): V_ACE psi_nk = (Vx psi)_nk on the orbitals; as a
    # matrix on a tiny grid it is Hermitian, negative semidefinite, of rank
    # norb, equal to the projector form W M^{-1} W^H (explicit inverse), and
    # zero on fields orthogonal to every W.
    n, h, order = (5, 4, 6), (0.5, 0.5, 0.5), 4
    kpts = [(0.25, 0.0, 0.0), (-0.25, 0.5, 0.0)]
    psi = bloch_orbitals(n, h, P3, kpts, 3, seed=31, n_centres=4)
    wk, occ = [0.5, 0.5], [[1.0, 0.7, 0.4], [0.9, 0.6, 0.3]]
    vx, _ = orc.exchange_bloch(psi, kpts, wk, occ, n, h, order, P3, "erfc", 0.3)
    dV = h[0] * h[1] * h[2]
    N = n[0] * n[1] * n[2]
    for k in range(2):
        xi = orc.ace_build_complex(psi[k], vx[k], dV)
        got = orc.ace_apply_complex(xi, psi[k], dV)
        assert np.max(np.abs(got - vx[k])) <= 1e-12 * np.max(np.abs(vx[k]))
        # dense matrix of the operator
        E = np.eye(N).reshape(N, n[2], n[1], n[0]).astype(np.complex128)
        A = orc.ace_apply_complex(xi, E, dV).reshape(N, N).T
        assert np.allclose(A, A.conj().T, atol=1e-12 * np.max(np.abs(A)))
        ev = np.linalg.eigvalsh(A)
        assert ev.max() <= 1e-12 * abs(ev.min())
        assert np.sum(np.abs(ev) > 1e-9 * abs(ev.min())) == 3
        Wm = vx[k].reshape(3, N)
        M = dV * np.conj(psi[k].reshape(3, N)) @ Wm.T
        P = -Wm.T @ np.linalg.inv(M) @ np.conj(Wm) * dV
        assert np.allclose(A, -P, atol=1e-10 * np.max(np.abs(A)))
        # a field orthogonal to every W
        rng = np.random.default_rng(k)
        f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        Q, _ = np.linalg.qr(Wm.T)  # orthonormal basis of span{W_j}
        f -= Q @ (np.conj(Q.T) @ f)
        out = orc.ace_apply_complex(xi, f.reshape(1, n[2], n[1], n[0]), dV)
        assert np.max(np.abs(out)) <= 1e-10 * np.max(np.abs(f))

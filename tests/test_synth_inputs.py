"""The seeded input generator: deterministic, orthonormal, correct layout."""
import numpy as np

from synth import WORKLOADS, gaussian_orbitals, make_workload, orthonormalise_cgs2


def test_small_workloads_orthonormal_and_deterministic():
    for name in ("dirichlet20x27x34_coulomb", "mixed40x36x44_erfc", "dirichlet32_coulomb"):
        w, psi, occ = make_workload(name)
        assert psi.shape == (w.norb, w.n[2], w.n[1], w.n[0])
        Q = psi.reshape(w.norb, -1)
        G = w.dV * Q @ Q.T
        assert np.max(np.abs(G - np.eye(w.norb))) < 1e-12
        _, psi2, _ = make_workload(name)
        assert np.array_equal(psi, psi2)
        assert np.all(occ == w.occ)


def test_gaussian_axis_layout():
    # one Gaussian on a non-cubic grid: its maximum sits at the drawn centre,
    # with axis 1 the fastest-varying index
    n, h = (30, 20, 10), (0.3, 0.3, 0.3)
    psi = gaussian_orbitals(n, h, ("periodic",) * 3, 1, 3, 1, True)
    assert psi.shape == (1, 10, 20, 30)
    i3, i2, i1 = np.unravel_index(np.argmax(np.abs(psi[0])), psi[0].shape)
    rng = np.random.default_rng(3)
    u = rng.random((1, 3))
    c = u[0] * np.array(n) * np.array(h)
    assert abs(i1 * h[0] - c[0]) <= h[0] and abs(i2 * h[1] - c[1]) <= h[1] and abs(i3 * h[2] - c[2]) <= h[2]


def test_cgs2_matches_qr_span():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 200))
    Q = orthonormalise_cgs2(A, 0.5)
    assert np.max(np.abs(0.5 * Q @ Q.T - np.eye(7))) < 1e-13
    # same flag of subspaces as a QR factorisation (Q = R^-T A, R upper triangular)
    R = 0.5 * Q @ A.T
    assert np.max(np.abs(np.tril(R, -1))) < 1e-12 * np.max(np.abs(R))


def test_workload_table():
    w = WORKLOADS["periodic96_erfc"]
    assert w.npairs == 8256 and w.N == 96 ** 3
    assert w.flops_per_pair() == 4 * 96 ** 3 * 288
    assert WORKLOADS["dirichlet32_coulomb"].npairs == 36

"""FP64 reference for the exact-exchange hot path of the Kronecker-product
real-space formalism (Jing & Suryanarayana, "Efficient real space formalism
for hybrid density functionals").

TEST INFRASTRUCTURE ONLY: this module is the oracle that the HIP library is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the library never does.  It shares no code with
the HIP path (no common tables, weights, eigen-solvers or kernels).

What it computes, in the paper's order:

* Sec. III, Eqs. (11)-(12): the discrete Laplacian is a Kronecker sum of 1-D
  centred finite-difference second-derivative matrices L_k with the boundary
  condition of axis k folded in.
* Eqs. (13)-(16): each L_k is diagonalised; the eigenvectors of L are
  products of the 1-D ones and its eigenvalues are sums of the 1-D ones.
* Eqs. (17)-(20): X = f(L) B with f applied to the summed eigenvalues.
  Reading used here: f acts on the spectrum of -L, f(lam) = 4 pi / lam for
  the unscreened kernel (Sec. II.A, Eq. (5)) and
  f(lam) = 4 pi (1 - exp(-lam / (4 omega^2))) / lam for the erfc-screened one
  (Sec. II.B, Eq. (10)), whose continuum symbol is the Fourier transform of
  erfc(omega r)/r.  The exponent constant printed in Eqs. (10) and (20)
  differs; the tests pin this reading against the closed-form real-space
  potential of a Gaussian charge.
* Eq. (21): the transform is evaluated one axis at a time (mode products),
  forward with V_k^T, a Hadamard product with f(Lambda), inverse with V_k.
* Sec. II.A, Eqs. (3)-(5): the exchange operator on orbital j is
  (Vx psi)_j = -sum_i occ_i phi_ij psi_i with phi_ij = f(-L)(psi_i psi_j),
  and E_x = -1/4 sum_{i,j} occ_i occ_j (rho_ij, phi_ij)_h for a closed shell
  with spin-summed occupations occ (per-spin g = occ/2, two spins).
* Sec. IV: the exchange operator is used in adaptively compressed (ACE)
  form, built from W = Vx psi by a Cholesky factorisation of -(psi, W)_h;
  V_ACE equals Vx on the span of the orbitals.

Arrays are indexed [..., i3, i2, i1] (axis 1 fastest).
Boundary conditions are homogeneous Dirichlet (values outside the n_k nodes
are zero) or periodic.
"""
from __future__ import annotations

import dataclasses
import math
from fractions import Fraction

import numpy as np

FOUR_PI = 4.0 * math.pi


# --------------------------------------------------------------------------
# Sec. III: 1-D finite-difference second-derivative matrices
# --------------------------------------------------------------------------
def fd_weights(order: int) -> list:
    """Centred FD weights w_0..w_m (m = order/2) for d^2/dx^2, as exact
    rationals.

    Taylor expansion of sum_p w_|p| f(x + p h) gives the moment conditions
    sum_{p=-m}^{m} w_|p| p^(2k) = 2 delta_{k,1} for k = 0..m; this solves that
    (m+1)x(m+1) system by Gaussian elimination over the rationals.
    """
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    m = order // 2
    # Row k: coefficient of w_0 is [k == 0]; of w_p (p>=1) is 2 p^(2k).
    rows = []
    for k in range(m + 1):
        row = [Fraction(1 if k == 0 else 0)]
        row += [Fraction(2 * p ** (2 * k)) for p in range(1, m + 1)]
        row.append(Fraction(2 if k == 1 else 0))
        rows.append(row)
    nvar = m + 1
    for col in range(nvar):
        piv = next(r for r in range(col, nvar) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        pv = rows[col][col]
        rows[col] = [x / pv for x in rows[col]]
        for r in range(nvar):
            if r != col and rows[r][col] != 0:
                fac = rows[r][col]
                rows[r] = [a - fac * b for a, b in zip(rows[r], rows[col])]
    return [rows[k][nvar] for k in range(nvar)]


def laplacian_1d(n: int, h: float, order: int, bc: str) -> np.ndarray:
    """n x n matrix L_k approximating d^2/dx^2 on n nodes of spacing h.

    Dirichlet: L[i, j] = w_|i-j| / h^2 for |i-j| <= m (neighbours outside the
    grid are zero).  Periodic: every stencil entry is wrapped modulo n and
    added, so entries that land on the same column sum.
    """
    w = [float(x) for x in fd_weights(order)]
    m = order // 2
    L = np.zeros((n, n))
    for i in range(n):
        for p in range(-m, m + 1):
            j = i + p
            if bc == "dirichlet":
                if 0 <= j < n:
                    L[i, j] += w[abs(p)]
            elif bc == "periodic":
                L[i, j % n] += w[abs(p)]
            else:
                raise ValueError(bc)
    return L / (h * h)


# --------------------------------------------------------------------------
# Eqs. (13)-(16): per-axis eigendecompositions
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    n: tuple
    h: tuple
    order: int
    bc: tuple
    lam: tuple      # eigenvalues of -L_k, ascending
    V: tuple        # V_k[:, a] = eigenvector a of -L_k

    @property
    def dV(self) -> float:
        return self.h[0] * self.h[1] * self.h[2]

    @property
    def shape3(self) -> tuple:
        return (self.n[2], self.n[1], self.n[0])

    def lam_sum(self) -> np.ndarray:
        """lam1[a] + lam2[b] + lam3[c] indexed [c, b, a] (the diagonal of Lambda)."""
        l1, l2, l3 = self.lam
        return l3[:, None, None] + l2[None, :, None] + l1[None, None, :]


def make_grid(n, h, order, bc) -> Grid:
    lams, Vs = [], []
    for k in range(3):
        A = -laplacian_1d(n[k], h[k], order, bc[k])
        lam, V = np.linalg.eigh(A)
        lams.append(lam)
        Vs.append(V)
    return Grid(tuple(n), tuple(h), order, tuple(bc), tuple(lams), tuple(Vs))


# --------------------------------------------------------------------------
# Eqs. (17)-(20): f applied to the spectrum of -L
# --------------------------------------------------------------------------
def kernel_values(lam: np.ndarray, kernel: str, omega: float = 0.0) -> np.ndarray:
    """f(lam) for lam in the spectrum of -L.

    coulomb: 4 pi / lam.
    erfc:    4 pi (1 - exp(-lam/(4 omega^2))) / lam
           = (pi / omega^2) * g(x),  x = lam / (4 omega^2),  g(x) = -expm1(-x)/x,
             g(0) = 1.
    """
    lam = np.asarray(lam, dtype=np.float64)
    if kernel == "coulomb":
        if np.any(lam <= 0.0):
            raise ZeroDivisionError("unscreened kernel on a spectrum containing zero")
        return FOUR_PI / lam
    if kernel == "erfc":
        if not omega > 0.0:
            raise ValueError("omega must be positive")
        x = lam / (4.0 * omega * omega)
        safe = np.where(x == 0.0, 1.0, x)
        g = np.where(x == 0.0, 1.0, -np.expm1(-safe) / safe)
        return (math.pi / (omega * omega)) * g
    raise ValueError(kernel)


def kernel_values_zero_mode(lam: np.ndarray, kernel: str, omega: float = 0.0,
                            zero_mode: float | None = None) -> np.ndarray:
    """kernel_values, except that with the unscreened kernel and zero_mode
    given, f at the zero eigenvalue (|lam| <= 1e-9 max |lam|: the constant
    mode of an all-periodic grid at the Gamma point) is zero_mode.  For 3D
    bulk systems the paper takes that value from auxiliary functions (Sec.
    IV); here it is an input."""
    lam = np.asarray(lam, dtype=np.float64)
    if kernel != "coulomb" or zero_mode is None:
        return kernel_values(lam, kernel, omega)
    zero = np.abs(lam) <= 1e-9 * np.max(np.abs(lam))
    out = np.empty_like(lam)
    out[~zero] = kernel_values(lam[~zero], kernel, omega)
    out[zero] = float(zero_mode)
    return out


def _mode(T: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """out[..., j, ...] = sum_i M[i, j] T[..., i, ...] along ``axis``."""
    out = np.tensordot(T, M, axes=([axis], [0]))
    return np.moveaxis(out, -1, axis)


def forward_transform(rho: np.ndarray, grid: Grid) -> np.ndarray:
    """B~ = (V1 (x) V2 (x) V3)^T rho, Eq. (21b) before the Hadamard product:
    axis 1 then axis 2 on every frontal slice, then axis 3."""
    V1, V2, V3 = grid.V
    T = _mode(rho, V1, -1)
    T = _mode(T, V2, -2)
    T = _mode(T, V3, -3)
    return T


def inverse_transform(X: np.ndarray, grid: Grid) -> np.ndarray:
    """X = (V1 (x) V2 (x) V3) X~, Eq. (21a)."""
    V1, V2, V3 = grid.V
    T = _mode(X, V1.T, -1)
    T = _mode(T, V2.T, -2)
    T = _mode(T, V3.T, -3)
    return T


def apply_fL(rho: np.ndarray, grid: Grid, kernel: str, omega: float = 0.0,
             F: np.ndarray | None = None) -> np.ndarray:
    """phi = f(-L) rho for rho of shape (..., n3, n2, n1), Eqs. (20)-(21)."""
    if F is None:
        F = kernel_values(grid.lam_sum(), kernel, omega)
    return inverse_transform(F * forward_transform(rho, grid), grid)


# --------------------------------------------------------------------------
# Sec. II: exchange operator and energy
# --------------------------------------------------------------------------
def pair_potential(psi_i, psi_j, grid, kernel, omega=0.0, F=None):
    """phi_ij = f(-L)(psi_i psi_j), the solution of Eq. (5) or Eq. (10)."""
    return apply_fL(np.asarray(psi_i, np.float64) * np.asarray(psi_j, np.float64),
                    grid, kernel, omega, F)


def pair_energy(psi_i, psi_j, grid, kernel, omega=0.0, F=None):
    """(rho_ij, phi_ij)_h = dV sum_r rho_ij phi_ij."""
    rho = np.asarray(psi_i, np.float64) * np.asarray(psi_j, np.float64)
    phi = apply_fL(rho, grid, kernel, omega, F)
    return grid.dV * float(np.sum(rho * phi))


def exchange(psi, occ, grid, kernel, omega=0.0, pair_energies=False, zero_mode=None):
    """All-pairs exact exchange, Eqs. (3)-(4) (unscreened) and (8)-(9)
    (screened), for real orbitals psi of shape (norb, n3, n2, n1).

    Loops over the symmetric pairs i <= j: rho = psi_i psi_j,
    phi = f(-L) rho, (Vx psi)_j -= occ_i phi psi_i and, for i != j,
    (Vx psi)_i -= occ_j phi psi_j.  Returns (vx, E_x[, {(i, j): e_ij}]) with
    e_ij = (rho_ij, phi_ij)_h and E_x = -1/4 sum_{i,j} occ_i occ_j e_ij.
    zero_mode: see kernel_values_zero_mode.
    """
    psi = np.asarray(psi, dtype=np.float64)
    norb = psi.shape[0]
    F = kernel_values_zero_mode(grid.lam_sum(), kernel, omega, zero_mode)
    vx = np.zeros_like(psi)
    ex = 0.0
    es = {}
    for i in range(norb):
        for j in range(i, norb):
            rho = psi[i] * psi[j]
            phi = apply_fL(rho, grid, kernel, omega, F)
            e = grid.dV * float(np.sum(rho * phi))
            es[(i, j)] = e
            vx[j] -= occ[i] * phi * psi[i]
            if i != j:
                vx[i] -= occ[j] * phi * psi[j]
            ex -= 0.25 * occ[i] * occ[j] * e * (1.0 if i == j else 2.0)
    if pair_energies:
        return vx, ex, es
    return vx, ex


def vx_orbital(psi, occ, j, grid, kernel, omega=0.0):
    """(Vx psi)_j = -sum_i occ_i phi_ij psi_i for one orbital j."""
    psi = np.asarray(psi, dtype=np.float64)
    F = kernel_values(grid.lam_sum(), kernel, omega)
    out = np.zeros_like(psi[j])
    for i in range(psi.shape[0]):
        phi = apply_fL(psi[i] * psi[j], grid, kernel, omega, F)
        out -= occ[i] * phi * psi[i]
    return out


# --------------------------------------------------------------------------
# Sec. IV: the exchange operator in adaptively compressed (ACE) form, the
# form in which the exchange enters the self-consistent iteration (the
# construction of Lin, J. Chem. Theory Comput. 12, 2242 (2016))
# --------------------------------------------------------------------------
def ace_build(psi, W, dV):
    """Compressed exchange vectors xi (norb, ...) from the orbitals psi and
    W = Vx psi (both (norb, n3, n2, n1)):

      M = (psi_j, W_k)_h                (norb x norb, symmetric, negative definite)
      -M = L L^T                        (Cholesky, L lower with positive diagonal)
      xi = L^{-1} W                     (row k of xi is xi_k)

    so that V_ACE phi = -sum_k xi_k (xi_k, phi)_h (ace_apply) reproduces
    Vx on the span of the orbitals.  Raises numpy.linalg.LinAlgError when -M
    is not positive definite."""
    psi = np.asarray(psi, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    norb = psi.shape[0]
    P = psi.reshape(norb, -1)
    Wm = W.reshape(norb, -1)
    M = dV * (P @ Wm.T)
    L = np.linalg.cholesky(-M)
    xi = np.linalg.solve(L, Wm)  # forward substitution written as a dense solve
    return xi.reshape(W.shape)


def ace_apply(xi, phi, dV):
    """V_ACE phi = -sum_k xi_k (xi_k, phi_v)_h for fields phi (nvec, ...)."""
    xi = np.asarray(xi, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    norb, nvec = xi.shape[0], phi.shape[0]
    X = xi.reshape(norb, -1)
    F = phi.reshape(nvec, -1)
    G = dV * (X @ F.T)          # (xi_k, phi_v)_h
    return (-(G.T @ X)).reshape(phi.shape)


def ace_build_complex(psi, W, dV):
    """The compressed exchange of one k-point (complex Bloch orbitals psi and
    W = (Vx psi) at that k, both (norb, n3, n2, n1) complex):

      M = (psi_j, W_k)_h = dV sum conj(psi_j) W_k    (Hermitian, negative definite)
      -M = L L^H                                      (Cholesky)
      xi = L^{-*} W, i.e. xi_k = sum_j conj((L^{-1})_kj) W_j

    so that V_ACE phi = -sum_k xi_k (xi_k, phi)_h (ace_apply_complex)
    reproduces Vx on the span of the orbitals."""
    psi = np.asarray(psi, dtype=np.complex128)
    W = np.asarray(W, dtype=np.complex128)
    norb = psi.shape[0]
    P = psi.reshape(norb, -1)
    Wm = W.reshape(norb, -1)
    M = dV * (np.conj(P) @ Wm.T)
    L = np.linalg.cholesky(-M)
    xi = np.linalg.solve(np.conj(L), Wm)
    return xi.reshape(W.shape)


def ace_apply_complex(xi, phi, dV):
    """V_ACE phi = -sum_k xi_k (xi_k, phi_v)_h for complex fields phi (nvec, ...)."""
    xi = np.asarray(xi, dtype=np.complex128)
    phi = np.asarray(phi, dtype=np.complex128)
    norb, nvec = xi.shape[0], phi.shape[0]
    X = xi.reshape(norb, -1)
    F = phi.reshape(nvec, -1)
    G = dV * (np.conj(X) @ F.T)          # (xi_k, phi_v)_h
    return (-(G.T @ X)).reshape(phi.shape)


# --------------------------------------------------------------------------
# Sec. IV: isolated systems.  The unscreened problem on an all-Dirichlet grid
# takes its boundary values from the multipole expansion of the Coulomb
# kernel, enforced by modifying the right-hand side.
# --------------------------------------------------------------------------
def node_coords(n, h):
    """Coordinates of the grid nodes along each axis: x_i = i h (i = 0..n-1)."""
    return tuple(np.arange(n[k], dtype=np.float64) * h[k] for k in range(3))


def _spherical(x, y, z):
    r = np.sqrt(x * x + y * y + z * z)
    cos_t = np.where(r > 0.0, z / np.where(r > 0.0, r, 1.0), 1.0)
    phi = np.arctan2(y, x)
    return r, cos_t, phi


def multipole_moments(rho, grid, centre, lmax):
    """Moments of a charge density (n3, n2, n1) about `centre`:
      A[l, m] = dV sum_r rho(r) |r-c|^l P_l^m(cos t) cos(m p),
      B[l, m] = dV sum_r rho(r) |r-c|^l P_l^m(cos t) sin(m p),   0 <= m <= l <= lmax,
    with (|r-c|, t, p) the spherical coordinates of r - c and P_l^m the
    associated Legendre function (scipy.special.lpmv)."""
    from scipy.special import lpmv
    x1, x2, x3 = node_coords(grid.n, grid.h)
    Z, Y, X = np.meshgrid(x3 - centre[2], x2 - centre[1], x1 - centre[0], indexing="ij")
    r, ct, ph = _spherical(X, Y, Z)
    A = np.zeros((lmax + 1, lmax + 1))
    B = np.zeros((lmax + 1, lmax + 1))
    rho = np.asarray(rho, dtype=np.float64)
    for l in range(lmax + 1):
        rl = r ** l
        for m in range(l + 1):
            P = lpmv(m, l, ct)
            A[l, m] = grid.dV * float(np.sum(rho * rl * P * np.cos(m * ph)))
            B[l, m] = grid.dV * float(np.sum(rho * rl * P * np.sin(m * ph)))
    return A, B


def multipole_potential(A, B, points, centre):
    """The Coulomb potential of the expanded charge at points (..., 3) outside
    the charge, by the addition theorem for 1/|r - r'|:
      phi(r) = sum_l sum_m (2 - delta_m0) (l-m)!/(l+m)! P_l^m(cos t) / |r-c|^(l+1)
                          * (A[l, m] cos(m p) + B[l, m] sin(m p))."""
    from scipy.special import lpmv
    pts = np.asarray(points, dtype=np.float64)
    r, ct, ph = _spherical(pts[..., 0] - centre[0], pts[..., 1] - centre[1],
                           pts[..., 2] - centre[2])
    lmax = A.shape[0] - 1
    out = np.zeros(r.shape)
    for l in range(lmax + 1):
        inv = 1.0 / r ** (l + 1)
        for m in range(l + 1):
            ratio = math.factorial(l - m) / math.factorial(l + m)
            w = (1.0 if m == 0 else 2.0) * ratio
            out += w * lpmv(m, l, ct) * inv * (A[l, m] * np.cos(m * ph) + B[l, m] * np.sin(m * ph))
    return out


def multipole_rhs_correction(rho, grid, centre, lmax):
    """c (n3, n2, n1): for every node, the stencil weights that reach nodes
    outside the grid times the expanded potential there,
      c(x) = sum_k sum_{p: x + p e_k outside} (w_|p| / h_k^2) phi_ext(x + p e_k),
    so that the full stencil at x reads (L_D phi)(x) + c(x).  Requires
    Dirichlet on every axis."""
    if any(b != "dirichlet" for b in grid.bc):
        raise ValueError("the multipole boundary values are for all-Dirichlet grids")
    A, B = multipole_moments(rho, grid, centre, lmax)
    w = [float(v) for v in fd_weights(grid.order)]
    mrad = grid.order // 2
    x1, x2, x3 = node_coords(grid.n, grid.h)
    axes = (x1, x2, x3)
    n1, n2, n3 = grid.n
    c = np.zeros((n3, n2, n1))
    for k in range(3):
        nk, hk = grid.n[k], grid.h[k]
        for i in range(nk):
            for p in range(1, mrad + 1):
                for j in (i - p, i + p):
                    if 0 <= j < nk:
                        continue
                    # the outside node: axis k at index j, the other axes on the grid
                    coords = [axes[0], axes[1], axes[2]]
                    coords[k] = np.array([j * hk])
                    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
                    pts = np.stack([X, Y, Z], axis=-1)
                    val = (w[p] / (hk * hk)) * multipole_potential(A, B, pts, centre)
                    sl = [slice(None)] * 3
                    sl[2 - k] = slice(i, i + 1)
                    c[tuple(sl)] += val
    return c


def apply_coulomb_multipole(rho, grid, centre, lmax):
    """phi = (-L_D)^{-1} (4 pi rho + c) for one density (n3, n2, n1): the
    unscreened problem with boundary values from the multipole expansion,
    through the same Kronecker solve as apply_fL (f = 4 pi / lam applied to
    rho + c / (4 pi))."""
    c = multipole_rhs_correction(rho, grid, centre, lmax)
    return apply_fL(np.asarray(rho, dtype=np.float64) + c / FOUR_PI, grid, "coulomb")


def exchange_multipole(psi, occ, grid, centre, lmax):
    """The unscreened exact exchange of an isolated system (Sec. II with the
    boundary values of Sec. IV): for every symmetric pair i <= j,
    phi_ij = apply_coulomb_multipole(psi_i psi_j), (Vx psi)_j -= occ_i phi_ij psi_i
    and, for i != j, (Vx psi)_i -= occ_j phi_ij psi_j;
    E_x = -1/4 sum_{i,j} occ_i occ_j (rho_ij, phi_ij)_h.  Returns (vx, E_x)."""
    psi = np.asarray(psi, dtype=np.float64)
    norb = psi.shape[0]
    vx = np.zeros_like(psi)
    ex = 0.0
    for i in range(norb):
        for j in range(i, norb):
            rho = psi[i] * psi[j]
            phi = apply_coulomb_multipole(rho, grid, centre, lmax)
            e = grid.dV * float(np.sum(rho * phi))
            vx[j] -= occ[i] * phi * psi[i]
            if i != j:
                vx[i] -= occ[j] * phi * psi[j]
            ex -= 0.25 * occ[i] * occ[j] * e * (1.0 if i == j else 2.0)
    return vx, ex


# --------------------------------------------------------------------------
# Sec. II with Brillouin-zone sampling: the Poisson problem for the pair
# (m q, n k) carries Bloch boundary conditions at the wavevector k - q along
# the extended (periodic) directions.  On the grid, a periodic axis of n
# nodes then wraps its stencil with the phase u(x + n h) = e^{i theta} u(x),
# theta = 2 pi (k - q)_a in reduced coordinates.
# --------------------------------------------------------------------------
def laplacian_1d_bloch(n: int, h: float, order: int, theta: float) -> np.ndarray:
    """n x n complex Hermitian L_k: the centred stencil with every entry that
    wraps past the end of the period multiplied by e^{+i theta} (one period
    forward) or e^{-i theta} (one period back)."""
    w = [float(x) for x in fd_weights(order)]
    m = order // 2
    L = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for p in range(-m, m + 1):
            j = i + p
            wrap = j // n  # -1, 0 or +1 periods (more for tiny n)
            L[i, j % n] += w[abs(p)] * np.exp(1j * theta * wrap)
    return L / (h * h)


def make_grid_bloch(n, h, order, bc, theta) -> Grid:
    """Eigendecompositions of -L_k(theta_k) (numpy eigh, complex Hermitian on
    periodic axes; Dirichlet axes take no phase and must have theta_k = 0)."""
    lams, Vs = [], []
    for k in range(3):
        if bc[k] == "periodic":
            A = -laplacian_1d_bloch(n[k], h[k], order, theta[k])
        else:
            if theta[k] != 0.0:
                raise ValueError("a Dirichlet axis carries no Bloch phase")
            A = -laplacian_1d(n[k], h[k], order, bc[k])
        lam, V = np.linalg.eigh(A)
        lams.append(lam)
        Vs.append(V)
    return Grid(tuple(n), tuple(h), order, tuple(bc), tuple(lams), tuple(Vs))


def apply_fL_bloch(rho: np.ndarray, grid: Grid, kernel: str, omega: float = 0.0,
                   zero_mode: float | None = None) -> np.ndarray:
    """phi = f(-L) rho for complex rho (..., n3, n2, n1) with the complex
    eigenbases of a Bloch grid: coefficients V^H rho mode by mode, the Hadamard
    product with f of the summed eigenvalues, then V back (Eqs. (17)-(21))."""
    V1, V2, V3 = grid.V
    F = kernel_values_zero_mode(grid.lam_sum(), kernel, omega, zero_mode)
    T = _mode(np.asarray(rho, dtype=np.complex128), V1.conj(), -1)
    T = _mode(T, V2.conj(), -2)
    T = _mode(T, V3.conj(), -3)
    T = F * T
    T = _mode(T, V1.T, -1)
    T = _mode(T, V2.T, -2)
    T = _mode(T, V3.T, -3)
    return T


def bloch_phases(kq, bc):
    """theta per axis for the reduced wavevector difference kq (3,): 2 pi kq_a on
    periodic axes, 0 on Dirichlet axes (which must have kq_a = 0)."""
    out = []
    for a in range(3):
        if bc[a] == "periodic":
            out.append(2.0 * math.pi * float(kq[a]))
        else:
            if float(kq[a]) != 0.0:
                raise ValueError("a Dirichlet axis carries no wavevector component")
            out.append(0.0)
    return tuple(out)


def exchange_bloch(psi, kpts, wk, occ, n, h, order, bc, kernel, omega=0.0, zero_mode=None):
    """Exact exchange with Brillouin-zone sampling for one spin channel,
    Sec. II, Eqs. (Vx:Poisson), (Ex:Poisson), (Poisson):
      (Vx psi)_{nk} = - sum_{m q} w_q occ_{mq} psi_{mq} phi_{mq,nk},
      -L phi_{mq,nk} = 4 pi conj(psi_{mq}) psi_{nk}  (Bloch at k - q),
      E_x = -1/4 sum_{nk, mq} w_k w_q occ_{nk} occ_{mq} (rho_{mq,nk}, phi_{mq,nk})_h
    with rho_{mq,nk} = conj(psi_{mq}) psi_{nk} and (u, v)_h = dV sum conj(u) v
    (the spin-summed convention of `exchange`: occ = 2 g for a closed shell,
    occ = g per spin channel, whose energy is then half the channel's E_X).
    psi: (K, norb, n3, n2, n1) complex grid values; kpts (K, 3) reduced;
    wk (K,) weights; occ (K, norb).  Every ordered pair is solved.
    zero_mode: f at the zero mode of the k = q problems (kernel_values_zero_mode)."""
    psi = np.asarray(psi, dtype=np.complex128)
    K, norb = psi.shape[:2]
    dV = h[0] * h[1] * h[2]
    grids = {}
    vx = np.zeros_like(psi)
    ex = 0.0
    for ki in range(K):
        for qi in range(K):
            th = bloch_phases(np.asarray(kpts[ki]) - np.asarray(kpts[qi]), bc)
            if th not in grids:
                grids[th] = make_grid_bloch(n, h, order, bc, th)
            grid = grids[th]
            for nb in range(norb):
                for mb in range(norb):
                    rho = np.conj(psi[qi, mb]) * psi[ki, nb]
                    phi = apply_fL_bloch(rho, grid, kernel, omega, zero_mode)
                    vx[ki, nb] -= wk[qi] * occ[qi][mb] * psi[qi, mb] * phi
                    e = dV * complex(np.sum(np.conj(rho) * phi))
                    ex -= 0.25 * wk[ki] * wk[qi] * occ[ki][nb] * occ[qi][mb] * e.real
    return vx, ex


# --------------------------------------------------------------------------
# Sec. III, closing remark: non-orthogonal cells with periodic or
# Bloch-periodic conditions on every axis.  With unit lattice directions e_a
# (the columns of E) and node i_a at xi_a = i_a h_a along e_a, the Laplacian
# in lattice coordinates is sum_ab g_ab d^2/(dxi_a dxi_b), g = E^-1 E^-T: the
# diagonal terms take the second-derivative matrices L_a, the mixed terms
# products of first-derivative matrices D_a D_b (which share the eigenbasis
# of L_a on a periodic axis).
# --------------------------------------------------------------------------
def fd_weights_d1(order: int) -> list:
    """Centred FD weights d_1..d_m (m = order/2) for d/dx, d_{-p} = -d_p and
    d_0 = 0, as exact rationals.

    Taylor expansion of sum_p d_p f(x + p h) gives the moment conditions
    sum_{p=-m}^{m} d_p p^(2k-1) = delta_{k,1} for k = 1..m, i.e.
    2 sum_{p>=1} d_p p^(2k-1) = delta_{k,1}; solved by Gaussian elimination
    over the rationals."""
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    m = order // 2
    rows = []
    for k in range(1, m + 1):
        row = [Fraction(2 * p ** (2 * k - 1)) for p in range(1, m + 1)]
        row.append(Fraction(1 if k == 1 else 0))
        rows.append(row)
    for col in range(m):
        piv = next(r for r in range(col, m) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        pv = rows[col][col]
        rows[col] = [x / pv for x in rows[col]]
        for r in range(m):
            if r != col and rows[r][col] != 0:
                fac = rows[r][col]
                rows[r] = [a - fac * b for a, b in zip(rows[r], rows[col])]
    return [rows[k][m] for k in range(m)]


def derivative_1d_bloch(n: int, h: float, order: int, theta: float) -> np.ndarray:
    """n x n complex D_k approximating d/dx on a periodic axis with the Bloch
    phase theta: D[i, (i + p) mod n] += sgn(p) d_|p| e^{i theta wrap} / h,
    wrap = floor((i + p) / n) periods (as in laplacian_1d_bloch)."""
    d = [float(x) for x in fd_weights_d1(order)]
    m = order // 2
    D = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for p in range(-m, m + 1):
            if p == 0:
                continue
            j = i + p
            dp = d[p - 1] if p > 0 else -d[-p - 1]
            D[i, j % n] += dp * np.exp(1j * theta * (j // n))
    return D / h


def cell_metric(lattice):
    """lattice: 3 x 3, row a the direction of lattice axis a (any length).
    Returns (g, jac): g = E^-1 E^-T with E the unit directions as columns,
    and jac = |det E|, the volume of a grid cell over h1 h2 h3."""
    A = np.asarray(lattice, dtype=np.float64)
    E = (A / np.linalg.norm(A, axis=1)[:, None]).T
    Ei = np.linalg.inv(E)
    return Ei @ Ei.T, abs(float(np.linalg.det(E)))


def laplacian_cell(n, h, order, lattice, theta) -> np.ndarray:
    """Dense N x N (complex) Laplacian of the lattice-coordinate form on an
    all-periodic grid with Bloch phases theta[a], field index
    (i3 n2 + i2) n1 + i1 (axis 1 fastest):
      L = sum_a g_aa L_a(theta_a) + sum_{a != b} g_ab D_a(theta_a) D_b(theta_b),
    each 1-D matrix acting in its own slot of the Kronecker product."""
    g, _ = cell_metric(lattice)
    L1 = [laplacian_1d_bloch(n[a], h[a], order, theta[a]) for a in range(3)]
    D1 = [derivative_1d_bloch(n[a], h[a], order, theta[a]) for a in range(3)]
    eye = [np.eye(n[a]) for a in range(3)]

    def slot(ops):
        # ops[a] acts on axis a; axis 3 is the slowest Kronecker factor
        return np.kron(ops[2], np.kron(ops[1], ops[0]))

    N = n[0] * n[1] * n[2]
    L = np.zeros((N, N), dtype=np.complex128)
    for a in range(3):
        ops = list(eye)
        ops[a] = L1[a]
        L += g[a, a] * slot(ops)
    for a in range(3):
        for b in range(3):
            if a != b and g[a, b] != 0.0:
                ops = list(eye)
                ops[a] = D1[a]
                ops[b] = D1[b]
                L += g[a, b] * slot(ops)
    return L


def apply_fL_cell(rho, n, h, order, lattice, theta, kernel, omega=0.0, eig=None):
    """phi = f(-L) rho for complex rho (..., n3, n2, n1) on a non-orthogonal
    all-periodic cell, by the dense eigendecomposition of the Hermitian -L
    (f(-L) = U f(lam) U^H).  eig: a precomputed (lam, U) of -L."""
    if eig is None:
        eig = np.linalg.eigh(-laplacian_cell(n, h, order, lattice, theta))
    lam, U = eig
    F = kernel_values(lam, kernel, omega)
    r = np.asarray(rho, dtype=np.complex128)
    flat = r.reshape(-1, n[0] * n[1] * n[2])
    out = (U @ (F[:, None] * (U.conj().T @ flat.T))).T
    return out.reshape(r.shape)


def exchange_cell(psi, kpts, wk, occ, n, h, order, lattice, kernel, omega=0.0):
    """exchange_bloch on a non-orthogonal all-periodic cell: the same sums
    over ordered state pairs, each pair solved with the dense f(-L) of its
    phases 2 pi (k - q), and (u, v)_h = h1 h2 h3 jac sum conj(u) v."""
    psi = np.asarray(psi, dtype=np.complex128)
    K, norb = psi.shape[:2]
    _, jac = cell_metric(lattice)
    dV = h[0] * h[1] * h[2] * jac
    bc = ("periodic",) * 3
    eigs = {}
    vx = np.zeros_like(psi)
    ex = 0.0
    for ki in range(K):
        for qi in range(K):
            th = bloch_phases(np.asarray(kpts[ki]) - np.asarray(kpts[qi]), bc)
            if th not in eigs:
                eigs[th] = np.linalg.eigh(-laplacian_cell(n, h, order, lattice, th))
            for nb in range(norb):
                for mb in range(norb):
                    rho = np.conj(psi[qi, mb]) * psi[ki, nb]
                    phi = apply_fL_cell(rho, n, h, order, lattice, th, kernel, omega, eigs[th])
                    vx[ki, nb] -= wk[qi] * occ[qi][mb] * psi[qi, mb] * phi
                    e = dV * complex(np.sum(np.conj(rho) * phi))
                    ex -= 0.25 * wk[ki] * wk[qi] * occ[ki][nb] * occ[qi][mb] * e.real
    return vx, ex

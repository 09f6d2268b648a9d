"""Non-orthogonal all-periodic cells on the GPU against the oracle (Sec. III,
closing remark): f(-L) with mixed derivatives through the Bloch entry points
on hexagonal and general skewed cells, with and without Bloch phases; the
k-point exchange and its energy with the cell's volume element; the error
statuses of kx_set_cell and of the real entry points while a cell is set."""
import math

import numpy as np
import pytest

import oracle as orc
from synth import bloch_orbitals

pytestmark = pytest.mark.gpu

TOL = 1e-10
P3 = ("periodic",) * 3
HEX = [[1.0, 0.0, 0.0], [-0.5, math.sqrt(3) / 2, 0.0], [0.0, 0.0, 1.0]]
SKEW = [[1.0, 0.0, 0.0], [0.3, 1.0, 0.0], [0.2, -0.25, 1.0]]
# rows of any length, a cell tilted out of every plane
TILT = [[2.0, 0.1, -0.3], [0.4, 1.5, 0.2], [-0.1, 0.35, 0.9]]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def kx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_16998_amd import kx as _kx
    _kx.lib()
    return _kx


def _cfields(n, batch, seed):
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    return rng.standard_normal((batch, n3, n2, n1)) + 1j * rng.standard_normal((batch, n3, n2, n1))


# (n, h, order, lattice, theta, kernel, omega, batch)
CASES = [
    ((8, 7, 6), (0.5, 0.45, 0.4), 4, HEX, (0.0, 0.0, 0.0), "erfc", 0.3, 2),
    ((9, 8, 7), (0.5, 0.45, 0.4), 8, SKEW, (0.7, -1.9, 2.5), "erfc", 0.25, 3),
    ((7, 9, 8), (0.4, 0.45, 0.5), 12, TILT, (1.1, 0.4, -0.6), "coulomb", 0.0, 2),
    ((10, 6, 9), (0.45, 0.5, 0.4), 6, HEX, (math.pi, 0.3, 0.0), "coulomb", 0.0, 1),
]


@pytest.mark.parametrize("n,h,order,lattice,theta,kernel,omega,batch", CASES)
def test_cell_solve_parity(kx, n, h, order, lattice, theta, kernel, omega, batch):
    import torch
    print(f"cell solve n={n} order={order} theta={theta} {kernel}", flush=True)
    rho = _cfields(n, batch, seed=sum(n) + order)
    ref = orc.apply_fL_cell(rho, n, h, order, lattice, theta, kernel, omega)
    with kx.Grid(n, h, order, P3) as g:
        g.set_cell(lattice)
        out = g.apply_fL_bloch(torch.from_numpy(rho).cuda(), theta, kernel, omega)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    assert _rel(got, ref) <= TOL


@pytest.mark.parametrize("lattice,kpts,norb", [
    (SKEW, [(0.0, 0.0, 0.0), (0.5, 0.0, 0.25)], 2),
    (HEX, [(0.0, 0.0, 0.0), (1 / 3, 1 / 3, 0.0), (0.5, 0.0, 0.5)], 2),
])
def test_cell_exchange_parity(kx, lattice, kpts, norb):
    import torch
    n, h, order = (7, 6, 8), (0.5, 0.5, 0.45), 6
    print(f"cell exchange nk={len(kpts)} norb={norb}", flush=True)
    psi = bloch_orbitals(n, h, P3, kpts, norb, seed=31, n_centres=5)
    nk = len(kpts)
    wk = np.full(nk, 1.0 / nk)
    occ = np.linspace(1.0, 0.5, nk * norb).reshape(nk, norb)
    vx_ref, ex_ref = orc.exchange_cell(psi, kpts, wk, occ, n, h, order, lattice, "erfc", 0.3)
    with kx.Grid(n, h, order, P3) as g:
        g.set_cell(lattice)
        vx = g.apply_exchange_bloch(torch.from_numpy(psi).cuda(), kpts, wk, occ, "erfc", 0.3)
        torch.cuda.synchronize()
        assert _rel(vx.cpu().numpy(), vx_ref) <= TOL
        assert abs(g.exchange_energy() - ex_ref) <= TOL * abs(ex_ref)


def test_cell_statuses(kx):
    import torch
    n, h = (8, 8, 8), (0.5, 0.5, 0.5)
    rho = torch.from_numpy(np.random.default_rng(2).standard_normal((1, 8, 8, 8))).cuda()
    with kx.Grid(n, h, 4, ("periodic", "periodic", "dirichlet")) as g:
        with pytest.raises(kx.KxError) as e:  # mixed derivatives need periodic ends
            g.set_cell(SKEW)
        assert e.value.status == 2
        g.set_cell(np.eye(3) * 2.0)  # an orthogonal cell is always accepted
    with kx.Grid(n, h, 4, P3) as g:
        with pytest.raises(kx.KxError) as e:  # coplanar directions
            g.set_cell([[1, 0, 0], [0, 1, 0], [1, 1, 0]])
        assert e.value.status == 1
        ref = g.apply_fL(rho, "erfc", 0.3)
        g.set_cell(HEX)
        with pytest.raises(kx.KxError) as e:
            g.apply_fL(rho, "erfc", 0.3)
        assert e.value.status == 2
        with pytest.raises(kx.KxError) as e:
            g.apply_exchange(rho, [1.0], "erfc", 0.3)
        assert e.value.status == 2
        g.set_cell(None)
        again = g.apply_fL(rho, "erfc", 0.3)
        torch.cuda.synchronize()
        assert torch.equal(again, ref)

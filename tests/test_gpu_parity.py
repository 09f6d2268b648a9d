"""Parity of the HIP library (through its C ABI) against the FP64 oracle.

FP64 tolerance: 1e-10 relative, as max|GPU - oracle| / max|oracle| per field
(per orbital for Vx psi) and |dE| / |E| for energies.
"""
import json
import os

import numpy as np
import pytest

import oracle as orc
from synth import WORKLOADS, make_workload, random_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
# FP32 mode products: unit roundoff 2^-24 ~ 6e-8, K <= 80 per product, six
# products in sequence -> a few 1e-6 relative per element in the worst case;
# the energy sums many independent roundings and is tighter.
# Split BF16 x3: each FP32 operand is carried exactly by its three terms (24
# significant bits), V_k to ~2^-25; the dropped terms (s + t >= 3) are
# <= 3 * 2^-24 relative and the accumulation is FP32, so the same bounds hold.
TOL32_FIELD = 1e-5
TOL32_ENERGY = 1e-6
REDUCED = ["fp32", "bf16x3", "fp16x3"]
# mixed: FP64 forward pass, f scaling and energies (energies at the FP64
# tolerance), split-BF16 back-transform and Vx psi update (FP32 tolerances)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_energies.json")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_16998_amd import kx
    kx.lib()
    return torch


def _kx():
    from paper_2406_16998_amd import kx
    return kx


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# ------------------------------------------------------------------ eigensystems
EIG_CASES = [(32, 0.3, 12, "dirichlet"), (96, 0.35, 12, "periodic"), (144, 0.3, 12, "periodic"),
             (60, 0.3, 12, "periodic"), (7, 0.4, 12, "periodic"), (1, 0.3, 12, "dirichlet"),
             (120, 0.3, 12, "dirichlet"), (37, 0.3, 2, "dirichlet"), (160, 0.25, 24, "dirichlet")]


@pytest.mark.parametrize("n,h,order,bc", EIG_CASES)
def test_device_eigensystem(torch_cuda, n, h, order, bc):
    kx = _kx()
    print(f"eig n={n} h={h} order={order} bc={bc}", flush=True)
    g = kx.Grid((n, 3, 4), (h, 0.5, 0.5), order, (bc, "dirichlet", "dirichlet"))
    lam, V = g.eigensystem(0)
    g.close()
    A = -orc.laplacian_1d(n, h, order, bc)
    lam_ref = np.linalg.eigvalsh(A)
    scale = max(np.max(np.abs(lam_ref)), 1e-300)
    assert np.max(np.abs(lam - lam_ref)) <= 1e-12 * scale
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13
    assert np.max(np.abs(A @ V - V * lam)) <= 1e-12 * scale


# ------------------------------------------------------------------ apply_fL
FL_CASES = [
    ((40, 36, 44), (0.35, 0.3, 0.4), 12, ("periodic", "dirichlet", "periodic"), "erfc", 0.106),
    ((20, 27, 34), (0.4, 0.35, 0.3), 8, ("dirichlet",) * 3, "coulomb", 0.0),
    ((4, 5, 6), (0.4, 0.3, 0.35), 12, ("dirichlet",) * 3, "coulomb", 0.0),
    ((5, 6, 7), (0.3, 0.3, 0.3), 12, ("periodic", "periodic", "dirichlet"), "erfc", 0.106),
    ((32, 32, 32), (0.3, 0.3, 0.3), 12, ("dirichlet",) * 3, "erfc", 0.5),
    ((17, 33, 16), (0.3, 0.3, 0.3), 12, ("periodic",) * 3, "erfc", 0.106),
    ((48, 16, 1), (0.3, 0.3, 0.3), 12, ("periodic", "dirichlet", "periodic"), "erfc", 0.3),
]


@pytest.mark.parametrize("n,h,order,bc,kernel,omega", FL_CASES)
def test_apply_fL_parity(torch_cuda, n, h, order, bc, kernel, omega):
    torch = torch_cuda
    kx = _kx()
    print(f"apply_fL n={n} bc={bc} kernel={kernel}", flush=True)
    rho = random_fields(n, 3, seed=sum(n))
    g = kx.Grid(n, h, order, bc)
    phi = g.apply_fL(torch.from_numpy(rho).cuda(), kernel, omega).cpu().numpy()
    g.close()
    grid = orc.make_grid(n, h, order, bc)
    ref = orc.apply_fL(rho, grid, kernel, omega)
    for b in range(3):
        assert _rel(phi[b], ref[b]) <= TOL64


def test_apply_fL_chunked_matches_unchunked(torch_cuda, monkeypatch):
    torch = torch_cuda
    kx = _kx()
    n, h, bc = (24, 20, 28), (0.3,) * 3, ("periodic", "dirichlet", "dirichlet")
    rho = torch.from_numpy(random_fields(n, 7, seed=3)).cuda()
    g1 = kx.Grid(n, h, 12, bc)
    a = g1.apply_fL(rho, "erfc", 0.106)
    monkeypatch.setenv("KX_MAX_SLOTS", "2")
    g2 = kx.Grid(n, h, 12, bc)
    b = g2.apply_fL(rho, "erfc", 0.106)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    g1.close()
    g2.close()


# ------------------------------------------------------------------ exchange
def _exchange_case(torch, name, occ=None, max_slots=None, monkeypatch=None):
    kx = _kx()
    w, psi, occ0 = make_workload(name)
    if occ is None:
        occ = occ0
    if max_slots is not None:
        monkeypatch.setenv("KX_MAX_SLOTS", str(max_slots))
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega)
    ex = g.exchange_energy()
    pairs = [(i, j) for i in range(w.norb) for j in range(i, w.norb)]
    pe = g.pair_energies(pairs)
    vx = vx.cpu().numpy()
    g.close()
    return w, psi, occ, vx, ex, dict(zip(pairs, pe))


@pytest.mark.parametrize("name,occ", [
    ("dirichlet20x27x34_coulomb", None),
    ("dirichlet20x27x34_coulomb", [2.0, 1.5, 0.5, 1.0, 0.25]),
    ("mixed40x36x44_erfc", None),
    ("dirichlet32_coulomb", None),
])
def test_exchange_parity_small(torch_cuda, name, occ):
    print(f"exchange {name} occ={occ}", flush=True)
    w, psi, occ, vx, ex, pe = _exchange_case(torch_cuda, name, occ)
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_ref, ex_ref, pe_ref = orc.exchange(psi, occ, grid, w.kernel, w.omega, pair_energies=True)
    for j in range(w.norb):
        assert _rel(vx[j], vx_ref[j]) <= TOL64, j
    assert abs(ex - ex_ref) <= TOL64 * abs(ex_ref)
    for p, e in pe_ref.items():
        assert abs(pe[p] - e) <= TOL64 * abs(e) + 1e-14 * abs(ex_ref), p


def test_exchange_odd_orbital_count_and_chunking(torch_cuda, monkeypatch):
    # 5 orbitals with at most 2 pairs per launch: ragged schedule batches
    w, psi, occ, vx, ex, pe = _exchange_case(torch_cuda, "dirichlet20x27x34_coulomb",
                                             max_slots=2, monkeypatch=monkeypatch)
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_ref, ex_ref = orc.exchange(psi, occ, grid, w.kernel, w.omega)
    assert abs(ex - ex_ref) <= TOL64 * abs(ex_ref)
    for j in range(w.norb):
        assert _rel(vx[j], vx_ref[j]) <= TOL64


def test_exchange_single_orbital_and_empty(torch_cuda):
    torch = torch_cuda
    kx = _kx()
    w, psi, occ = make_workload("mixed40x36x44_erfc")
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    one = np.ascontiguousarray(psi[2:3])
    vx = g.apply_exchange(torch.from_numpy(one).cuda(), [2.0], w.kernel, w.omega).cpu().numpy()
    ex = g.exchange_energy()
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_ref, ex_ref = orc.exchange(one, [2.0], grid, w.kernel, w.omega)
    assert _rel(vx[0], vx_ref[0]) <= TOL64 and abs(ex - ex_ref) <= TOL64 * abs(ex_ref)
    empty = torch.zeros((0,) + one.shape[1:], dtype=torch.float64, device="cuda")
    g.apply_exchange(empty, [], w.kernel, w.omega)
    assert g.exchange_energy() == 0.0
    g.close()


def test_exchange_bitwise_deterministic(torch_cuda):
    torch = torch_cuda
    kx = _kx()
    w, psi, occ = make_workload("dirichlet32_coulomb")
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    p = torch.from_numpy(psi).cuda()
    a = g.apply_exchange(p, occ, w.kernel, w.omega).clone()
    ea = g.exchange_energy()
    b = g.apply_exchange(p, occ, w.kernel, w.omega)
    eb = g.exchange_energy()
    torch.cuda.synchronize()
    assert torch.equal(a, b) and ea == eb
    g.close()


# orbitals whose Vx psi every full-size test compares with the oracle
VX_ORBITALS = (0, 40, 77, 127)
_VX_REF = {}


def _vx_ref_96(psi, occ, w, j):
    """Oracle (Vx psi)_j of the 96^3 workload, computed once per session."""
    if j not in _VX_REF:
        grid = orc.make_grid(w.n, w.h, w.order, w.bc)
        _VX_REF[j] = orc.vx_orbital(psi, occ, j, grid, w.kernel, w.omega)
    return _VX_REF[j]


@pytest.mark.slow
def test_exchange_production_size_sampled(torch_cuda):
    """128 orbitals on 96^3 periodic, erfc: E_x over all 8256 pairs and a
    sample of pair energies against stored oracle values, and Vx psi of two
    orbitals against the oracle computed here."""
    torch = torch_cuda
    name = "periodic96_erfc"
    with open(GOLDEN) as fh:
        gold = json.load(fh)[name]
    kx = _kx()
    w, psi, occ = make_workload(name)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega)
    ex = g.exchange_energy()
    pe = g.pair_energies(gold["pairs"])
    print(f"E_x gpu={ex!r} oracle={gold['E_x']!r}", flush=True)
    assert abs(ex - gold["E_x"]) <= TOL64 * abs(gold["E_x"])
    for e, r in zip(pe, gold["pair_energies"]):
        assert abs(e - r) <= TOL64 * abs(r) + 1e-15 * abs(gold["E_x"])
    for j in VX_ORBITALS:
        got = vx[j].cpu().numpy()
        assert _rel(got, _vx_ref_96(psi, occ, w, j)) <= TOL64, j
    g.close()


@pytest.mark.slow
@pytest.mark.parametrize("prec", REDUCED + ["mixed"])
def test_exchange_production_size_reduced_precision(torch_cuda, prec):
    """The 128-orbital 96^3 erfc workload in reduced precision: E_x and the
    sampled pair energies against the stored oracle values, Vx psi of one
    orbital against the oracle.  Prints |dE_x| in Hartree."""
    torch = torch_cuda
    name = "periodic96_erfc"
    with open(GOLDEN) as fh:
        gold = json.load(fh)[name]
    kx = _kx()
    w, psi, occ = make_workload(name)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega, prec=prec)
    ex = g.exchange_energy()
    pe = g.pair_energies(gold["pairs"])
    print(f"{prec} E_x gpu={ex!r} oracle={gold['E_x']!r} |dE|={abs(ex - gold['E_x']):.3e} Ha", flush=True)
    tol_e = TOL64 if prec == "mixed" else TOL32_ENERGY
    assert abs(ex - gold["E_x"]) <= tol_e * abs(gold["E_x"])
    emax = max(abs(r) for r in gold["pair_energies"])
    worst = max(abs(e - r) / abs(r) for e, r in zip(pe, gold["pair_energies"]))
    print(f"{prec} worst sampled pair-energy rel err {worst:.2e}", flush=True)
    for e, r in zip(pe, gold["pair_energies"]):
        assert abs(e - r) <= tol_e * abs(r) + 0.1 * tol_e * emax
    for j in VX_ORBITALS:
        assert _rel(vx[j].cpu().numpy(), _vx_ref_96(psi, occ, w, j)) <= TOL32_FIELD, j
    g.close()


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp64", "mixed"] + REDUCED)
def test_exchange_production_size_tuned(torch_cuda, prec):
    """The 128-orbital 96^3 erfc workload with the launch shapes the
    benchmark times (autotuned first, as it does): E_x and the sampled pair
    energies against the stored oracle values, Vx psi of one orbital against
    the oracle."""
    torch = torch_cuda
    name = "periodic96_erfc"
    with open(GOLDEN) as fh:
        gold = json.load(fh)[name]
    kx = _kx()
    w, psi, occ = make_workload(name)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    g.autotune(prec=prec, dtype="f64")
    print(f"tuned {prec} plan {g.plan(prec)}", flush=True)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega, prec=prec)
    ex = g.exchange_energy()
    pe = g.pair_energies(gold["pairs"])
    print(f"tuned {prec} E_x gpu={ex!r} oracle={gold['E_x']!r}", flush=True)
    if prec in ("fp64", "mixed"):
        assert abs(ex - gold["E_x"]) <= TOL64 * abs(gold["E_x"])
        for e, r in zip(pe, gold["pair_energies"]):
            assert abs(e - r) <= TOL64 * abs(r) + 1e-15 * abs(gold["E_x"])
    else:
        assert abs(ex - gold["E_x"]) <= TOL32_ENERGY * abs(gold["E_x"])
        emax = max(abs(r) for r in gold["pair_energies"])
        for e, r in zip(pe, gold["pair_energies"]):
            assert abs(e - r) <= TOL32_ENERGY * abs(r) + 0.1 * TOL32_ENERGY * emax
    tol_f = TOL64 if prec == "fp64" else TOL32_FIELD
    for j in VX_ORBITALS:
        assert _rel(vx[j].cpu().numpy(), _vx_ref_96(psi, occ, w, j)) <= tol_f, j
    g.close()


# ------------------------------------------------------------------ error paths
def test_error_statuses_on_device(torch_cuda):
    torch = torch_cuda
    kx = _kx()
    n = (16, 12, 8)
    g = kx.Grid(n, (0.3,) * 3, 12, ("periodic",) * 3)
    rho = torch.zeros((1, 8, 12, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(kx.KxError) as e:
        g.apply_fL(rho, "coulomb")
    assert e.value.status == 3
    with pytest.raises(kx.KxError) as e:
        g.apply_fL(rho, "erfc", 0.0)
    assert e.value.status == 1
    with pytest.raises(kx.KxError) as e:
        g.exchange_energy()
    assert e.value.status == 6
    L = kx.lib()
    assert L.kx_apply_fL(g._h, 1, 0.1, 0, 0, None, None, 0) == 0  # empty batch is a no-op
    g.close()


# ------------------------------------------------------------------ reduced precision


@pytest.mark.parametrize("prec", REDUCED + ["mixed"])
@pytest.mark.parametrize("n,h,order,bc,kernel,omega", FL_CASES)
def test_apply_fL_reduced_precision(torch_cuda, n, h, order, bc, kernel, omega, prec):
    torch = torch_cuda
    kx = _kx()
    print(f"apply_fL {prec} n={n} bc={bc} kernel={kernel}", flush=True)
    rho = random_fields(n, 2, seed=sum(n) + 1)
    g = kx.Grid(n, h, order, bc)
    phi = g.apply_fL(torch.from_numpy(rho).cuda(), kernel, omega, prec=prec).cpu().numpy()
    g.close()
    ref = orc.apply_fL(rho, orc.make_grid(n, h, order, bc), kernel, omega)
    for b in range(2):
        assert _rel(phi[b], ref[b]) <= TOL32_FIELD


@pytest.mark.parametrize("prec", REDUCED)
@pytest.mark.parametrize("name", ["mixed40x36x44_erfc", "dirichlet32_coulomb", "dirichlet20x27x34_coulomb"])
def test_exchange_reduced_precision(torch_cuda, name, prec):
    torch = torch_cuda
    kx = _kx()
    print(f"exchange {prec} {name}", flush=True)
    w, psi, occ = make_workload(name)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega, prec=prec)
    ex = g.exchange_energy()
    vx = vx.cpu().numpy()
    g.close()
    vx_ref, ex_ref = orc.exchange(psi, occ, orc.make_grid(w.n, w.h, w.order, w.bc), w.kernel, w.omega)
    print(f"{prec} {name}: dE/E={abs(ex - ex_ref) / abs(ex_ref):.2e}", flush=True)
    assert abs(ex - ex_ref) <= TOL32_ENERGY * abs(ex_ref)
    for j in range(w.norb):
        assert _rel(vx[j], vx_ref[j]) <= TOL32_FIELD, j


@pytest.mark.parametrize("name", ["mixed40x36x44_erfc", "dirichlet32_coulomb", "dirichlet20x27x34_coulomb"])
def test_exchange_mixed_precision(torch_cuda, name):
    """Energies (total and per pair) at the FP64 tolerance, Vx psi at the FP32
    tolerance; non-uniform occupations."""
    torch = torch_cuda
    kx = _kx()
    print(f"exchange mixed {name}", flush=True)
    w, psi, occ = make_workload(name)
    occ = occ * np.linspace(1.0, 0.25, w.norb)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi).cuda(), occ, w.kernel, w.omega, prec="mixed")
    ex = g.exchange_energy()
    pairs = [(i, j) for i in range(w.norb) for j in range(i, w.norb)]
    pe = g.pair_energies(pairs)
    vx = vx.cpu().numpy()
    g.close()
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_ref, ex_ref, pe_ref = orc.exchange(psi, occ, grid, w.kernel, w.omega, pair_energies=True)
    print(f"mixed {name}: dE/E={abs(ex - ex_ref) / abs(ex_ref):.2e}", flush=True)
    assert abs(ex - ex_ref) <= TOL64 * abs(ex_ref)
    for p, e in zip(pairs, pe):
        assert abs(e - pe_ref[p]) <= TOL64 * abs(pe_ref[p]) + 1e-14 * abs(ex_ref), p
    for j in range(w.norb):
        assert _rel(vx[j], vx_ref[j]) <= TOL32_FIELD, j


# Grids far from cubic: x much longer than y (forward staging beyond the
# register budget) and y much longer than x (long staged rows in the inverse
# pass); and axes with four and five 16-row tiles per parity (n_k up to 160).
# Every precision accepts every shape.
ANISO = [((70, 8, 12), ("dirichlet",) * 3), ((10, 70, 9), ("dirichlet",) * 3),
         ((9, 66, 20), ("periodic", "periodic", "dirichlet")),
         ((150, 36, 40), ("periodic", "dirichlet", "periodic")),
         ((40, 130, 36), ("dirichlet", "periodic", "dirichlet")),
         ((36, 40, 150), ("periodic", "periodic", "dirichlet")),
         ((112, 100, 72), ("dirichlet",) * 3)]


@pytest.mark.parametrize("n,bc", ANISO)
@pytest.mark.parametrize("prec", ["fp64"] + REDUCED)
def test_apply_fL_anisotropic_grids(torch_cuda, n, bc, prec):
    torch = torch_cuda
    kx = _kx()
    print(f"apply_fL {prec} anisotropic n={n}", flush=True)
    h = (0.3, 0.3, 0.3)
    rho = random_fields(n, 2, seed=sum(n) + 7)
    g = kx.Grid(n, h, 12, bc)
    ref = orc.apply_fL(rho, orc.make_grid(n, h, 12, bc), "coulomb", 0.0)
    try:
        phi = g.apply_fL(torch.from_numpy(rho).cuda(), "coulomb", 0.0, prec=prec).cpu().numpy()
    finally:
        g.close()
    tol = TOL64 if prec == "fp64" else TOL32_FIELD
    for b in range(2):
        assert _rel(phi[b], ref[b]) <= tol


def test_exchange_f32_storage_fp64_arithmetic(torch_cuda):
    """Orbitals stored as float32 (promoted exactly to FP64 by the oracle),
    FP64 mode products; Vx psi is rounded to float32 on output."""
    torch = torch_cuda
    kx = _kx()
    w, psi, occ = make_workload("mixed40x36x44_erfc")
    psi32 = psi.astype(np.float32)
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    vx = g.apply_exchange(torch.from_numpy(psi32).cuda(), occ, w.kernel, w.omega, prec="fp64")
    ex = g.exchange_energy()
    assert vx.dtype == torch.float32
    vx = vx.cpu().numpy().astype(np.float64)
    g.close()
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    vx_ref, ex_ref = orc.exchange(psi32.astype(np.float64), occ, grid, w.kernel, w.omega)
    assert abs(ex - ex_ref) <= TOL64 * abs(ex_ref)
    for j in range(w.norb):
        assert _rel(vx[j], vx_ref[j]) <= 1e-6, j


def test_unknown_precision_reports_status(torch_cuda):
    torch = torch_cuda
    kx = _kx()
    g = kx.Grid((16, 16, 16), (0.3,) * 3, 12, ("dirichlet",) * 3)
    rho = torch.zeros((1, 16, 16, 16), dtype=torch.float64, device="cuda")
    phi = torch.empty_like(rho)
    L = kx.lib()
    for prec in (-1, 5, 99):
        assert L.kx_apply_fL(g._h, 0, 0.0, 1, 0, rho.data_ptr(), phi.data_ptr(), prec) == 1
    g.close()

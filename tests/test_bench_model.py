"""The benchmark's flop and byte model and its roofline arithmetic, checked on
the CPU against direct counts (no GPU, no library calls)."""
import itertools

import pytest

import bench
from synth import WORKLOADS
from synth.orbitals import Workload


def _toy(norb=3, n=(6, 5, 7), storage="f64"):
    return Workload("toy", n, (0.5,) * 3, 4, ("periodic",) * 3, "erfc", 0.2, norb, 2.0, 1, 8, True,
                    storage)


@pytest.mark.parametrize("n", [1, 2, 7, 48, 96, 144])
def test_mode_flops_counts_folded_products(n):
    # brute force: for every vector along the axis, a ceil(n/2)-square and a
    # floor(n/2)-square product, one multiply and one add per element
    N = n * 10
    me, mo = (n + 1) // 2, n // 2
    direct = sum(2 * (me * me + mo * mo) for _ in range(N // n))
    assert bench.mode_flops(N, n) == direct
    if n % 2 == 0:  # half of the unfolded 2 n flops per point
        assert bench.mode_flops(N, n) == N * n


def test_phase_flops_at_96_cubed():
    w = WORKLOADS["periodic96_erfc"]
    pf = bench.phase_flops(w)
    assert pf["forward"] == pf["inverse"] == 2 * w.N * 96
    assert pf["pencil"] == 2 * w.N * 96
    # folding halves the unfolded count 4 N (n1 + n2 + n3)
    assert sum(pf.values()) * 2 == w.flops_per_pair()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3", "mixed"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_phase_bytes_sum_over_pairs(prec, storage):
    # the per-step byte model against a loop over the pairs (i <= j)
    w = _toy(norb=4, storage=storage)
    s_store = 8 if storage == "f64" else 4
    s = s_store if prec == "fp64" else 4
    t = {"fp64": 8, "fp32": 4, "bf16x3": 4, "fp16x3": 4, "mixed": 8}[prec]
    tot = {"forward": 0, "pencil": 0, "inverse": 0, "accum": 0}
    for i, j in itertools.combinations_with_replacement(range(w.norb), 2):
        orbs = 1 if i == j else 2
        # the toy grid is one tile per parity block: every precision but
        # FP16x3 (and FP64 on FP32 storage) runs in two stages, the inverse
        # pass writing phi_ij (FP64 for fp64, else FP32) that the
        # accumulation reads once
        two = prec != "fp16x3" and not (prec == "fp64" and storage == "f32")
        pb = 8 if prec == "fp64" else 4
        if prec == "mixed":
            tot["forward"] += (orbs * s_store + 8) * w.N
            tot["pencil"] += (8 + 4) * w.N
            tot["inverse"] += (4 + pb) * w.N
            tot["accum"] += pb * w.N
        elif two:
            tot["forward"] += (orbs * s + t) * w.N
            tot["pencil"] += 2 * t * w.N
            tot["inverse"] += (t + pb) * w.N
            tot["accum"] += pb * w.N
        else:
            tot["forward"] += (orbs * s + t) * w.N
            tot["pencil"] += 2 * t * w.N
            tot["inverse"] += (t + 3 * orbs * s) * w.N
    if prec != "fp16x3" and not (prec == "fp64" and storage == "f32"):
        # plus psi read and Vx psi read-modify-written once per orbital and
        # tile: a tile of 8 x 8 orbitals, here 4 orbitals, is one diagonal tile
        tot["accum"] += w.norb * 3 * s * w.N
    assert bench.phase_bytes(w, prec) == tot


def test_xtiles_cover_every_pair_once():
    for norb in (1, 7, 8, 9, 16, 33, 128):
        tiles = bench.xtiles(norb)
        assert sum(nb for nb, _ in tiles) == norb * (norb + 1) // 2
        nbk = (norb + 7) // 8
        assert len(tiles) == nbk * (nbk + 1) // 2


def test_roofline_picks_the_bound_and_the_dominant_phase():
    w = WORKLOADS["periodic96_erfc"]
    launches = 129
    # forward dominant: 2 ms a launch
    phases = {"forward": {"ms": 2.0 * launches, "launches": launches},
              "pencil": {"ms": 1.0 * launches, "launches": launches},
              "inverse": {"ms": 1.5 * launches, "launches": launches},
              "energy": {"ms": 0.1, "launches": launches}}
    r = bench.roofline(w, "fp64", phases, launches_per_step=launches)
    assert r["kernel"] == "forward" and r["avg_launch_ms"] == pytest.approx(2.0)
    pb = bench.phase_bytes(w, "fp64")["forward"] / launches
    pf = bench.phase_flops(w)["forward"] * w.npairs / launches
    # FP64 forward at 96^3: 24 N bytes against 192 N flops per pair, so the
    # HBM time at 8 TB/s exceeds the MFMA time at 78.6 TF/s
    assert pb / 8e12 > pf / 78.6e12 and r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(pb / 2e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    # a split path is priced against its own peak
    r = bench.roofline(w, "bf16x3", phases, launches_per_step=launches)
    assert r["mfma_peak"] == 2500.0


def test_vx_energy_is_the_exchange_energy_of_the_exact_operator():
    # 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h = E_x for the operator the oracle
    # applies (non-uniform occupations), so the benchmark's second energy
    # measure has the oracle's E_x as its reference
    import numpy as np
    import oracle as orc
    from synth import make_workload
    w, psi, occ = make_workload("dirichlet20x27x34_coulomb")
    occ = occ * np.linspace(1.0, 0.3, w.norb)
    vx, ex = orc.exchange(psi, occ, orc.make_grid(w.n, w.h, w.order, w.bc), w.kernel, w.omega)
    assert abs(bench.vx_energy(psi, vx, occ, w.dV) - ex) <= 1e-12 * abs(ex)
    assert abs(bench.vx_energy(psi, 1.001 * vx, occ, w.dV) - ex) > 1e-4 * abs(ex)

"""Ragged multi-system batches through kx_batch_apply_exchange (one recorded
HIP graph, one branch per system): against the oracle, against the
one-system entry point, and across replays with other work in between."""
import numpy as np
import pytest

import oracle as orc
from synth import Workload, make_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-10

# small systems with different shapes, boundary conditions, kernels and
# orbital counts (the oracle finishes each in seconds)
SMALL = [
    "dirichlet20x27x34_coulomb",
    "mixed40x36x44_erfc",
    Workload("periodic24x20x28_erfc", (24, 20, 28), (0.35, 0.3, 0.33), 12,
             ("periodic",) * 3, "erfc", 0.106, 4, 2.0, 11, 8, True),
    Workload("slab30x26x18_coulomb", (30, 26, 18), (0.3, 0.3, 0.3), 12,
             ("periodic", "periodic", "dirichlet"), "coulomb", 0.0, 3, 2.0, 12, 12, False),
]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def systems():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_16998_amd import kx
    out = []
    for spec in SMALL:
        w, psi, occ = make_workload(spec)
        occ = occ * np.linspace(1.0, 0.5, w.norb)  # distinct occupations
        g = kx.Grid(w.n, w.h, w.order, w.bc)
        out.append((w, psi, occ, g, torch.from_numpy(psi).cuda()))
    yield out
    for s in out:
        s[3].close()


def _batch(systems, prec, outs=None):
    from paper_2406_16998_amd import kx
    return kx.batch_apply_exchange([s[3] for s in systems], [s[4] for s in systems],
                                   [s[2] for s in systems], [s[0].kernel for s in systems],
                                   [s[0].omega for s in systems], prec=prec, outs=outs)


def test_batch_matches_oracle_fp64(systems):
    print("batch fp64 vs oracle", flush=True)
    vxs, exs = _batch(systems, "fp64")
    for (w, psi, occ, g, _), vx, ex in zip(systems, vxs, exs):
        grid = orc.make_grid(w.n, w.h, w.order, w.bc)
        vx_ref, ex_ref = orc.exchange(psi, occ, grid, w.kernel, w.omega)
        assert abs(ex - ex_ref) <= TOL64 * abs(ex_ref), w.name
        assert abs(g.exchange_energy() - ex) == 0.0
        vx = vx.cpu().numpy()
        for j in range(w.norb):
            assert _rel(vx[j], vx_ref[j]) <= TOL64, (w.name, j)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp16x3", "mixed"])
def test_batch_replays_match_single_system_calls(systems, prec):
    """Three replays of the recorded graph, each after eager single-system work
    that reuses the same handles, must equal the eager results bitwise."""
    import torch
    print(f"batch replays {prec}", flush=True)
    eager = []
    for w, psi, occ, g, psi_d in systems:
        vx = g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=prec)
        eager.append((vx.clone(), g.exchange_energy()))
    outs = [torch.empty_like(s[4]) for s in systems]
    for rep in range(3):
        for k, s in enumerate(systems):  # other work on the same handles in between
            if (rep + k) % 2 == 0:
                s[3].apply_exchange(s[4], s[2], s[0].kernel, s[0].omega,
                                    prec="fp32" if prec == "fp64" else "fp64")
        torch.cuda.synchronize()
        for o in outs:
            o.fill_(float("nan"))
        vxs, exs = _batch(systems, prec, outs=outs)
        for (vx_e, ex_e), vx, ex in zip(eager, vxs, exs):
            assert ex == ex_e, rep
            assert torch.equal(vx, vx_e), rep


def test_batch_rejects_bad_arguments(systems):
    from paper_2406_16998_amd import kx
    s = systems[0]
    with pytest.raises(kx.KxError) as e:
        kx.batch_apply_exchange([s[3], s[3]], [s[4], s[4]], [s[2], s[2]], [s[0].kernel] * 2,
                                [s[0].omega] * 2)
    assert e.value.status == 1
    L = kx.lib()
    assert L.kx_batch_apply_exchange(0, None, None, None, None, 0, None, None, None, 0, None) == 1


# ------------------------------------------------------------------ full size
# The six-system ragged workload (48^3 Dirichlet .. 112^3 periodic, 16 .. 128
# orbitals), with the autotuned launch shapes the benchmark times, against the
# oracle: sampled pair energies (diagonals included) on every system, E_x of
# the two smallest systems over all their pairs, Vx psi of one orbital on the
# three smallest systems.
TOL32_FIELD = 1e-5
TOL32_ENERGY = 1e-6
VX_SYSTEMS = 3


@pytest.fixture(scope="module")
def ragged():
    import torch
    from paper_2406_16998_amd import kx
    from synth import RAGGED_BATCH
    out = []
    for k, name in enumerate(RAGGED_BATCH):
        print(f"generating {name}", flush=True)
        w, psi, occ = make_workload(name)
        rng = np.random.default_rng(100 + k)
        n = w.norb
        sample = [(0, 0), (n // 2, n // 2), (n - 1, n - 1), (0, n - 1)]
        while len(sample) < 10:
            p = tuple(int(v) for v in sorted(rng.choice(n, 2, replace=False)))
            if p not in sample:
                sample.append(p)
        grid = orc.make_grid(w.n, w.h, w.order, w.bc)
        F = orc.kernel_values(grid.lam_sum(), w.kernel, w.omega)
        ref = np.array([orc.pair_energy(psi[i], psi[j], grid, w.kernel, w.omega, F)
                        for i, j in sample])
        vx_ref = ex_ref = None
        if k < VX_SYSTEMS:
            vx_ref = orc.vx_orbital(psi, occ, n // 3, grid, w.kernel, w.omega)
        if k < 2:
            ex_ref = orc.exchange(psi, occ, grid, w.kernel, w.omega)[1]
        print(f"oracle {name} done", flush=True)
        out.append(dict(w=w, psi=psi, occ=occ, sample=sample, ref=ref, vx_ref=vx_ref,
                        ex_ref=ex_ref, g=kx.Grid(w.n, w.h, w.order, w.bc),
                        psi_d=torch.from_numpy(psi).cuda()))
    yield out
    for s in out:
        s["g"].close()


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp64", "mixed", "bf16x3"])
def test_ragged_six_systems_against_oracle(ragged, prec):
    from paper_2406_16998_amd import kx
    for s in ragged:
        s["g"].autotune(prec=prec, dtype="f64")
    vxs, exs = kx.batch_apply_exchange([s["g"] for s in ragged], [s["psi_d"] for s in ragged],
                                       [s["occ"] for s in ragged], [s["w"].kernel for s in ragged],
                                       [s["w"].omega for s in ragged], prec=prec)
    energy64 = prec in ("fp64", "mixed")
    for s, vx, ex in zip(ragged, vxs, exs):
        w, g = s["w"], s["g"]
        pe = g.pair_energies(s["sample"])
        ref = s["ref"]
        emax = float(np.max(np.abs(ref)))
        worst = max(abs(e - r) / abs(r) for e, r in zip(pe, ref))
        print(f"{prec} {w.name}: E_x={ex!r} worst sampled pair rel err {worst:.2e}", flush=True)
        for p, e, r in zip(s["sample"], pe, ref):
            if energy64:
                assert abs(e - r) <= TOL64 * abs(r) + 1e-15 * emax, (w.name, p)
            else:
                assert abs(e - r) <= TOL32_ENERGY * abs(r) + 0.1 * TOL32_ENERGY * emax, (w.name, p)
        if s["ex_ref"] is not None:
            tol = TOL64 if energy64 else TOL32_ENERGY
            assert abs(ex - s["ex_ref"]) <= tol * abs(s["ex_ref"]), w.name
        if s["vx_ref"] is not None:
            got = vx[w.norb // 3].cpu().numpy()
            tol = TOL64 if prec == "fp64" else TOL32_FIELD
            assert _rel(got, s["vx_ref"]) <= tol, w.name

"""kx_apply_exchange and kx_apply_fL recorded into a caller's HIP graph.

Both calls only enqueue kernels once the workspace is reserved (the f table,
the pair schedule and the occupations are written by kernels, the
occupations travelling as kernel arguments), so a graph recorded from them
replays the same work.  Each replay follows eager work on the same handle
with another kernel, other occupations and another precision, and must equal
the eager result bitwise."""
import numpy as np
import pytest

from synth import make_workload, random_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_16998_amd import kx
    kx.lib()
    return torch, kx


@pytest.mark.parametrize("prec", ["fp64", "mixed", "bf16x3", "fp16x3", "fp32"])
def test_exchange_graph_replays_equal_eager(env, prec):
    torch, kx = env
    print(f"graph exchange {prec}", flush=True)
    w, psi, occ = make_workload("mixed40x36x44_erfc")
    occ = occ * np.linspace(1.0, 0.5, w.norb)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = kx.Grid(w.n, w.h, w.order, w.bc, stream=s)
        psi_d = torch.from_numpy(psi).cuda()
        g.reserve(w.norb, prec, "f64")
        g.reserve(w.norb, "fp64", "f64")
        eager = g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=prec).clone()
        ex_eager = g.exchange_energy()
        out = torch.empty_like(psi_d)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=prec, out=out, reserve=False)
    for rep in range(3):
        with torch.cuda.stream(s):
            # other kernel, occupations and precision on the same handle
            other = g.apply_exchange(psi_d, occ[::-1].copy(), "coulomb", 0.0, prec="fp64")
            out.fill_(float("nan"))
        s.synchronize()
        assert not torch.equal(other, eager)
        graph.replay()
        s.synchronize()
        assert torch.equal(out, eager), rep
        assert g.exchange_energy() == ex_eager, rep
    del graph
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "mixed"])
def test_apply_fL_graph_replays_equal_eager(env, prec):
    torch, kx = env
    print(f"graph apply_fL {prec}", flush=True)
    n, h, bc = (24, 20, 28), (0.3,) * 3, ("periodic", "dirichlet", "dirichlet")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = kx.Grid(n, h, 12, bc, stream=s)
        rho = torch.from_numpy(random_fields(n, 5, seed=5)).cuda()
        g.reserve(0, prec, "f64")
        eager = g.apply_fL(rho, "erfc", 0.2, prec=prec).clone()
        out = torch.empty_like(rho)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.apply_fL(rho, "erfc", 0.2, prec=prec, out=out, reserve=False)
    for rep in range(3):
        with torch.cuda.stream(s):
            g.apply_fL(rho, "coulomb", 0.0, prec="fp64")
            out.fill_(float("nan"))
        s.synchronize()
        graph.replay()
        s.synchronize()
        assert torch.equal(out, eager), rep
    del graph
    g.close()


def test_apply_without_reserve_reports_state(env):
    torch, kx = env
    w, psi, occ = make_workload("dirichlet20x27x34_coulomb")
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    psi_d = torch.from_numpy(psi).cuda()
    with pytest.raises(kx.KxError) as e:
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, reserve=False)
    assert e.value.status == 6
    with pytest.raises(kx.KxError) as e:
        g.apply_fL(psi_d, w.kernel, w.omega, reserve=False)
    assert e.value.status == 6
    # reserved for fewer orbitals, or another precision's buffers missing
    g.reserve(3, "fp64", "f64")
    with pytest.raises(kx.KxError) as e:
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, reserve=False)
    assert e.value.status == 6
    g.reserve(w.norb, "fp64", "f64")
    with pytest.raises(kx.KxError) as e:
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec="mixed", reserve=False)
    assert e.value.status == 6
    vx = g.apply_exchange(psi_d, occ, w.kernel, w.omega, reserve=False)
    torch.cuda.synchronize()
    assert torch.isfinite(vx).all()
    g.close()


def test_bloch_and_isolated_exchange_graph_replays_equal_eager(env):
    # the k-point exchange and the isolated-system exchange also enqueue
    # kernels only once reserved (k-points, weights and occupations travel as
    # kernel arguments)
    torch, kx = env
    from synth import bloch_orbitals
    from synth.orbitals import gaussian_orbitals, orthonormalise_cgs2
    print("graph bloch + isolated exchange", flush=True)
    n, h, P3 = (12, 10, 9), (0.5, 0.5, 0.5), ("periodic",) * 3
    kpts = [(0.0, 0.0, 0.0), (0.5, 0.25, 0.0)]
    psi = bloch_orbitals(n, h, P3, kpts, 3, seed=12, n_centres=6)
    wk, occ = [0.5, 0.5], [[1.0, 0.8, 0.6], [0.9, 0.7, 0.5]]
    D3 = ("dirichlet",) * 3
    nd, hd = (16, 14, 18), (0.45, 0.45, 0.45)
    psi_r = orthonormalise_cgs2(gaussian_orbitals(nd, hd, D3, 4, 3, 8, True), hd[0] * hd[1] * hd[2])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = kx.Grid(n, h, 6, P3, stream=s)
        gd = kx.Grid(nd, hd, 8, D3, stream=s)
        p = torch.from_numpy(psi).cuda()
        pr = torch.from_numpy(psi_r).cuda()
        g.reserve_bloch(2, 3)
        gd.reserve(4, "fp64", "f64")
        eager = g.apply_exchange_bloch(p, kpts, wk, occ, "erfc", 0.3).clone()
        ex_eager = g.exchange_energy()
        eager_d = gd.apply_exchange_multipole(pr, [2.0, 1.5, 1.0, 0.5], lmax=4).clone()
        exd_eager = gd.exchange_energy()
        out = torch.empty_like(p)
        out_d = torch.empty_like(pr)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.apply_exchange_bloch(p, kpts, wk, occ, "erfc", 0.3, out=out, reserve=False)
        gd.apply_exchange_multipole(pr, [2.0, 1.5, 1.0, 0.5], lmax=4, out=out_d, reserve=False)
    for rep in range(3):
        with torch.cuda.stream(s):
            g.apply_exchange_bloch(p, kpts, [0.3, 0.7], occ, "erfc", 0.5)
            gd.apply_exchange_multipole(pr, [1.0, 1.0, 1.0, 1.0], lmax=2)
            out.fill_(float("nan"))
            out_d.fill_(float("nan"))
        s.synchronize()
        graph.replay()
        s.synchronize()
        assert torch.equal(out, eager), rep
        assert torch.equal(out_d, eager_d), rep
        assert g.exchange_energy() == ex_eager and gd.exchange_energy() == exd_eager, rep
    del graph
    g.close()
    gd.close()

"""Opt-in finite checks (KX_CHECK_FINITE), KX_LOG lines and KX_ROCTX ranges.

A NaN or infinity in an input is refused before any work (outputs left as
they were); an overflow inside the solve is reported after it; checked and
unchecked calls give the same bits; KX_LOG=1 prints the set-up and
application lines; KX_ROCTX=1 runs with the ranges on."""
import os
import subprocess
import sys

import numpy as np
import pytest

from synth import bloch_orbitals, make_workload

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_16998_amd import kx as _kx
    _kx.lib()
    return _kx


def test_finite_checks(kx):
    import torch
    w, psi, occ = make_workload("dirichlet20x27x34_coulomb")
    with kx.Grid(w.n, w.h, w.order, w.bc) as g:
        p = torch.from_numpy(psi).cuda()
        ref = g.apply_exchange(p, occ, "coulomb")
        torch.cuda.synchronize()
        ref_e = g.exchange_energy()
        g.set_checks(True)
        got = g.apply_exchange(p, occ, "coulomb")
        torch.cuda.synchronize()
        assert torch.equal(got, ref) and g.exchange_energy() == ref_e
        bad = p.clone()
        bad[1, 3, 4, 5] = float("nan")
        out = torch.full_like(p, 7.0)
        with pytest.raises(kx.KxError) as e:
            g.apply_exchange(bad, occ, "coulomb", out=out)
        assert e.value.status == 7
        torch.cuda.synchronize()
        assert bool(torch.all(out == 7.0))  # nothing written
        bad[1, 3, 4, 5] = float("inf")
        rho = bad[:2].contiguous()
        with pytest.raises(kx.KxError) as e:
            g.apply_fL(rho, "coulomb")
        assert e.value.status == 7
        # finite input, overflow inside the solve: reported after the work
        huge = torch.full_like(p[:1], 1e307)
        with pytest.raises(kx.KxError) as e:
            g.apply_fL(huge, "coulomb")
        assert e.value.status == 7
        g.set_checks(False)
        out = g.apply_fL(huge, "coulomb")  # unchecked: runs, returns the overflowed values
        torch.cuda.synchronize()
        assert not bool(torch.all(torch.isfinite(out)))


def test_finite_checks_bloch(kx):
    import torch
    n, h = (8, 7, 6), (0.5, 0.5, 0.5)
    P3 = ("periodic",) * 3
    psi = torch.from_numpy(bloch_orbitals(n, h, P3, [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)], 2, 5, 4)).cuda()
    with kx.Grid(n, h, 4, P3) as g:
        g.set_checks(True)
        g.apply_exchange_bloch(psi, [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)], [0.5, 0.5], [[1, 1], [1, 1]],
                               "erfc", 0.3)
        bad = psi.clone()
        bad[1, 0, 2, 2, 2] = complex(float("nan"), 0.0)
        with pytest.raises(kx.KxError) as e:
            g.apply_exchange_bloch(bad, [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)], [0.5, 0.5],
                                   [[1, 1], [1, 1]], "erfc", 0.3)
        assert e.value.status == 7
        with pytest.raises(kx.KxError) as e:
            g.apply_fL_bloch(bad[1], (0.3, 0.0, 0.0), "erfc", 0.3)
        assert e.value.status == 7


_CHILD = """
import sys, torch
sys.path.insert(0, {root!r})
from paper_2406_16998_amd import kx
g = kx.Grid((12, 10, 8), (0.4, 0.4, 0.4), 4, ('dirichlet',) * 3)
rho = torch.ones((2, 8, 10, 12), dtype=torch.float64, device='cuda')
phi = g.apply_fL(rho, 'coulomb')
torch.cuda.synchronize()
print('phi', float(phi.abs().max()))
g.close()
"""


@pytest.mark.parametrize("env", [{"KX_LOG": "1"}, {"KX_ROCTX": "1"}, {"KX_LOG": "0"}])
def test_log_and_ranges(kx, env):
    e = dict(os.environ)
    e.update(env)
    print(f"child with {env}", flush=True)
    r = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], env=e, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "phi" in r.stdout
    if env.get("KX_LOG") == "1":
        assert "[kx] setup n=(12, 10, 8)" in r.stderr
        assert "[kx] apply_fL batch=2 prec=fp64" in r.stderr
        assert "[kx] workspace:" in r.stderr
    else:
        assert "[kx]" not in r.stderr

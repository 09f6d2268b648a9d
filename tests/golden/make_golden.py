"""Write oracle-derived expected values for the full-size parity tests.

Calls only the oracle and the seeded input generator.  Output:
tests/golden/oracle_energies.json with, per workload, E_x over all pairs and
the pair energies e_ij = (rho_ij, phi_ij)_h of a seeded sample of pairs.

    python tests/golden/make_golden.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
from synth import WORKLOADS, make_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_energies.json")


def sample_pairs(norb, k, seed):
    rng = np.random.default_rng(seed)
    pairs = {(0, 0), (0, norb - 1), (norb - 1, norb - 1)}
    while len(pairs) < min(k, norb * (norb + 1) // 2):
        i, j = sorted(int(v) for v in rng.integers(0, norb, 2))
        pairs.add((i, j))
    return sorted(pairs)


def golden_for(name):
    w, psi, occ = make_workload(name)
    psi = psi.astype(np.float64)
    g = orc.make_grid(w.n, w.h, w.order, w.bc)
    F = orc.kernel_values(g.lam_sum(), w.kernel, w.omega)
    t0 = time.time()
    ex = 0.0
    es = {}
    for i in range(w.norb):
        for j in range(i, w.norb):
            e = orc.pair_energy(psi[i], psi[j], g, w.kernel, w.omega, F)
            es[(i, j)] = e
            ex -= 0.25 * occ[i] * occ[j] * e * (1.0 if i == j else 2.0)
        print(f"{name}: row {i} done, {time.time() - t0:.0f} s", flush=True)
    sample = sample_pairs(w.norb, 48, 123)
    return {
        "workload": name,
        "E_x": ex,
        "pairs": [[i, j] for i, j in sample],
        "pair_energies": [es[p] for p in sample],
        "oracle_seconds": time.time() - t0,
    }


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names:
        if name not in WORKLOADS:
            raise SystemExit(f"unknown workload {name}")
        data[name] = golden_for(name)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or ["dirichlet32_coulomb", "periodic96_erfc"])

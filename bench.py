"""Benchmark: all-pairs exact-exchange application on one MI355X.

One step = one kx_apply_exchange over every symmetric orbital pair of the
workload (pair products, forward transforms, f(Lambda) scaling, pair
energies, inverse transforms, Vx psi accumulation, E_x), inputs resident in
HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec fp64] [--workload periodic96_erfc]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-solves/s + Vxψ time, 128 orb 96³ HSE: FP64 vs split-BF16 MFMA"
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}
HBM_PEAK_GBS = 8000.0


def mode_flops(N, n):
    """Flops of one folded mode product along an axis of length n on a field of
    N points: N/n vectors, each through two half-size products (even block
    ceil(n/2)^2, odd block floor(n/2)^2), 2 flops per multiply-add."""
    me, mo = n - n // 2, n // 2
    return N // n * 2 * (me * me + mo * mo)


def phase_flops(w):
    """Algorithmic flops per item (pair) of each transform phase."""
    n1, n2, n3 = w.n
    N = w.N
    fw = mode_flops(N, n1) + mode_flops(N, n2)
    return {"forward": fw, "pencil": 2 * mode_flops(N, n3), "inverse": fw}


def cpu_baseline(w, psi, occ, target_s=15.0):
    """Time the FP64 oracle as it stands on a bounded sample of the same
    workload: exchange over the first k orbitals (k(k+1)/2 pairs)."""
    import numpy as np
    import oracle as orc
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    grid = orc.make_grid(w.n, w.h, w.order, w.bc)
    # calibrate with 2 orbitals (3 pairs), then size the sample
    t0 = time.perf_counter()
    orc.exchange(np.asarray(psi[:2], dtype=np.float64), occ[:2], grid, w.kernel, w.omega)
    per_pair = (time.perf_counter() - t0) / 3
    k = 2
    while k < w.norb and (k + 1) * (k + 2) / 2 * per_pair < target_s:
        k += 1
    pairs = k * (k + 1) // 2
    t0 = time.perf_counter()
    orc.exchange(np.asarray(psi[:k], dtype=np.float64), occ[:k], grid, w.kernel, w.omega)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pair-solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle exchange over the first {k} orbitals ({pairs} of {w.npairs} pairs) "
                      f"of the same workload, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp64", choices=sorted(PEAKS_TFLOPS))
    ap.add_argument("--workload", default="periodic96_erfc")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exchange path has no multi-GPU mode in this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2406_16998_amd import kx
    from synth import make_workload

    torch.cuda.set_device(0)
    w, psi, occ = make_workload(args.workload)
    t_setup = time.perf_counter()
    g = kx.Grid(w.n, w.h, w.order, w.bc)
    setup_s = time.perf_counter() - t_setup
    psi_d = torch.from_numpy(psi).cuda()
    vx = torch.empty_like(psi_d)
    print(f"# workload {w.name}: {w.n} {w.bc} norb={w.norb} pairs={w.npairs} prec={args.prec}",
          file=sys.stderr, flush=True)

    for k in range(args.warmup):
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=args.prec, out=vx)
        g.exchange_energy()
        print(f"# warmup {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    g.profile(True)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=args.prec, out=vx)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(stop)
    ex = g.exchange_energy()
    phases = {}
    for ph in ("forward", "pencil", "inverse", "energy"):
        ms, cnt = g.profile_read(ph)
        phases[ph] = {"ms": ms, "launches": cnt}
    g.profile(False)
    print(f"# timed {args.steps} steps: {ms_total:.1f} ms (wall {wall * 1e3:.1f} ms)",
          file=sys.stderr, flush=True)

    ms_step = ms_total / args.steps
    value = w.npairs * args.steps / (ms_total * 1e-3)
    # dominant kernel: the transform phase with the largest summed time
    pf = phase_flops(w)
    dom = max(pf, key=lambda p: phases[p]["ms"])
    avg_ms = phases[dom]["ms"] / max(phases[dom]["launches"], 1)
    items_per_launch = w.npairs / max(phases[dom]["launches"] / args.steps, 1)
    flops_launch = pf[dom] * items_per_launch
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.prec]
    total_flops = sum(pf.values()) * w.npairs
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x3": "fp16x3"}[args.prec],
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "h": list(w.h), "fd_order": w.order,
                   "bc": list(w.bc), "kernel": w.kernel, "omega": w.omega, "norb": w.norb,
                   "pairs": w.npairs, "prec": args.prec, "storage": w.storage},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_ms": avg_ms, "flops_per_launch": flops_launch},
        "vx_time_ms": ms_step,
        "tflops_whole_step": total_flops / (ms_step * 1e-3) / 1e12,
        "flops_per_pair": sum(pf.values()),
        "unfolded_flops_per_pair": w.flops_per_pair(),
        "phases_ms_per_step": {p: v["ms"] / args.steps for p, v in phases.items()},
        "E_x": ex,
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, psi, occ)
    g.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()

"""Benchmark: all-pairs exact-exchange application on one MI355X.

One step = one kx_apply_exchange over every symmetric orbital pair of the
workload (pair products, forward transforms, f(Lambda) scaling, pair
energies, inverse transforms, Vx psi accumulation, E_x), inputs resident in
HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec fp64] [--workload periodic96_erfc]
    python bench.py --calibrate-copy     # plain 1 GiB device copy, for counter scaling
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-solves/s + Vxψ time, 128 orb 96³ HSE: FP64 vs split-BF16 MFMA"
# the mixed path's MFMA-heavy forward and pencil passes run in FP64
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0, "mixed": 78.6}
HBM_PEAK_GBS = 8000.0


def mode_flops(N, n):
    """Flops of one folded mode product along an axis of length n on a field of
    N points: N/n vectors, each through two half-size products (even block
    ceil(n/2)^2, odd block floor(n/2)^2), 2 flops per multiply-add."""
    me, mo = n - n // 2, n // 2
    return N // n * 2 * (me * me + mo * mo)


def phase_flops(w):
    """Algorithmic flops per item (pair) of each transform phase (the FP64
    exchange's accumulation of Vx psi from stored potentials is VALU work,
    counted as none)."""
    n1, n2, n3 = w.n
    N = w.N
    fw = mode_flops(N, n1) + mode_flops(N, n2)
    return {"forward": fw, "pencil": 2 * mode_flops(N, n3), "inverse": fw, "accum": 0}


XTILE = 8             # orbital tile edge of the FP64 exchange (two-stage)
XTILE_MAX_ORB = 4096  # above it the FP64 exchange keeps the fused inverse pass


def xtiles(norb):
    """(pairs, orbitals) of every tile of the FP64 exchange: rows of block a,
    columns of block b >= a; a diagonal tile holds its i <= j pairs."""
    nbk = (norb + XTILE - 1) // XTILE
    size = [min(XTILE, norb - XTILE * a) for a in range(nbk)]
    out = []
    for a in range(nbk):
        for b in range(a, nbk):
            if a == b:
                out.append((size[a] * (size[a] + 1) // 2, size[a]))
            else:
                out.append((size[a] * size[b], size[a] + size[b]))
    return out


T_BYTES = {"fp64": 8, "fp32": 4, "bf16x3": 4, "fp16x3": 4, "mixed": 8}


def phase_bytes(w, prec):
    """Algorithmic HBM bytes of each phase summed over all pairs of one step
    (N values per field; s bytes per orbital value, t per intermediate value):
      forward  reads psi_i, psi_j, writes T            (2s + t) N
      pencil   reads and writes T                       2t N  (+ the f table once a launch)
      inverse  reads T, psi_i, psi_j, read-modify-writes Vx psi_i, Vx psi_j   (t + 6s) N
    A diagonal pair (i = i) touches one orbital: (s + t), 2t, (t + 3s) N.
    The FP64 exchange on FP64 storage, and the mixed, FP32 and BF16x3 ones
    (up to 4096 orbitals), run in two stages instead: the inverse pass reads T and writes the potential
    phi_ij (FP64 for fp64, else FP32: p bytes), (t + p) N, and per tile of
    pairs the accumulation reads the tile's potentials (p N each) and reads
    psi and read-modify-writes Vx psi of each of its orbitals once (3 s N
    each).
    Reduced precision on FP64 storage runs on FP32 working copies (s = 4).
    The mixed path reads the stored orbitals in its FP64 forward pass, writes
    an FP32 intermediate from the pencil pass (8 + 4 bytes there) and runs
    its inverse pass on the FP32 copies."""
    s_store = 8 if w.storage == "f64" else 4
    s = s_store if prec == "fp64" else 4
    t = T_BYTES[prec]
    off, diag = w.norb * (w.norb - 1) // 2, w.norb
    N = w.N
    two = w.norb <= XTILE_MAX_ORB and (
        (prec == "fp64" and w.storage == "f64") or prec in ("mixed", "fp32", "bf16x3"))
    # two stages: the potentials in FP64 (fp64) or FP32, read back once
    phi_b = 8 if prec == "fp64" else 4
    acc = sum(nb * phi_b + orbs * 3 * s for nb, orbs in xtiles(w.norb)) * N if two else 0
    if prec == "mixed":
        inv = ((off + diag) * (4 + phi_b) if two else off * (4 + 6 * s) + diag * (4 + 3 * s)) * N
        return {"forward": (off * (2 * s_store + 8) + diag * (s_store + 8)) * N,
                "pencil": (off + diag) * 12 * N, "inverse": inv, "accum": acc}
    if two:
        return {"forward": (off * (2 * s + t) + diag * (s + t)) * N,
                "pencil": (off + diag) * 2 * t * N,
                "inverse": (off + diag) * (t + phi_b) * N, "accum": acc}
    return {"forward": (off * (2 * s + t) + diag * (s + t)) * N,
            "pencil": (off + diag) * 2 * t * N,
            "inverse": (off * (t + 6 * s) + diag * (t + 3 * s)) * N, "accum": 0}


# the sources of the exchange's transform kernels and of their launch shapes
KERNEL_SOURCES = ("kx_fold.inc", "kx_epilogue.inc", "kx_fold_d.hip", "kx_fold_f.hip",
                  "kx_split.hip", "kx_energy_plan.hip", "kx_internal.h")


def kernel_sources_digest():
    """Digest of the transform kernels' sources: counter figures recorded for
    other sources no longer describe the kernels."""
    files = sorted(os.path.join(ROOT, "paper_2406_16998_amd", "csrc", f) for f in KERNEL_SOURCES)
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, prec, phase):
    """HBM bytes per launch from the committed counter summary (copy-scaled
    FETCH_SIZE + WRITE_SIZE), or None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest, val = None, None
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) >= 2 and f[0] == "sources_digest":
                digest = f[1]
            if len(f) >= 4 and f[0] == "bytes_per_launch" and f[1] == prec and f[2] == phase:
                val = float(f[3])
    return val if digest == kernel_sources_digest() else None


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, three times: what FETCH_SIZE and
    WRITE_SIZE read for it scales the counters of the exchange kernels."""
    import torch
    n = 128 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": 8 * n, "launches": 3}))


def cpu_baseline(w, psi, occ, target_s=20.0):
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
    # calibrate with 4 orbitals (10 pairs), then size the sample
    t0 = time.perf_counter()
    orc.exchange(np.asarray(psi[:4], dtype=np.float64), occ[:4], grid, w.kernel, w.omega)
    per_pair = (time.perf_counter() - t0) / 10
    k = 2
    while k < w.norb and (k + 1) * (k + 2) / 2 * per_pair < target_s:
        k += 1
    pairs = k * (k + 1) // 2
    t0 = time.perf_counter()
    orc.exchange(np.asarray(psi[:k], dtype=np.float64), occ[:k], grid, w.kernel, w.omega)
    dt = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pairs / dt, "unit": "pair-solves/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": model,
            "sample": f"oracle exchange over the first {k} orbitals ({pairs} of {w.npairs} pairs) "
                      f"of the same workload, {dt:.1f} s"}


# the mixed path forms every energy in FP64: only its potential's back-transform
# and the Vx psi update are split BF16
DTYPE_NAME = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x3": "fp16x3",
              "mixed": "f64-energy+bf16x3-potential"}
# variants whose every mode product runs on split MFMA
SPLIT_PRECS = ("bf16x3", "fp16x3")
TARGET_DEX_HA = 1e-8  # exchange-energy accuracy the speedup is quoted at


def roofline(w, prec, phases, launches_per_step):
    """Roofline of the dominant transform phase (largest summed time): bound
    is whichever of MFMA and HBM time at peak is larger.  phases[dom] holds
    the summed time and count of the timed launches of that phase."""
    pf = phase_flops(w)
    pb = phase_bytes(w, prec)
    dom = max((p for p in pf if p in phases), key=lambda p: phases[p]["ms"])
    avg_ms = phases[dom]["ms"] / max(phases[dom]["launches"], 1)
    flops_launch = pf[dom] * w.npairs / launches_per_step
    bytes_launch = pb[dom] / launches_per_step
    peak_f = PEAKS_TFLOPS[prec]
    hbm_bound = bytes_launch / (HBM_PEAK_GBS * 1e9) >= flops_launch / (peak_f * 1e12)
    if hbm_bound:
        roof = {"bound": "hbm", "achieved": bytes_launch / (avg_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "algorithmic_bytes_per_launch": bytes_launch}
    else:
        roof = {"bound": "mfma", "achieved": flops_launch / (avg_ms * 1e-3) / 1e12, "peak": peak_f,
                "unit": "TFLOP/s", "algorithmic_flops_per_launch": flops_launch}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = recorded_traffic(w.name, prec, dom)
    roof.update({"kernel": dom, "avg_launch_ms": avg_ms,
                 "mfma_tflops": flops_launch / (avg_ms * 1e-3) / 1e12, "mfma_peak": peak_f,
                 "hbm_gbs": bytes_launch / (avg_ms * 1e-3) / 1e9})
    return roof


def vx_energy(psi, vx, occ, dV):
    """The exchange energy Vx psi implies, 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h
    (equal to E_x for the exact operator), in FP64 on the host."""
    import numpy as np
    tot = 0.0
    for j in range(psi.shape[0]):
        a = np.asarray(psi[j], dtype=np.float64).ravel()
        b = np.asarray(vx[j], dtype=np.float64).ravel()
        tot += occ[j] * dV * float(a @ b)
    return 0.25 * tot


def measure(g, w, psi_d, occ, vx, prec, steps, warmup, tune, tune_cache=None, graph=True):
    """Warm-up, then `steps` timed exchange applications on the stream the
    library runs on: replays of one kx_apply_exchange recorded into a HIP
    graph (eager calls with graph=False).  Per-phase times
    (phases_ms_per_step) come from the library's events on the last warm-up
    step; the roofline's launch time from events around the dominant phase's
    launches, recorded into the graph with the launches (their times are
    those of the last replay)."""
    import torch
    dt = "f64" if psi_d.dtype == torch.float64 else "f32"
    t0 = time.perf_counter()
    if tune:
        g.autotune(prec=prec, dtype=dt, cache_path=tune_cache)
    tune_s = time.perf_counter() - t0
    g.reserve(w.norb, prec, dt)
    s = g.stream

    def step():
        g.apply_exchange(psi_d, occ, w.kernel, w.omega, prec=prec, out=vx, reserve=False)

    for k in range(max(warmup, 1)):
        if k == max(warmup, 1) - 1:
            g.profile(True)
        step()
        g.exchange_energy()
        print(f"# {prec} warmup {k + 1}/{max(warmup, 1)} done", file=sys.stderr, flush=True)
    phases1 = {}
    for ph in ("forward", "pencil", "inverse", "accum", "energy"):
        ms, cnt = g.profile_read(ph)
        phases1[ph] = {"ms": ms, "launches": cnt}
    g.profile(False)
    dom = max(("forward", "pencil", "inverse", "accum"), key=lambda p: phases1[p]["ms"])
    # one eager step creates the dominant phase's events; recording the step
    # into the graph then records them as graph nodes
    g.profile_phases([dom])
    step()
    g.profile_phases([dom])
    G = None
    if graph:
        G = torch.cuda.CUDAGraph()
        with torch.cuda.graph(G, stream=s):
            step()
        with torch.cuda.stream(s):  # a replay runs on the current stream
            G.replay()
        s.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        start.record(s)
        for _ in range(steps):
            if G is not None:
                G.replay()
            else:
                step()
        stop.record(s)
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    ex = g.exchange_energy()
    timing = "graph replay" if G is not None else "eager"
    try:
        ms, cnt = g.profile_read(dom)
        per_step = cnt if G is not None else max(cnt / steps, 1)
    except Exception as e:  # event nodes without timestamps: time eager launches instead
        print(f"# {prec}: graph event times unavailable ({e}); timing eager launches",
              file=sys.stderr, flush=True)
        g.profile_phases([dom])
        step()
        ms, cnt = g.profile_read(dom)
        per_step = cnt
        timing = "graph replay (launch times from an eager step)"
    g.profile(False)
    del G
    phases = {p: {"ms": 0.0, "launches": 0} for p in phases1}
    phases[dom] = {"ms": ms, "launches": cnt}
    ms_step = ms_total / steps
    print(f"# {prec}: {steps} steps {ms_total:.1f} ms ({timing})", file=sys.stderr, flush=True)
    pf = phase_flops(w)
    return {"value": w.npairs / (ms_step * 1e-3), "ms_per_step": ms_step, "E_x": ex,
            "timing": timing,
            "phases_ms_per_step": {p: v["ms"] for p, v in phases1.items()},
            "roofline": roofline(w, prec, phases, per_step),
            "tflops_whole_step": sum(pf.values()) * w.npairs / (ms_step * 1e-3) / 1e12,
            "plan": g.plan(prec), "tune_s": tune_s}


def golden_ex(name):
    """E_x of a workload as stored from the oracle, or None."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_energies.json")
    try:
        with open(path) as fh:
            return json.load(fh).get(name, {}).get("E_x")
    except OSError:
        return None


def prec_line(p, r):
    return (f"{p}: {r['value']:.0f} pair-solves/s, E_x={r['E_x']!r}, "
            f"E_vx={r['E_vx']!r}")


def measure_ace(g, psi_d, vx, w, reps=5):
    """The compressed exchange built from the last Vx psi (kx_ace_build: one
    status read-back included) and applied to the orbitals themselves
    (kx_ace_apply, norb fields); average of `reps` calls after one warm-up.
    Bytes: build reads psi and W, then W again, and writes xi; apply reads xi
    and phi, then xi again, and writes the output (4 fields each)."""
    import torch
    xi = g.ace_build(psi_d, vx)
    out = g.ace_apply(xi, psi_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.ace_build(psi_d, vx, out=xi)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3 / reps
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(g.stream)
    for _ in range(reps):
        g.ace_apply(xi, psi_d, out=out)
    stop.record(g.stream)
    torch.cuda.synchronize()
    apply_ms = start.elapsed_time(stop) / reps
    field = psi_d.numel() * psi_d.element_size()
    return {"build_ms": build_ms, "apply_ms": apply_ms, "nvec": w.norb,
            "apply_GBps": 4 * field / (apply_ms * 1e-3) / 1e9,
            "build_GBps": 4 * field / (build_ms * 1e-3) / 1e9}


def measure_multipole(nfields=64, lmax=6, reps=5):
    """Single solves on an isolated-system grid (80^3 Dirichlet, h = 0.3,
    order 12, the grid of the ragged batch's third system): kx_apply_fL with
    homogeneous Dirichlet values against kx_apply_fL_multipole (boundary
    values from the multipole expansion to lmax), FP64, on the pair densities
    psi_0 psi_j of that system's orbitals; then the exchange of its orbitals
    with homogeneous ends against kx_apply_exchange_multipole.  Mean of
    `reps` calls after one warm-up, HIP events on the library's stream."""
    import numpy as np
    import torch

    from paper_2406_16998_amd import kx
    from synth import make_workload
    w, psi, _ = make_workload("ragged_c_dirichlet80")
    k = min(nfields, w.norb)
    rho = torch.from_numpy(np.ascontiguousarray(psi[0:1] * psi[:k])).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    g = kx.Grid(w.n, w.h, w.order, w.bc, stream=stream)
    out = torch.empty_like(rho)
    res = {}
    for name, call in (("homogeneous", lambda: g.apply_fL(rho, "coulomb", out=out)),
                       ("multipole", lambda: g.apply_fL_multipole(rho, lmax=lmax, out=out))):
        call()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            start.record(stream)
            for _ in range(reps):
                call()
            stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / reps
        res[name] = {"ms_per_call": ms, "solves_per_s": k / (ms * 1e-3)}
    # the exchange of the same system (its orbitals, occupation 2): homogeneous
    # ends against multipole boundary values for every pair
    occ = np.full(w.norb, 2.0)
    psi_d = torch.from_numpy(psi).cuda()
    vx = torch.empty_like(psi_d)
    for name, call in (("exchange_homogeneous",
                        lambda: g.apply_exchange(psi_d, occ, "coulomb", out=vx)),
                       ("exchange_multipole",
                        lambda: g.apply_exchange_multipole(psi_d, occ, lmax=lmax, out=vx))):
        call()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            start.record(stream)
            for _ in range(reps):
                call()
            stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / reps
        res[name] = {"ms_per_call": ms, "pair_solves_per_s": w.npairs / (ms * 1e-3),
                     "E_x": g.exchange_energy()}
    g.close()
    res.update({"grid": list(w.n), "fields": k, "orbitals": w.norb, "lmax": lmax, "prec": "fp64"})
    return res


def measure_solve_scaling(sizes=(32, 48, 64, 80, 96, 112, 128, 144, 160), nfields=64, reps=5,
                          precs=("fp64", "mixed")):
    """Single solves phi = f(-L) rho against the grid size (the paper's
    solve-time comparison, Fig. 1, for this library alone): cubic periodic
    grids of n^3 nodes, h = 0.3, order 12, erfc with omega = 0.106, a batch
    of `nfields` N(0, 1) fields per call, planner launch shapes; mean of
    `reps` calls after one warm-up, HIP events on the library's stream.
    Reports ms per solve and the exponent of a fit t ~ N^a over the grids of
    64^3 and more (the Kronecker solve costs O(N^(4/3)) flops)."""
    import numpy as np
    import torch

    from paper_2406_16998_amd import kx
    from synth import random_fields
    out = {"grids": list(sizes), "fields": nfields, "kernel": "erfc", "omega": 0.106}
    stream = torch.cuda.Stream()
    for prec in precs:
        rows = []
        for n in sizes:
            rho = torch.from_numpy(random_fields((n, n, n), nfields, seed=n)).cuda()
            res = torch.empty_like(rho)
            torch.cuda.synchronize()
            g = kx.Grid((n, n, n), (0.3,) * 3, 12, ("periodic",) * 3, stream=stream)
            g.apply_fL(rho, "erfc", 0.106, prec=prec, out=res)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                start.record(stream)
                for _ in range(reps):
                    g.apply_fL(rho, "erfc", 0.106, prec=prec, out=res, reserve=False)
                stop.record(stream)
            torch.cuda.synchronize()
            ms = start.elapsed_time(stop) / reps / nfields
            rows.append({"n": n, "N": n ** 3, "ms_per_solve": ms})
            g.close()
            del rho, res
        # below 64^3 a batch is too small to fill the GPU: fit the larger grids
        big = [r for r in rows if r["n"] >= 64] or rows
        logN = np.log([r["N"] for r in big])
        logt = np.log([r["ms_per_solve"] for r in big])
        a = float(np.polyfit(logN, logt, 1)[0])
        out[prec] = {"rows": rows, "fit_exponent": a}
        print(f"# solve scaling {prec}: t ~ N^{a:.2f}; " +
              ", ".join(f"{r['n']}^3 {r['ms_per_solve']:.3f} ms" for r in rows),
              file=sys.stderr, flush=True)
    return out


BLOCH_KMESH = [(a, b, c) for c in (0.0, 0.5) for b in (0.0, 0.5) for a in (0.0, 0.5)]


def measure_bloch(norb=8, reps=3, tune=True, tune_cache=None):
    """The k-point exchange on the headline grid (96^3 periodic, h = 0.35,
    order 12, erfc with omega = 0.106): a 2 x 2 x 2 Gamma-centred mesh of
    k-points with norb bands each (one spin channel, occupation 1, equal
    weights), FP64; seeded Bloch orbitals (sums of Gaussians times the
    k ramp).  The forward and inverse passes use the launch shapes the
    autotuner picks for the grid.  Mean of `reps` applications after one
    warm-up, HIP events on the library's stream."""
    import numpy as np
    import torch

    from paper_2406_16998_amd import kx
    from synth import WORKLOADS, bloch_orbitals
    w = WORKLOADS["periodic96_erfc"]
    kpts = BLOCH_KMESH
    nk = len(kpts)
    psi_h = bloch_orbitals(w.n, w.h, w.bc, kpts, norb, seed=11, n_centres=48)
    psi = torch.from_numpy(psi_h).cuda()
    del psi_h
    wk = np.full(nk, 1.0 / nk)
    occ = np.ones((nk, norb))
    stream = torch.cuda.Stream()
    g = kx.Grid(w.n, w.h, w.order, w.bc, stream=stream)
    if tune:
        g.autotune(prec="fp64", dtype="f64", cache_path=tune_cache)
    out = torch.empty_like(psi)
    call = lambda: g.apply_exchange_bloch(psi, kpts, wk, occ, w.kernel, w.omega, out=out)  # noqa: E731
    call()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(reps):
            call()
        stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    M = nk * norb
    npairs = M * (M + 1) // 2
    ex = g.exchange_energy()
    g.close()
    return {"grid": list(w.n), "kpoints": nk, "bands": norb, "state_pairs": npairs,
            "ms_per_application": ms, "state_pairs_per_s": npairs / (ms * 1e-3),
            "E_x": ex, "prec": "fp64"}


def bench_ragged(args):
    """The six-system ragged batch through kx_batch_apply_exchange (one graph
    replay per step).  The call synchronises, so steps are timed on the host
    clock around it."""
    import torch

    from paper_2406_16998_amd import kx
    from synth import RAGGED_BATCH, make_workload
    precs = ["fp64", "bf16x3", "mixed"] if args.prec == "all" else [args.prec]
    systems = []
    for name in RAGGED_BATCH:
        w, psi, occ = make_workload(name)
        systems.append((w, psi, occ, kx.Grid(w.n, w.h, w.order, w.bc), torch.from_numpy(psi).cuda()))
    npairs = sum(s[0].npairs for s in systems)
    print(f"# ragged batch: {len(systems)} systems, {npairs} pairs", file=sys.stderr, flush=True)
    outs = [torch.empty_like(s[4]) for s in systems]
    res = {}
    for prec in precs:
        if not args.no_tune:
            for s in systems:
                s[3].autotune(prec=prec, dtype="f64", cache_path=args.tune_cache)
        call = lambda: kx.batch_apply_exchange([s[3] for s in systems], [s[4] for s in systems],  # noqa: E731
                                               [s[2] for s in systems], [s[0].kernel for s in systems],
                                               [s[0].omega for s in systems], prec=prec, outs=outs)
        for _ in range(max(args.warmup, 1)):  # the first call records the graph
            call()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, exs = call()
        dt = (time.perf_counter() - t0) / args.steps
        # the same systems one after another through the single-system entry point
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s, o in zip(systems, outs):
            s[3].apply_exchange(s[4], s[2], s[0].kernel, s[0].omega, prec=prec, out=o)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t1
        res[prec] = {"value": npairs / dt, "ms_per_step": dt * 1e3, "E_x": exs,
                     "sequential_single_calls_ms": seq * 1e3,
                     "plans": [s[3].plan(prec) for s in systems]}
        print(f"# ragged {prec}: {dt * 1e3:.1f} ms per batch", file=sys.stderr, flush=True)
    head = precs[0]
    result = {
        "metric": METRIC + " (ragged six-system batch)",
        "value": res[head]["value"], "unit": "pair-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res[head]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_NAME[head], "data": "synthetic",
        "config": {"workload": "ragged6", "systems": [s[0].name for s in systems], "pairs": npairs,
                   "prec": head},
        "variants": res,
    }
    for s in systems:
        s[3].close()
    print(json.dumps(result))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="all", choices=["all"] + sorted(PEAKS_TFLOPS),
                    help="all: FP64, FP32, split-BF16 and mixed in one run")
    ap.add_argument("--workload", default="periodic96_erfc", help="a synth workload, or 'ragged'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the planner's launch shapes")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner result file: read if it holds this grid, else appended")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-multipole", action="store_true",
                    help="skip the isolated-system single-solve timing")
    ap.add_argument("--no-bloch", action="store_true",
                    help="skip the k-point exchange timing")
    ap.add_argument("--bloch-only", action="store_true",
                    help="time only the k-point exchange (for profiling)")
    ap.add_argument("--solve-scaling", action="store_true",
                    help="time single solves against the grid size and exit")
    ap.add_argument("--multipole-only", action="store_true",
                    help="time only the isolated-system solves and exchange (for profiling)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls instead of replays of a recorded graph")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exchange path runs on a single GPU",
              file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch

    from paper_2406_16998_amd import kx
    from synth import make_workload

    torch.cuda.set_device(0)
    if args.solve_scaling:
        print(json.dumps({"solve_scaling": measure_solve_scaling()}))
        return
    if args.multipole_only:
        print(json.dumps({"multipole": measure_multipole()}))
        return
    if args.bloch_only:
        print(json.dumps({"bloch": measure_bloch(tune=not args.no_tune,
                                                  tune_cache=args.tune_cache)}))
        return
    if args.workload == "ragged":
        bench_ragged(args)
        return
    w, psi, occ = make_workload(args.workload)
    psi_d = torch.from_numpy(psi).cuda()
    vx = torch.empty_like(psi_d)
    torch.cuda.synchronize()
    # the library's stream: a stream of its own, so that a step can be
    # recorded into a graph
    stream = torch.cuda.Stream()
    t_setup = time.perf_counter()
    g = kx.Grid(w.n, w.h, w.order, w.bc, stream=stream)
    setup_s = time.perf_counter() - t_setup
    precs = ["fp64", "fp32", "bf16x3", "fp16x3", "mixed"] if args.prec == "all" else [args.prec]
    print(f"# workload {w.name}: {w.n} {w.bc} norb={w.norb} pairs={w.npairs} prec={precs}",
          file=sys.stderr, flush=True)
    # the reference energy: the oracle's (stored by tests/golden/make_golden.py)
    # when it has this workload, else the FP64 GPU path's
    ref_ex, ref_kind = golden_ex(w.name), "oracle"
    runs = {}
    for p in precs:
        runs[p] = measure(g, w, psi_d, occ, vx, p, args.steps, args.warmup, not args.no_tune,
                          args.tune_cache, graph=not args.eager)
        # the energy the operator itself implies, from the Vx psi just computed
        runs[p]["E_vx"] = float(vx_energy(psi, vx.cpu().numpy(), occ, w.dV))
        print(f"# {prec_line(p, runs[p])}", file=sys.stderr, flush=True)
    if ref_ex is None and "fp64" in runs:
        ref_ex, ref_kind = runs["fp64"]["E_x"], "fp64 GPU path"
    # the headline: the fastest variant whose E_x and Vx-psi-implied energy are
    # both within 1e-8 Ha of the reference (else the fastest that ran)
    for p, r in runs.items():
        r["dEx_vs_ref_Ha"] = None if ref_ex is None else abs(r["E_x"] - ref_ex)
        r["dEvx_vs_ref_Ha"] = None if ref_ex is None else abs(r["E_vx"] - ref_ex)
        r["meets_1e-8_Ha"] = (None if ref_ex is None else
                              bool(max(r["dEx_vs_ref_Ha"], r["dEvx_vs_ref_Ha"]) <= TARGET_DEX_HA))
    ok = [p for p, r in runs.items() if r["meets_1e-8_Ha"]] or list(runs)
    head = max(ok, key=lambda p: runs[p]["value"])
    hr = runs[head]
    result = {
        "metric": METRIC,
        "value": hr["value"],
        "unit": "pair-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[head],
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "h": list(w.h), "fd_order": w.order,
                   "bc": list(w.bc), "kernel": w.kernel, "omega": w.omega, "norb": w.norb,
                   "pairs": w.npairs, "prec": head, "storage": w.storage},
        "roofline": hr["roofline"],
        "vx_time_ms": hr["ms_per_step"],
        "E_x": hr["E_x"],
        "flops_per_pair": sum(phase_flops(w).values()),
        "unfolded_flops_per_pair": w.flops_per_pair(),
        "setup_s": setup_s,
        "variants": runs,
    }
    result["energy_reference"] = {"E_x": ref_ex, "source": ref_kind}
    result["headline_rule"] = ("fastest variant with |E_x - E_ref| and |E_vx - E_ref| <= 1e-8 Ha, "
                               "E_vx = 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h")
    if "fp64" in runs:
        result["speedup_vs_fp64"] = {p: r["value"] / runs["fp64"]["value"] for p, r in runs.items()}
        result["speedup_vs_fp64_at_1e-8_Ha"] = hr["value"] / runs["fp64"]["value"]
        split_ok = [p for p in SPLIT_PRECS if p in runs and runs[p]["meets_1e-8_Ha"]]
        result["split_mfma_speedup_at_1e-8_Ha"] = (
            None if not split_ok else
            {p: runs[p]["value"] / runs["fp64"]["value"] for p in split_ok})
    result["ace"] = measure_ace(g, psi_d, vx, w)
    if not args.no_multipole:
        result["multipole"] = measure_multipole()
    if not args.no_bloch:
        result["bloch"] = measure_bloch(tune=not args.no_tune, tune_cache=args.tune_cache)
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, psi, occ)
    g.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()

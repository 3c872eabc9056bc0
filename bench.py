#!/usr/bin/env python3
"""Throughput benchmark of the batched shifted-Laplace preconditioned Helmholtz
solve on one MI355X.

Workload: the 401 x 801 layered model (h = 10 m, eight layers 1500-4500 m/s
with a seeded 5 % rms, 200 m correlation perturbation), 64 surface shots x
frequencies {3, 5, 8, 12} Hz = 256 right-hand sides, complex128, BiCGSTAB
to relative residual 1e-8 with the LFA-planned V(2,2) shifted-Laplace
(1, 0.5) preconditioner, all right-hand sides in one batch.

A step = set the model (level hierarchy, coarse inverses per frequency) +
solve all 256 right-hand sides; inputs are resident in HBM before timing.
Prints one JSON line (see the field list at the end of main()).

  python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
  python bench.py --copy-calibration     # a plain copy kernel of known size,
                                         # for scaling rocprofv3 byte counters
  python bench.py --compare       # preconditioned vs not, shifts, GMRES vs BiCGSTAB,
                                  # Gauss-Newton schedules (a report, not a throughput line)
  python bench.py --3d            # batched solves on a 3D box (129^3, 16 right-hand sides) and its gradient; a report line
  python bench.py --density       # the same batch with a variable density (Eq. (1)); a report line
  python bench.py --gmres         # the same batch with GMRES(30), its Gram-Schmidt kernels' roofline
                                  # and BiCGSTAB beside it; a report line
  python bench.py --fwi           # gradient and Gauss-Newton step on the full inversion survey
                                  # (301 x 601, 32 shots x 6 frequencies; a report line)
  python bench.py --serving [--requests R] [--slots S]
      # serving stream: Poisson arrivals of mixed requests (side 129/257/513,
      # f ~ U(2, 15) Hz, 1-32 shots), rate set to 80 % of the measured
      # one-request-at-a-time service rate; p50/p99 latency and solves/s
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6  # dense FP64 matrix-core (and vector) peak
METRIC = "Helmholtz solves/s (2D 401x801, 64 RHS), HBM GB/s, p50/p99 solve latency"


def level_sizes(shape, levels):
    sizes, shp = [], tuple(shape)
    for _ in range(levels):
        sizes.append(int(shp[0] * shp[1]))
        shp = tuple((s - 1) // 2 + 1 for s in shp)
    return sizes


def bytes_per_iteration(sizes):
    """Algorithmic HBM bytes of one BiCGSTAB iteration of one right-hand side
    with two V(2,2) cycles, as the kernels run it: each complex vector a
    kernel touches is read or written once (16 B per node); the shared
    slowness and the per-frequency tables are not counted, nor the dense
    coarse inverse (one copy per frequency, shared by all its right-hand
    sides and read from cache). The benchmark's right-hand sides are point
    sources, so the shadow residual r^ = b is held as a one-entry list and
    the inner products with it stream no vector; v = B p^ is then never
    stored (the pre-smoothing kernels form it from p^), nor t = B s^ (the
    dot-product pass and the update each form it from s^). The iterate x
    is advanced every second iteration (with both iterations' p^ and s^;
    the current s^ is already read for t)."""
    z = 16
    n0 = sizes[0]
    total = n0 * z * (4 + 3)        # p and s updates (B p^ formed in the kernel) fused with the pre-sweeps
    total += n0 * z * 2             # <B s^, s>, <B s^, B s^>: reads s^, s
    total += n0 * z * 11 // 2       # r = s - omega B s^ (s^, s / r), x every second iteration (x, ph, ph0, sh0 / x)
    for l, n in enumerate(sizes[:-1]):
        nc = sizes[l + 1]
        per_cycle = nc * z                      # restricted residual
        per_cycle += n * z * 2 + nc * z         # post-smoothing: reads b, coarse e; writes u
        if l > 0:
            per_cycle += n * z                  # pre-sweeps from zero and restriction: read b
        total += 2 * per_cycle
    nc = sizes[-1]
    total += 2 * (2 * nc * z)                   # coarse right-hand side in, solution out
    return total


# Per fine-level kernel class: algorithmic bytes per right-hand side per
# BiCGSTAB iteration (two launches of each V-cycle kernel per iteration).
def class_bytes_per_iteration(sizes):
    z = 16
    n0, n1 = sizes[0], sizes[1]
    return {
        "presmooth": n0 * z * 4 + n1 * z,       # reads r, p_old, p^_old; writes p; coarse right-hand side
        "presmooth_s": n0 * z * 3 + n1 * z,     # reads r, p^; writes s; coarse right-hand side
        "prolong": 2 * (n0 * z * 2 + n1 * z),   # reads b, coarse e; writes u (two V-cycles)
        "apply": n0 * z * 2,                    # reads p^, r^ (only while some r^ is dense)
        "apply_s": n0 * z * 2,                  # reads s^, s (t = B s^ is not stored)
        # r = s - omega B s^ every iteration (reads s^, s; writes r), x every second
        # one (reads x, two p^, the other s^; writes x): 5.5 vectors per iteration
        "update": n0 * z * 11 // 2,
    }


def percentile(vals, q):
    s = sorted(vals)
    if not s:
        return None
    k = (len(s) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def _cpu_sample_worker(args):
    """One process of the CPU baseline: the oracle's set-up of B and the
    V-cycle for one frequency (the library's default plan: LFA levels and
    weights, coarse="auto"), then sample_iters BiCGSTAB iterations on one
    shot. Returns (freq, setup seconds, seconds per iteration)."""
    f, shot, sample_iters = args
    import numpy as np
    import workloads
    from oracle import operator as op, multigrid as mg, krylov, lfa
    w = workloads.model_2d_layered()
    om = 2 * np.pi * f
    t0 = time.perf_counter()
    B = op.operator_B(w.m, w.h, om, w.alpha)
    L, wj = lfa.plan(w.shape, w.h, om, w.m.min(), w.m.max(), 1.0, 0.5)
    V = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    t_setup = time.perf_counter() - t0
    b = op.point_source(w.shape, w.h, [w.src[shot]])
    t0 = time.perf_counter()
    _, it, _, _ = krylov.bicgstab(B, b, V, tol=1e-30, maxit=sample_iters)
    return f, t_setup, (time.perf_counter() - t0) / it


def host_cores():
    """Cores this process may run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, iters_per_freq, sample_iters=24):
    """Time the oracle (plain FP64 CPU: SciPy sparse matrices, BiCGSTAB, the
    V-cycle with the GPU's plan and coarse policy) with one process per host
    core and one BLAS thread each. All processes run at once (so the memory
    bandwidth they share is part of the measurement): process k takes
    frequency k mod 4 and a shot of its own, sets up the oracle's operator
    and V-cycle and runs sample_iters BiCGSTAB iterations. The full step is
    then P cores sharing 64 shots x the oracle's own iteration counts to
    convergence per frequency, each core also paying every frequency's
    set-up: wall = (sum_f 64 its_f t_f + P sum_f setup_f) / P."""
    import multiprocessing as mp
    import numpy as np
    P = host_cores()
    shots = [(k * 7 + 3) % len(w.src) for k in range(P)]
    jobs = [(float(w.freqs[k % len(w.freqs)]), shots[k], sample_iters) for k in range(P)]
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(P) as pool:
            res = pool.map(_cpu_sample_worker, jobs, chunksize=1)
        sample_s = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    per_freq = {}
    work = 0.0
    setup_all = 0.0
    for f in w.freqs:
        rs = [r for r in res if r[0] == float(f)]
        t_setup = float(np.mean([r[1] for r in rs]))
        t_it = float(np.mean([r[2] for r in rs]))
        n_it = iters_per_freq[str(f)]
        per_freq[str(f)] = {"setup_s": t_setup, "s_per_iteration": t_it, "iterations": n_it, "processes": len(rs)}
        work += len(w.src) * n_it * t_it
        setup_all += t_setup
    wall = (work + P * setup_all) / P
    nrhs = len(w.src) * len(w.freqs)
    return {"value": nrhs / wall, "unit": "solves/s", "cores": P, "kind": "oracle",
            "sample": (f"{P} processes at once (one per core, 1 BLAS thread each), each the oracle's set-up for one "
                       f"of the {len(w.freqs)} frequencies plus {sample_iters} BiCGSTAB iterations on its own shot "
                       f"({sample_s:.1f} s wall); scaled to {len(w.src)} shots x the oracle's mean iterations to "
                       "1e-8 per frequency (tests/golden/c3_oracle_iterations.json) shared by the "
                       f"{P} cores, each paying every frequency's set-up"),
            "host_cpus": os.cpu_count(), "per_freq": per_freq}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_direct_baseline(w, shots=4):
    """The paper's own way of solving (its observed data come from an LU
    factorisation): SuperLU of B at the first frequency plus `shots`
    triangular solves, on one core, scaled to the step (one factorisation per
    frequency, one solve per right-hand side)."""
    import numpy as np
    from oracle import operator as op, direct
    om = 2 * np.pi * w.freqs[0]
    t0 = time.perf_counter()
    lu = direct.factor_superlu(op.operator_B(w.m, w.h, om, w.alpha))
    t_factor = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k in range(shots):
        lu.solve(op.point_source(w.shape, w.h, [w.src[k]]))
    t_solve = (time.perf_counter() - t0) / shots
    nrhs = len(w.src) * len(w.freqs)
    total = len(w.freqs) * t_factor + nrhs * t_solve
    return {"value": nrhs / total, "unit": "solves/s", "cores": 1, "kind": "oracle, direct (SuperLU)",
            "sample": f"SuperLU factorisation of B at {w.freqs[0]} Hz ({t_factor:.1f} s) plus {shots} triangular "
                      f"solves ({t_solve:.2f} s each), scaled to {len(w.freqs)} factorisations and {nrhs} solves"}


def copy_calibration():
    """A plain copy of a known size through the library's copy kernel (the
    identity preconditioner): 64 vectors of 401 x 801 complex128 read and
    written once, for scaling hardware byte counters."""
    import torch
    import paper_1712_08743_amd as hz
    import workloads
    w = workloads.model_2d_layered()
    c = hz.Context(0)
    c.set_model(torch.from_numpy(w.m).cuda(), w.h)
    x = torch.randn((64,) + w.shape, dtype=torch.complex128, device="cuda")
    for _ in range(5):
        c.precond(3.0, x, precond="none")
    torch.cuda.synchronize()
    nbytes = x.numel() * 16
    print(json.dumps({"copy_kernel": "k_copy", "read_bytes": nbytes, "write_bytes": nbytes,
                      "launches": 5}), flush=True)


def serving_report(nreq=48, slots=4):
    """The serving stream (requests of the serving workload: sides 129/257/513,
    f ~ U(2, 15) Hz, 1-32 surface shots, one seeded model each) through the
    continuous-batching server: one request at a time through one context
    (the reference results and the one-at-a-time rate), then every request
    submitted at once (saturation), then Poisson arrivals at 80 % of the
    saturated served rate. Returns a dict of rates, latencies and the count
    of served results bitwise equal to the one-at-a-time ones."""
    import torch
    import paper_1712_08743_amd as hz
    import workloads

    reqs = [workloads.serving_request(r) for r in range(nreq)]
    dev = []
    for w in reqs:
        n = w.shape[0]
        b = torch.zeros((1, len(w.src), n, n), dtype=torch.complex128)
        for k, ix in enumerate(w.src):
            b[0, k, 0, ix] = 1.0 / w.h ** 2
        dev.append((torch.from_numpy(w.m).cuda(), b.cuda()))
    nsolve = sum(len(w.src) for w in reqs)
    tol = 1e-8

    ctx = hz.Context(0)
    for side in sorted({w.shape[0] for w in reqs}):  # warm up each grid size once
        k = next(i for i, w in enumerate(reqs) if w.shape[0] == side)
        ctx.set_model(dev[k][0], reqs[k].h)
        ctx.solve(reqs[k].freqs, reqs[k].alpha, dev[k][1], tol=tol)
    torch.cuda.synchronize()
    alone = []
    t0 = time.perf_counter()
    for w, (m, b) in zip(reqs, dev):
        ctx.set_model(m, w.h)
        u, _ = ctx.solve(w.freqs, w.alpha, b, tol=tol)
        alone.append(u)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    ctx.close()
    torch.cuda.empty_cache()
    print(f"# serving: one at a time, {nreq} requests, {nsolve} solves in {t_seq:.2f} s", file=sys.stderr, flush=True)

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)

    def run(arrivals):
        srv = hz.Server(0, budget_bytes=budget, slots=slots)
        tickets = []
        start = time.perf_counter()
        for w, (m, b), ta in zip(reqs, dev, arrivals):
            delay = start + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(m, w.h, w.freqs, w.alpha, b, tol=tol))
        lat, ends, same, conv = [], [], 0, 0
        for w, tk, ta, ref in zip(reqs, tickets, arrivals, alone):
            u, info, times = srv.wait(tk)
            lat.append(times[2])
            ends.append(ta + times[2])
            same += int(torch.equal(u, ref))
            conv += sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED)
        st = srv.stats()
        srv.close()
        makespan = max(ends)
        return {"solves_per_s": nsolve / makespan, "makespan_s": makespan,
                "latency_s": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
                "converged": conv, "identical_to_alone": same, "peak_running": st["peak_running"]}

    # warm the server path (engine set-up and launch-shape trials per grid size)
    run([0.0] * len(reqs))
    sat = run([0.0] * len(reqs))
    print(f"# serving: saturation {sat['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)
    rate = 0.8 * sat["solves_per_s"] * nreq / nsolve
    poi = run(list(workloads.poisson_arrivals(len(reqs), rate, seed=7)))
    print(f"# serving: Poisson arrivals {poi['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)
    return {
        "workload": f"serving stream: {nreq} requests, sides 129/257/513, f ~ U(2,15) Hz, 1-32 shots each, "
                    f"layered + Gaussian anomaly (one model per request), BiCGSTAB tol {tol:g}",
        "requests": nreq, "solves": nsolve, "server_workers": slots, "budget_bytes": budget,
        "one_at_a_time_solves_per_s": nsolve / t_seq,
        "saturation": sat,
        "poisson": dict(poi, arrival_rate_requests_per_s=rate),
        "saturation_speedup_over_one_at_a_time": sat["solves_per_s"] / (nsolve / t_seq),
    }


def serving(args):
    """Serving stream report (a report line, not the benchmark's throughput line)."""
    rep = serving_report(args.requests, args.slots)
    out = {"metric": "served Helmholtz solves/s (serving stream, saturation), p50/p99 request latency",
           "value": rep["saturation"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "c128", "data": "synthetic", "config": {"workload": rep["workload"]}, "serving": rep}
    print(json.dumps(out), flush=True)


def compare(args):
    """The paper's comparisons on synthetic inputs: Krylov iterations and time
    with and without the shifted-Laplace preconditioner, shift (1, 0.5)
    against the paper's 1 + j, GMRES(30) against BiCGSTAB (layered
    401 x 801 model, 4 shots x 4 frequencies); Gauss-Newton convergence with
    all frequencies inverted together and with low-to-high frequency groups
    (reduced inversion model), and the Krylov work of one Gauss-Newton
    iteration with and without the preconditioner."""
    import numpy as np
    import torch
    import paper_1712_08743_amd as hz
    from paper_1712_08743_amd import fwi
    import workloads

    out = {"metric": "comparisons (not a throughput line)", "data": "synthetic"}
    w = workloads.model_2d_layered()
    ctx = hz.Context(0)
    ctx.set_model(torch.from_numpy(w.m).cuda(), w.h)
    shots = [0, 21, 42, 63]
    b1 = ctx.point_rhs([0] * len(shots), [w.src[s] for s in shots])
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    cases = [("bicgstab", "mg", (1.0, 0.5)), ("bicgstab", "mg", (1.0, 1.0)), ("gmres", "mg", (1.0, 0.5)),
             ("gmres", "mg", (1.0, 1.0)), ("bicgstab", "none", (1.0, 0.5)), ("gmres", "none", (1.0, 0.5))]
    krylov = []
    for kr, pre, beta in cases:
        opt = dict(krylov=kr, precond=pre, beta=beta, tol=1e-8, maxit=args.compare_maxit if pre == "none" else 10000)
        ctx.solve(w.freqs[:1], w.alpha, b[:1, :1].contiguous(), **dict(opt, maxit=2))  # launch-shape trials
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = ctx.solve(w.freqs, w.alpha, b, **opt)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ns = len(shots)
        per = {}
        for k, f in enumerate(w.freqs):
            blk = info[k * ns:(k + 1) * ns]
            per[str(f)] = {"iterations_mean": float(np.mean([i[1] for i in blk])),
                           "converged": sum(1 for i in blk if i[0] == hz.HZ_RHS_CONVERGED)}
        krylov.append({"krylov": kr, "precond": pre, "shift": list(beta) if pre != "none" else None,
                       "seconds": sec, "per_freq": per,
                       "operator_applications_per_rhs": float(np.mean([i[1] for i in info])) *
                       (2 if kr == "bicgstab" else 1)})
        print(f"# {kr} {pre} {beta}: {sec:.2f} s", file=sys.stderr, flush=True)
    out["krylov"] = {"workload": f"2d-layered-401x801, shots {shots} x {w.freqs} Hz, tol 1e-8", "cases": krylov}
    ctx.close()

    # Gauss-Newton on a reduced inversion model; observed data from the
    # library's own solves on the true model at tolerance 1e-12
    g = workloads.model_fwi(nz=151, nx=301)
    src = [(0, ix) for ix in g.src]
    rec = [(0, ix) for ix in g.rec]
    ctx = hz.Context(0)
    ctx.set_model(torch.from_numpy(g.m), g.h)
    _, d_obs, _ = ctx.misfit(g.freqs, g.alpha, src, rec,
                             torch.zeros((len(g.freqs), len(src), len(rec)), dtype=torch.complex128), 0.0,
                             tol=1e-12)
    d_obs = d_obs.cpu()
    gn = {}
    for name, kw in (("simultaneous", dict(schedule="simultaneous", gn_iters=4)),
                     ("sequential", dict(schedule="sequential", groups=[[0, 1], [2, 3], [4, 5]], gn_iters=2))):
        t0 = time.perf_counter()
        _, hist = fwi.invert(ctx, g.m_start, g.h, g.freqs, g.alpha, src, rec, d_obs, g.lam, cg_iters=5,
                             m_true=g.m, tol=1e-8, **kw)
        gn[name] = {"seconds": time.perf_counter() - t0, "history": hist}
        print(f"# gauss-newton {name}: {gn[name]['seconds']:.1f} s", file=sys.stderr, flush=True)
    work = {}
    for pre in ("mg", "none"):
        ctx.set_model(torch.from_numpy(g.m_start), g.h)
        t0 = time.perf_counter()
        dm, J, it, info = ctx.gn_step(g.freqs, g.alpha, src, rec, d_obs, g.lam, 1, precond=pre, tol=1e-8,
                                      maxit=args.compare_maxit)
        torch.cuda.synchronize()
        work[pre] = {"seconds": time.perf_counter() - t0,
                     "forward_krylov_iterations_mean": float(np.mean([i[1] for i in info])),
                     "forward_converged": sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED),
                     "forward_solves": len(info)}
    ctx.close()
    out["gauss_newton"] = {"workload": f"fwi-151x301, {len(src)} shots, {len(rec)} receivers, {g.freqs} Hz, "
                                       f"lambda {g.lam}, 5 CG iterations per step (1 in the "
                                       f"with/without-preconditioner step)",
                           "schedules": gn, "one_step_with_and_without_preconditioner": work}
    print(json.dumps(out), flush=True)


def fwi_report(args):
    """The FWI pieces on the full inversion survey (301 x 601, 32 surface shots,
    151 receivers, six frequencies, lambda 1e-3): the adjoint-state gradient of
    Eq. (7) (a forward and an adjoint solve per shot and frequency) and one
    Gauss-Newton step of Eq. (9) (each CG iteration a Born and an adjoint
    batch), BiCGSTAB to 1e-8. Observed data come from the library's own solves
    on the true model at tolerance 1e-12. One JSON line (a report, not the
    throughput line)."""
    import torch
    import numpy as np
    import paper_1712_08743_amd as hz
    import workloads
    g = workloads.model_fwi()
    src = [(0, ix) for ix in g.src]
    rec = [(0, ix) for ix in g.rec]
    ctx = hz.Context(0)
    ctx.set_model(torch.from_numpy(g.m), g.h)
    _, d_obs, _ = ctx.misfit(g.freqs, g.alpha, src, rec,
                             torch.zeros((len(g.freqs), len(src), len(rec)), dtype=torch.complex128), 0.0,
                             tol=1e-12)
    d_obs = d_obs.cpu()
    ctx.set_model(torch.from_numpy(g.m_start), g.h)
    print("# fwi: warm-up gradient (also runs the launch-shape trials)", file=sys.stderr, flush=True)
    ctx.gradient(g.freqs, g.alpha, src, rec, d_obs, g.lam, tol=1e-8)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(reps):
        J, grad, info = ctx.gradient(g.freqs, g.alpha, src, rec, d_obs, g.lam, tol=1e-8)
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    nsol = len(info)
    print(f"# fwi: gradient {t_grad:.3f} s ({nsol} solves)", file=sys.stderr, flush=True)
    cg = 2
    t0 = time.perf_counter()
    dm, J_gn, cg_it, info_gn = ctx.gn_step(g.freqs, g.alpha, src, rec, d_obs, g.lam, cg, tol=1e-8)
    torch.cuda.synchronize()
    t_gn = time.perf_counter() - t0
    # solves of one step: the forward and adjoint batches of the gradient (nsol together), then a
    # Born and an adjoint batch per CG iteration (nsol again)
    gn_solves = nsol * (1 + int(cg_it))
    print(f"# fwi: Gauss-Newton step {t_gn:.3f} s ({cg_it} CG iterations)", file=sys.stderr, flush=True)
    ctx.close()
    nodes = g.shape[0] * g.shape[1]
    out = {
        "metric": "FWI gradient and Gauss-Newton step time",
        "unit": "s",
        "higher_is_better": False,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"fwi-{g.shape[0]}x{g.shape[1]}, {len(src)} shots, {len(rec)} receivers, "
                               f"{list(g.freqs)} Hz, lambda {g.lam}, BiCGSTAB tol 1e-8, V(2,2) shifted-Laplace "
                               f"(1,0.5)", "grid": list(g.shape), "nodes": nodes},
        "gradient": {"seconds": t_grad, "repeats": reps, "solves": nsol, "solves_per_s": nsol / t_grad,
                     "iterations_mean": float(np.mean([i[1] for i in info])),
                     "converged": sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED), "J": J},
        "gauss_newton_step": {"seconds": t_gn, "cg_iterations": int(cg_it), "solves": gn_solves,
                              "solves_per_s": gn_solves / t_gn, "J": J_gn,
                              "dm_norm": float(torch.linalg.norm(dm).item())},
    }
    print(json.dumps(out), flush=True)


def bench_3d(args):
    """Batched solves on a 3D box (Eq. (1) with d = 3, constant density): the
    layered 129 x 129 x 129 model (h = 20 m), 8 surface shots x 3 and 5 Hz =
    16 right-hand sides, BiCGSTAB to 1e-8 with the planned V(2,2)
    shifted-Laplace (1, 0.5) preconditioner. A step = set the model + solve
    the 16 right-hand sides, inputs resident in HBM. Kernel classes are timed
    with HIP events; the dominant one gives the roofline line. The CPU
    oracle is timed on a bounded sample (set-up plus a few BiCGSTAB
    iterations of one shot per frequency) and scaled to the batch with the
    oracle's own iteration counts to convergence
    (tests/golden/l3d_oracle_iterations.json). One JSON line, a report beside
    the 2D throughput line."""
    import torch
    import numpy as np
    import paper_1712_08743_amd as hz
    import workloads
    w = workloads.model_3d_layered(129, 129, 129, h=20.0, nshots=8, freqs=(3.0, 5.0))
    tol = 1e-8
    ctx = hz.Context(0)
    m = torch.from_numpy(w.m).cuda()
    ctx.set_model(m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b1 = ctx.point_rhs_3d(iz, iy, ix)
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    u = torch.empty_like(b)
    nrhs = b.shape[0] * b.shape[1]

    def step():
        ctx.set_model(m, w.h)
        _, info = ctx.solve(w.freqs, w.alpha, b, out=u, tol=tol)
        return info

    print(f"# 3d: warm-up step on {w.name}, {nrhs} right-hand sides", file=sys.stderr, flush=True)
    step()
    torch.cuda.synchronize()
    classes = ["smooth", "restrict", "prolong", "apply", "apply_s", "update", "coarse"]
    ctx.timing_start(classes)
    steps = max(1, min(args.steps, 3))
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(step())
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    timing = {k: ctx.timing_read(k) for k in classes}
    ctx.timing_start([])
    print(f"# 3d: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    info = infos[-1]
    iters = [i[1] for i in info]
    slot_iters = sum(sum(i[1] for i in inf) for inf in infos)
    n0 = int(np.prod(w.shape))
    n1 = int(np.prod(ctx.level_shape(1)))
    z = 16
    # algorithmic bytes per right-hand side and iteration of the finest-level classes (two V-cycles;
    # the p and s updates are not timed)
    cb = {"smooth": 2 * 2 * n0 * z,                  # both pre-sweeps from zero: b / u
          "restrict": 2 * (2 * n0 * z + n1 * z),     # b, u / coarse b
          "prolong": 2 * (3 * n0 * z + n1 * z),      # coarse e, b, u / u (with both post-sweeps)
          "apply": 2 * n0 * z,                       # p^ / v
          "apply_s": 3 * n0 * z,                     # s^, s / t
          "update": 6 * n0 * z}                      # s, t / r; x every second iteration
    breakdown = {}
    for k in classes:
        n, ms = timing[k]
        e = {"launches": n, "ms": ms / steps}
        if k in cb and ms > 0:
            e["GB/s"] = slot_iters * cb[k] / (ms * 1e-3) / 1e9
        breakdown[k] = e
    dom = max((k for k in cb if timing[k][0] > 0), key=lambda k: timing[k][1])
    achieved = slot_iters * cb[dom] / (timing[dom][1] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "launches": timing[dom][0], "avg_launch_ms": timing[dom][1] / max(timing[dom][0], 1)}
    levels = [ctx.plan(f)[0] for f in w.freqs]
    # the adjoint-state gradient (Eq. (7)) on the same box: observed data from the library's own
    # solves on the layered model at tolerance 1e-12, the gradient at a second seed's model
    rec = [(0, y, x) for y in range(0, 129, 8) for x in range(0, 129, 8)]
    _, d_obs, _ = ctx.misfit_3d(w.freqs, w.alpha, w.src, rec,
                                torch.zeros((len(w.freqs), len(w.src), len(rec)), dtype=torch.complex128), 0.0,
                                tol=1e-12)
    start = workloads.model_3d_layered(129, 129, 129, h=20.0, nshots=8, freqs=(3.0, 5.0), seed=3)
    ctx.set_model(torch.from_numpy(start.m).cuda(), w.h)
    print("# 3d: warm-up gradient", file=sys.stderr, flush=True)
    ctx.gradient_3d(w.freqs, w.alpha, w.src, rec, d_obs, 1e-3, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, ginfo = ctx.gradient_3d(w.freqs, w.alpha, w.src, rec, d_obs, 1e-3, tol=tol)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    print(f"# 3d: gradient {t_grad:.3f} s ({len(ginfo)} solves)", file=sys.stderr, flush=True)
    gradient = {"seconds": t_grad, "solves": len(ginfo), "solves_per_s": len(ginfo) / t_grad,
                "converged": sum(1 for i in ginfo if i[0] == hz.HZ_RHS_CONVERGED),
                "receivers": len(rec), "lambda": 1e-3,
                "note": "forward and adjoint batch of 8 shots x 2 frequencies, data from the library at 1e-12"}
    ctx.close()
    cpu = None
    if not args.no_cpu_baseline:
        print("# 3d: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        with open(os.path.join(ROOT, "tests", "golden", "l3d_oracle_iterations.json")) as fh:
            gold = json.load(fh)
        cpu = cpu_baseline_3d(w, {k: v["mean_iterations"] for k, v in gold["freqs"].items()}, len(w.src))
    out = {
        "metric": "Helmholtz solves/s (3D 129^3, 16 RHS)",
        "value": nrhs / sec, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"{w.name}, h {w.h} m, 8 surface shots x {w.freqs} Hz = 16 RHS, BiCGSTAB tol 1e-8, "
                               "V(2,2) shifted-Laplace (1,0.5), LFA-planned weights",
                   "grid": list(w.shape), "levels": levels},
        "converged": sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED and i[2] <= tol),
        "iterations_mean_per_freq": {str(f): float(np.mean(iters[k * len(w.src):(k + 1) * len(w.src)]))
                                     for k, f in enumerate(w.freqs)},
        "kernel_breakdown": breakdown,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "gradient": gradient,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_3d(w, iters_per_freq, nshot, sample_iters=3):
    """The oracle on one shot per frequency: its V-cycle set-up plus
    sample_iters BiCGSTAB iterations, scaled to the batch (nshot shots per
    frequency, the oracle's mean iterations to convergence per frequency)."""
    import numpy as np
    from oracle import operator as op
    from oracle import multigrid as mg
    from oracle import krylov
    from oracle import lfa
    total = 0.0
    per_freq = {}
    t_all = time.perf_counter()
    for k, f in enumerate(w.freqs):
        om = 2 * np.pi * f
        t0 = time.perf_counter()
        B = op.operator_B(w.m, w.h, om, w.alpha)
        L, wj = lfa.plan(w.shape, w.h, om, float(w.m.min()), float(w.m.max()), 1.0, 0.5)
        vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
        t_setup = time.perf_counter() - t0
        iz, iy, ix = w.src[0]
        bn = op.point_source(w.shape, w.h, [(iz * w.shape[1] + iy) * w.shape[2] + ix])
        t0 = time.perf_counter()
        krylov.bicgstab(B, bn, vc, tol=1e-30, maxit=sample_iters)
        t_it = (time.perf_counter() - t0) / sample_iters
        n_it = iters_per_freq[str(f)]
        total += t_setup + nshot * n_it * t_it
        per_freq[str(f)] = {"setup_s": t_setup, "s_per_iteration": t_it, "iterations": n_it}
    sample_s = time.perf_counter() - t_all
    return {"value": nshot * len(w.freqs) / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one shot per frequency: the oracle's V-cycle set-up plus {sample_iters} BiCGSTAB "
                      f"iterations ({sample_s:.1f} s of CPU), scaled to {nshot} shots x the oracle's mean "
                      "iterations to 1e-8 per frequency (tests/golden/l3d_oracle_iterations.json)",
            "host_cpus": os.cpu_count(), "per_freq": per_freq}


def one_rhs_per_call(ctx, w, b1, tol, shot=31, plain=False):
    """One right-hand side per solve call (shot ``shot`` at every frequency of
    the workload); solves/s over the four solves and their mean iterations.
    plain=False: the library's batched path called with a batch of one;
    plain=True: the plain per-launch path (every step of the iteration a
    kernel of its own, scalars read back by the host every iteration)."""
    import torch
    secs, its = [], []
    for f in w.freqs:
        bb = b1[shot:shot + 1].reshape((1, 1) + tuple(b1.shape[1:])).contiguous()
        ctx.solve([f], w.alpha, bb, tol=tol, plain=plain)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = ctx.solve([f], w.alpha, bb, tol=tol, plain=plain)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        its.append(info[0][1])
    return len(secs) / sum(secs), its


def bench_density(args):
    """Variable density (Eq. (1)) on the benchmark batch: the layered 401 x 801
    model with a density that follows it (Gardner's rule, relative to the
    slowest velocity), 64 surface shots x 3/5/8/12 Hz = 256 right-hand sides,
    BiCGSTAB to 1e-8 with the planned V(2,2) shifted-Laplace (1, 0.5)
    preconditioner, which a density solve applies with its per-step kernels.
    A step = set the model and the density + solve, inputs resident in HBM.
    The constant-density batch is timed beside it in the same process. One
    JSON line, a report beside the headline line."""
    import torch
    import numpy as np
    import paper_1712_08743_amd as hz
    import workloads
    w = workloads.model_2d_layered()
    rho = torch.from_numpy(workloads.gardner_density(w.m)).cuda()
    nshot, nfreq = len(w.src), len(w.freqs)
    nrhs = nshot * nfreq
    ctx = hz.Context(0)
    m = torch.from_numpy(w.m).cuda()
    ctx.set_model(m, w.h)
    b1 = ctx.point_rhs([0] * nshot, w.src)
    b = torch.stack([b1] * nfreq).contiguous()
    u = torch.empty_like(b)
    tol = 1e-8
    out = {"metric": "Helmholtz solves/s (2D 401x801, 256 RHS, variable density of Eq. (1))", "unit": "solves/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "2d-layered-401x801 with a Gardner density (rho ~ c^(1/4), 1 to 1.3), 64 surface "
                                  "shots x {3,5,8,12} Hz = 256 RHS, BiCGSTAB tol 1e-8, V(2,2) shifted-Laplace "
                                  "(1,0.5), LFA-planned weights for m / sqrt(rho)"}}
    for name, dens in (("density", rho), ("constant", None)):
        def step():
            ctx.set_model(m, w.h)
            if dens is not None:
                ctx.set_density(dens)
            _, info = ctx.solve(w.freqs, w.alpha, b, out=u, tol=tol)
            return info
        print(f"# {name}: warm-up step", file=sys.stderr, flush=True)
        step()
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(steps):
            info = step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        print(f"# {name}: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
        iters = [i[1] for i in info]
        res = {"value": nrhs / sec, "ms_per_step": sec * 1e3, "steps": steps, "warmup": 1,
               "converged": sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED and i[2] <= tol),
               "iterations_mean_per_freq": {str(f): float(np.mean(iters[k * nshot:(k + 1) * nshot]))
                                            for k, f in enumerate(w.freqs)},
               "levels": ctx.plan(w.freqs[0])[0]}
        if name == "density":
            out.update(res)
        else:
            out["constant_density"] = res
    out["ratio_to_constant_density"] = out["value"] / out["constant_density"]["value"]
    print(json.dumps(out), flush=True)


def gmres_step_bytes(iters, m, n, z=16):
    """Algorithmic bytes of GMRES(m)'s Gram-Schmidt step kernels for one
    right-hand side that took `iters` Arnoldi columns: step j of a cycle
    reads the j finished basis vectors, u_j and the operator's product twice
    (the dot pass and the update pass) and writes v_j and u_{j+1}; the step
    that decides a cycle's last column k < m only makes the dot pass over
    k + 2 vectors, and a cycle of m columns ends with a dot pass over its
    m + 1 vectors. Cycles are taken as m columns each but the last (a restart
    on a residual estimate that the true residual does not confirm would add
    one more short cycle)."""
    full, rest = divmod(int(iters), m)
    cycles = [m] * full + ([rest] if rest else [])
    vecs = 0
    for k in cycles:
        vecs += sum(2 * j + 6 for j in range(k)) + (k + 2 if k < m else m + 1)
    return vecs * n * z


def bench_gmres(args):
    """GMRES(30), the paper's Krylov method, on the benchmark batch: the
    layered 401 x 801 model, 64 surface shots x 3/5/8/12 Hz = 256 right-hand
    sides, tolerance 1e-8, V(2,2) shifted-Laplace (1, 0.5) preconditioner.
    A step = set the model + solve, inputs resident in HBM. The Gram-Schmidt
    step kernels (the `update` timing class: the dot pass, the per-slot
    scalars and the update pass of each Arnoldi step) are timed with HIP
    events and priced by their algorithmic bytes; BiCGSTAB's rate on the same
    batch is measured beside it. One JSON line, a report beside the headline
    line."""
    import torch
    import numpy as np
    import paper_1712_08743_amd as hz
    import workloads
    w = workloads.model_2d_layered()
    nshot, nfreq = len(w.src), len(w.freqs)
    nrhs = nshot * nfreq
    gm = 30
    ctx = hz.Context(0)
    m = torch.from_numpy(w.m).cuda()
    ctx.set_model(m, w.h)
    b1 = ctx.point_rhs([0] * nshot, w.src)
    b = torch.stack([b1] * nfreq).contiguous()
    u = torch.empty_like(b)
    tol = 1e-8
    n0 = int(np.prod(w.shape))
    out = {"metric": "Helmholtz solves/s (2D 401x801, 256 RHS, GMRES(30))", "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "2d-layered-401x801, 64 surface shots x {3,5,8,12} Hz = 256 RHS, GMRES(30) "
                                  "tol 1e-8, V(2,2) shifted-Laplace (1,0.5), LFA-planned weights"}}
    for kr in ("gmres", "bicgstab"):
        def step():
            ctx.set_model(m, w.h)
            _, info = ctx.solve(w.freqs, w.alpha, b, out=u, tol=tol, krylov=kr, gmres_m=gm)
            return info
        print(f"# {kr}: warm-up step", file=sys.stderr, flush=True)
        step()
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 3))
        if kr == "gmres":
            ctx.timing_start(["update", "apply"])
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(step())
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        print(f"# {kr}: {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
        info = infos[-1]
        iters = [i[1] for i in info]
        res = {"value": nrhs / sec, "ms_per_step": sec * 1e3, "steps": steps, "warmup": 1,
               "converged": sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED and i[2] <= tol),
               "iterations_mean_per_freq": {str(f): float(np.mean(iters[k * nshot:(k + 1) * nshot]))
                                            for k, f in enumerate(w.freqs)}}
        if kr == "gmres":
            n_up, ms_up = ctx.timing_read("update")
            n_ap, ms_ap = ctx.timing_read("apply")
            ctx.timing_start([])
            gs_bytes = sum(gmres_step_bytes(i[1], gm, n0) for inf in infos for i in inf)
            achieved = gs_bytes / (ms_up * 1e-3) / 1e9
            res["gram_schmidt"] = {"launch_groups": n_up, "ms_per_step": ms_up / steps,
                                   "share_of_step": ms_up / steps / (sec * 1e3),
                                   "algorithmic_GB_per_step": gs_bytes / steps / 1e9,
                                   "operator_apply_ms_per_step": ms_ap / steps}
            traffic = None
            tf = os.path.join(ROOT, "profiles", "gmres_step_traffic.json")
            if os.path.exists(tf):
                from paper_1712_08743_amd import profiling
                with open(tf) as fh:
                    tr = json.load(fh)
                if tr.get("kernel_source_hash") == profiling.kernel_source_hash():
                    traffic = tr["bytes_per_step"]
            res["roofline"] = {"bound": "hbm", "kernel": "Gram-Schmidt step (k_gm_dots2 + k_gm_fin2 + "
                                                         "k_gm_update2)",
                               "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                               "traffic_unit": "HBM bytes per benchmark step (rocprofv3 FETCH_SIZE + WRITE_SIZE "
                                               "over the step's Gram-Schmidt kernels, copy-calibrated)",
                               "algorithmic_bytes_per_step": gs_bytes / steps}
            out.update(res)
        else:
            out["bicgstab"] = res
    out["ratio_to_bicgstab"] = out["value"] / out["bicgstab"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--no-single-rhs", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--fwi", action="store_true")
    ap.add_argument("--3d", dest="three_d", action="store_true")
    ap.add_argument("--density", action="store_true")
    ap.add_argument("--gmres", action="store_true")
    ap.add_argument("--compare-maxit", type=int, default=20000)
    ap.add_argument("--maxit", type=int, default=10000,
                    help="iteration cap (below convergence only for short hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the batched solve of one GPU's share); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.serving:
        serving(args)
        return
    if args.compare:
        compare(args)
        return
    if args.fwi:
        fwi_report(args)
        return
    if args.three_d:
        bench_3d(args)
        return
    if args.density:
        bench_density(args)
        return
    if args.gmres:
        bench_gmres(args)
        return

    import numpy as np
    import torch
    import paper_1712_08743_amd as hz
    import workloads

    w = workloads.model_2d_layered()
    nshot, nfreq = len(w.src), len(w.freqs)
    nrhs = nshot * nfreq
    ctx = hz.Context(0)
    m = torch.from_numpy(w.m).cuda()
    ctx.set_model(m, w.h)
    b1 = ctx.point_rhs([0] * nshot, w.src)
    b = torch.stack([b1] * nfreq).contiguous()
    u = torch.empty_like(b)
    tol = 1e-8

    def step():
        ctx.set_model(m, w.h)
        _, info = ctx.solve(w.freqs, w.alpha, b, out=u, tol=tol, maxit=args.maxit)
        return info

    print(f"# warmup {args.warmup} step(s) on {w.name}, {nrhs} right-hand sides", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    classes = ["presmooth", "presmooth_s", "restrict", "prolong", "smooth", "apply", "apply_s", "update", "coarse"]
    ctx.timing_start(classes)
    infos, lat, lat_steps = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos.append(step())
        lat.extend(ctx.last_seconds)
        lat_steps.append(list(ctx.last_seconds))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = {k: ctx.timing_read(k) for k in classes}
    ctx.timing_start([])
    sec = (t1 - t0) / args.steps
    print(f"# timed {args.steps} step(s): {sec * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    # the V-cycle's coarser levels, timed in one more step after the timed region: events around
    # their many short launches would lengthen the timed steps (by about 4 %)
    ctx.timing_start(["levels"])
    step()
    torch.cuda.synchronize()
    levels = ctx.timing_read("levels")
    ctx.timing_start([])

    info = infos[-1]
    conv = sum(1 for i in info if i[0] == hz.HZ_RHS_CONVERGED and i[2] <= tol)
    iters = [i[1] for i in info]
    L, _ = ctx.plan(w.freqs[0])
    sizes = level_sizes(w.shape, L)
    per_freq_iters = {str(f): float(np.mean(iters[k * nshot:(k + 1) * nshot])) for k, f in enumerate(w.freqs)}
    # per frequency (its shots share one operator): solve-time percentiles from the device clock,
    # and its shots over the time until the last of them converged, within the shared batch
    per_freq = {}
    for k, f in enumerate(w.freqs):
        sl = slice(k * nshot, (k + 1) * nshot)
        fl = [x for st in lat_steps for x in st[sl]]
        last = float(np.mean([max(st[sl]) for st in lat_steps]))
        per_freq[str(f)] = {"iterations_mean": per_freq_iters[str(f)],
                            "latency_s": {"p50": percentile(fl, 50), "p99": percentile(fl, 99)},
                            "solves_per_s": nshot / last if last > 0 else None}
    slot_iters = sum(sum(i[1] for i in inf) for inf in infos)  # over the timed steps
    step_bytes = sum(iters) * bytes_per_iteration(sizes)

    # per-class achieved bandwidth; the dominant class is the one with the most time
    cb = class_bytes_per_iteration(sizes)
    breakdown = {}
    for k in classes:
        n, ms = timing[k]
        entry = {"launches": n, "ms": ms}
        if k in cb and ms > 0:
            entry["GB/s"] = slot_iters * cb[k] / (ms * 1e-3) / 1e9
        if k == "coarse" and ms > 0:
            entry["TFLOP/s"] = slot_iters * 2 * 8 * sizes[-1] ** 2 / (ms * 1e-3) / 1e12
            entry["frac_fp64_peak"] = entry["TFLOP/s"] / PEAK_FP64_TFLOPS
        breakdown[k] = entry
    breakdown["levels"] = {"launches": levels[0], "ms": levels[1], "steps": 1,
                           "note": "coarser V-cycle levels, timed in one extra step after the timed ones"}
    dom = max((k for k in classes if k in cb and timing[k][0] > 0), key=lambda k: timing[k][1])
    n_dom, ms_dom = timing[dom]
    dom_bytes = slot_iters * cb[dom]
    achieved = dom_bytes / (ms_dom * 1e-3) / 1e9 if ms_dom > 0 else None
    # measured HBM bytes per launch: counters per right-hand side (from a
    # committed rocprofv3 --pmc summary of the same kernel sources) times the
    # right-hand sides an average launch carries here
    from paper_1712_08743_amd import profiling
    launches_per_iter = 2 if dom == "prolong" else 1
    rhs_per_launch = slot_iters * launches_per_iter / max(n_dom, 1)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "dominant_kernel_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        ent = tr.get("classes", {}).get(dom)
        if tr.get("kernel_source_hash") == profiling.kernel_source_hash() and ent:
            traffic = (ent["fetch_bytes_per_rhs"] + ent["write_bytes_per_rhs"]) * rhs_per_launch
    roofline = {"bound": "hbm", "kernel": dom, "symbol": " + ".join(profiling.symbols_of(dom)),
                "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": (achieved / PEAK_HBM_GBS) if achieved else None, "traffic": traffic,
                "launches": n_dom, "avg_launch_ms": ms_dom / max(n_dom, 1),
                "algorithmic_bytes_per_launch": dom_bytes / max(n_dom, 1), "rhs_per_launch": rhs_per_launch}

    single = plain = None
    if not args.no_single_rhs and args.maxit >= 10000:
        print("# timing one right-hand side per call (batched library, then the plain path)", file=sys.stderr,
              flush=True)
        rate, its = one_rhs_per_call(ctx, w, b1, tol)
        single = {"solves_per_s": rate, "iterations": its, "speedup": (nrhs / sec) / rate}
        rate, its = one_rhs_per_call(ctx, w, b1, tol, plain=True)
        plain = {"solves_per_s": rate, "iterations": its, "speedup": (nrhs / sec) / rate,
                 "what": "one right-hand side per call, every step of the iteration a kernel of its own "
                         "(single smoothing sweeps, residual and restriction, prolongation, operator apply, "
                         "vector updates), dense shadow residual, the host reading every iteration's scalars "
                         "back before it issues the next"}

    # the same batch with the paper's own shift 1 + j, (beta1, beta2) = (1, 1) (its Examples)
    paper_shift = None
    if not args.no_single_rhs and args.maxit >= 10000:
        print("# the same batch with the shift (1, 1)", file=sys.stderr, flush=True)

        def step11():
            ctx.set_model(m, w.h)
            _, inf = ctx.solve(w.freqs, w.alpha, b, out=u, tol=tol, beta=(1.0, 1.0))
            return inf
        step11()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            info11 = step11()
        torch.cuda.synchronize()
        sec11 = (time.perf_counter() - t0) / 2
        its11 = [i[1] for i in info11]
        paper_shift = {"solves_per_s": nrhs / sec11, "ms_per_step": sec11 * 1e3, "steps": 2,
                       "converged": sum(1 for i in info11 if i[0] == hz.HZ_RHS_CONVERGED and i[2] <= tol),
                       "iterations_mean_per_freq": {str(f): float(np.mean(its11[k * nshot:(k + 1) * nshot]))
                                                    for k, f in enumerate(w.freqs)},
                       "levels": ctx.plan(w.freqs[0], beta=(1.0, 1.0))[0],
                       "what": "the benchmark batch with the shifted Laplacian of the paper's examples, "
                               "(beta1, beta2) = (1, 1); value keeps (1, 0.5)"}

    serve = None
    if not args.no_serving and args.maxit >= 10000:
        del ctx
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print("# serving stream (continuous batching)", file=sys.stderr, flush=True)
        serve = serving_report(args.requests, args.slots)

    cpu = cpu_lu = None
    if not args.no_cpu_baseline:
        gpath = os.path.join(ROOT, "tests", "golden", "c3_oracle_iterations.json")
        with open(gpath) as fh:
            gold = json.load(fh)
        its = {k: v["mean_iterations"] for k, v in gold["freqs"].items()}
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, its)
        cpu["cpu_model"] = cpu_model()
        print("# timing the direct (LU) solve on the CPU", file=sys.stderr, flush=True)
        cpu_lu = cpu_direct_baseline(w)

    out = {
        "metric": METRIC,
        "value": nrhs / sec,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "2d-layered-401x801, 64 surface shots x {3,5,8,12} Hz = 256 RHS, "
                               "BiCGSTAB tol 1e-8, V(2,2) shifted-Laplace (1,0.5), LFA-planned weights",
                   "grid": list(w.shape), "h": w.h, "rhs": nrhs, "levels": L, "tol": tol},
        "converged": conv,
        "iterations_mean_per_freq": per_freq_iters,
        "per_freq": per_freq,
        "per_freq_note": f"{nshot} shots per frequency share its operator; solves_per_s = {nshot} / the time "
                         "until the frequency's last shot converged inside the shared batch (the "
                         "frequencies run at the same time, so these rates do not add up to value)",
        "hbm_gbps_step_model": step_bytes / sec / 1e9,
        "latency_s": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "single_rhs_batched_library": single,
        "plain_per_launch": plain,
        "roofline": roofline,
        "kernel_breakdown": breakdown,
        "paper_shift": paper_shift,
        "serving": serve,
        "cpu_baseline": cpu,
        "cpu_direct_lu": cpu_lu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: time to ||r||/||y|| < 1e-6 on the 256^3 Helmholtz workload, GB/s per
iteration and the roofline of the dominant pass kernel, on one MI355X.

    python bench.py [--steps K] [--warmup W] [--shape 256,256,256]

Workload: 3-D Helmholtz, 256^3 grid at lambda/4, background n = 1.33 with 200
seeded random spheres (radius 2-12 px, n in [1.33, 1.5]), 16-px absorbing faces
ramping to 0.2i, Gaussian-beam source on the z = 20 plane (seed 2).  Canonical
form with the complex smallest-circle bias and ||V|| = 0.95; alpha = 0.9 (the
fastest of 0.7-1.0 on this workload: 240 iterations against 260 at 0.8).

A step is one full solve from x = 0 to ||y - A x||/||y|| < 1e-6 with the
default solver: complex64 iterations with the residual recomputed and
accumulated in FP64 every 100 iterations, the last cycle shortened to the
crossing of the tolerance that the rate between the last two checks predicts
(each FP64 check costs about three iterations; measured 20 -> 100: 70.6 ->
62.9 ms).  Inputs (B, y) are resident in HBM
before the timed region.  Reported beside it: the plain complex128 solve, the
plain complex64 solve's attainable residual, per-pass kernel times (hipEvents
on the solver's stream), the FP64 CPU oracle timed on a bounded sample, and
the other workloads under "modes": BiCGSTAB and GMRES(m) on the same
preconditioned operator, the pantograph in direct and antisymmetrised
form, diffusion (plain vs refined), flux-form tensor diffusion on the
256 x 256 ring and on a 128^3 random tensor medium, the five lowest eigenmodes of a double-ring well (512 x 512,
Lanczos with CG inner solves), 96 batched
2-D problems in one graph-captured schedule, and the learned initial guess
on 128^3 media (2000 training / 200 held-out media by default;
--learned-train/--learned-test/--learned-epochs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak (MI355X)
METRIC = "time to ‖r‖/‖y‖<1e-6 + GB/s/iter, 256³ Helmholtz; plain vs learned-x0 vs batched"


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "x_fused_helmholtz3d_256_traffic.md")


def recorded_traffic(plan, shape):
    """HBM bytes per x_fused launch from the committed rocprofv3 counter summary
    (one entry per load plan of the fused pass), or None if the kernel sources
    changed since the counters were taken or the plan has no entry."""
    import hashlib
    if shape != (256, 256, 256) or not os.path.exists(TRAFFIC_FILE):
        return None
    sha, per_plan = None, {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line.startswith("sources_sha256_16:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("traffic x_prefetch="):
            key, v = line.split(":", 1)
            f = dict(t.split("=") for t in key.split()[1:])
            per_plan[(int(f["x_prefetch"]), int(f["x_stream"]))] = int(v)
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2207_14222_amd", "csrc")
    src = open(os.path.join(csrc, "fft.hpp"), "rb").read() + open(os.path.join(csrc, "passes.hpp"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != sha:
        return None
    return per_plan.get((plan["x_prefetch"], plan["x_stream"]))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(prob, iters_needed, n_iter=3):
    """The FP64 oracle, as it stands, on the host: n_iter iterations of Algorithm 1
    timed, scaled to the GPU's iteration count (extrapolated time-to-tolerance)."""
    from oracle import canon, operators, richardson
    t0 = time.perf_counter()
    cp = canon.canonical_helmholtz(prob.k2, prob.source, prob.spacing)
    op = operators.Operator(cp)
    t_prep = time.perf_counter() - t0
    x = np.zeros(op.shape, dtype=np.complex128)
    t0 = time.perf_counter()
    for i in range(n_iter):
        x, _ = richardson.step(op, x, cp.y, 0.8)
        log(f"oracle iteration {i + 1}/{n_iter}")
    per_it = (time.perf_counter() - t0) / n_iter
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = operators.FFT_WORKERS if operators._sfft is not None else 1
    return {"value": per_it * iters_needed, "unit": "s", "cores": threads, "kind": "oracle",
            "cpu": model, "host_cpus": os.cpu_count(),
            "sample": f"{n_iter} FP64 oracle iterations at {'x'.join(map(str, op.shape))} "
                      f"({per_it:.2f} s/iteration; pocketfft transforms on {threads} threads, element-wise "
                      f"NumPy on one), extrapolated to {iters_needed} iterations; oracle canonicalisation "
                      f"{t_prep:.1f} s not included",
            "per_iteration_s": per_it}


def bench_diffusion(args, log):
    """Frequency-domain diffusion, 256 x 256 x 128 (constant D = 0.03 cm, log-normal mu_a
    blobs, 100 MHz, seed 3), alpha = 1: plain complex64, plain complex128 and complex64 +
    FP64 refinement every 20 iterations (the interval the workload names) and every
    --refine-every iterations (last cycle cut to the predicted crossing), each to
    ||r||/||y|| < 1e-6."""
    import torch
    from paper_2207_14222_amd import media, solver
    d = media.diffusion_blobs(seed=3)
    out = {"grid": list(d.shape), "alpha": 1.0, "tol": args.tol}
    runs = (("plain_c64", torch.complex64, False, args.check_every),
            ("plain_c128", torch.complex128, False, args.check_every),
            ("refined_c64_k20", torch.complex128, True, 20),
            ("refined_c64", torch.complex128, True, args.refine_every))
    for name, dt, refine, ce in runs:
        can = solver.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing, dtype=dt)
        op = solver.Operator(can.symbol, can.B, refine=refine)
        op.solve(can.y, alpha=1.0, tol=args.tol, maxit=5000, check_every=ce)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.solve(can.y, alpha=1.0, tol=args.tol, maxit=5000, check_every=ce)
        torch.cuda.synchronize()
        out[name] = {"time_ms": round((time.perf_counter() - t0) * 1e3, 3), "iterations": r.iterations,
                     "status": r.status_name, "rho": float(r.hist_true[-1, 1]),
                     ("refine_every" if refine else "check_every"): ce}
        log(f"diffusion {name}: {out[name]}")
        del op, can
    return out


def bench_config1(args, log):
    """1-D Helmholtz, N = 256 at lambda/4 (random n in [1, 1.5], 32-px absorbing ramps,
    point source at the centre, seed 1), complex128, alpha 0.8, the true residual
    checked every iteration: time to ||r||/||y|| < 1e-10 (the whole solve is one
    workgroup; launch and latency bound, no roofline)."""
    import torch
    from paper_2207_14222_amd import media, solver
    p = media.helmholtz_1d()
    can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
    op = solver.Operator(can.symbol, can.B)
    tol = 1e-10
    for _ in range(3):
        op.solve(can.y, alpha=0.8, tol=tol, maxit=5000, check_every=1)
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.solve(can.y, alpha=0.8, tol=tol, maxit=5000, check_every=1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    out = {"grid": [256], "dtype": "c128", "alpha": 0.8, "tol": tol, "check_every": 1,
           "iterations": r.iterations, "status": r.status_name, "rho": float(r.hist_true[-1, 1]),
           "time_to_tol_ms": round(t * 1e3, 4), "iterations_per_s": round(r.iterations / t, 1)}
    log(f"config 1 (1-D N = 256): {out}")
    return out


def bench_batch(args, log, sequential=True):
    """96 independent 2-D Helmholtz problems (sides drawn from {128, 256, 512, 1024},
    random disks, beam on row 20; seeds 4 / 4000+i) solved together by the autotuned
    batched schedule (grouped graph-captured launches in practice; complex64 + FP64
    refinement every --batch-refine-every iterations with each problem's final cycle
    predicted, tol 1e-6, alpha 0.9), against solving the same problems one at a time
    (plain complex128 checked every 20, and refined complex64)."""
    import torch
    from paper_2207_14222_amd import media, solver
    sizes = [args.batch_side] * args.batch_n if args.batch_side else media.batch_sizes(args.batch_n, seed=4)
    cans, ops = [], []
    for i, n in enumerate(sizes):
        p = media.helmholtz_disks(n=n, seed=4000 + i)
        cans.append(solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128))
        ops.append(solver.Operator(cans[-1].symbol, cans[-1].B, refine=True))
    log(f"batch: {len(sizes)} problems prepared")
    xs = [torch.zeros_like(c.y) for c in cans]
    b = solver.Batch(ops, [c.y for c in cans], xs, alpha=args.batch_alpha, tol=args.tol, maxit=args.batch_maxit)
    if args.batch_variant is None:
        variant = b.autotune(refine_every=args.batch_refine_every)
    else:
        variant = b.variant = args.batch_variant
    b.solve(refine_every=args.batch_refine_every, use_graph=True)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = b.solve(refine_every=args.batch_refine_every, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sched = "one persistent launch" if variant & 4 else "grouped launches, one graph replay per refinement cycle"
    log(f"batch: {sched}: {out.elapsed_ms:.1f} ms device, {wall * 1e3:.1f} ms wall, variant {variant}")
    if not sequential:
        return {"n_problems": len(sizes), "variant": variant, "schedule": sched,
                "aggregate_time_to_tol_ms": round(out.elapsed_ms, 3),
                "all_converged": bool(all(st == 0 for st in out.status))}
    # one problem at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op, c in zip(ops, cans):
        op.solve(c.y, alpha=args.batch_alpha, tol=args.tol, maxit=20000, check_every=args.batch_refine_every)
    torch.cuda.synchronize()
    seq_ref = time.perf_counter() - t0
    log(f"batch: sequential refined {seq_ref * 1e3:.1f} ms")
    ops128 = [solver.Operator(c.symbol, c.B) for c in cans]
    for op, c in zip(ops128[:2], cans[:2]):
        op.solve(c.y, alpha=args.batch_alpha, tol=args.tol, maxit=20000, check_every=args.check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its128 = []
    for op, c in zip(ops128, cans):
        its128.append(op.solve(c.y, alpha=args.batch_alpha, tol=args.tol, maxit=20000,
                               check_every=args.check_every).iterations)
    torch.cuda.synchronize()
    seq_plain = time.perf_counter() - t0
    log(f"batch: sequential plain complex128 {seq_plain * 1e3:.1f} ms")
    tdone = np.array(out.t_done_ms)
    it = np.array(out.iterations)
    n_pts = int(sum(n * n for n in sizes))
    per_size = {}
    for n in sorted(set(sizes)):
        m = np.array(sizes) == n
        per_size[str(n)] = {"count": int(m.sum()), "median_ms": round(float(np.median(tdone[m])), 3),
                            "max_ms": round(float(tdone[m].max()), 3), "median_iterations": int(np.median(it[m]))}
    # complex64 inner-iteration model bytes (2-D: 8 arrays per iteration); FP64 refinement passes excluded
    inner_bytes = float(sum(8 * 8 * n * n * int(k) for n, k in zip(sizes, it)))
    return {"n_problems": len(sizes), "points": n_pts, "graph": True, "variant": variant,
            "model_GB/s_inner": round(inner_bytes / (out.elapsed_ms * 1e-3) / 1e9, 1),
            "schedule": sched,
            "aggregate_time_to_tol_ms": round(out.elapsed_ms, 3), "wall_ms": round(wall * 1e3, 3),
            "all_converged": bool(all(st == 0 for st in out.status)),
            "per_problem_time_to_tol_ms": {"median": round(float(np.median(tdone)), 3),
                                           "p90": round(float(np.percentile(tdone, 90)), 3),
                                           "max": round(float(tdone.max()), 3)},
            "per_size": per_size, "max_rho": float(max(out.rho)),
            "sequential_refined_ms": round(seq_ref * 1e3, 3), "sequential_plain_c128_ms": round(seq_plain * 1e3, 3),
            "speedup_vs_sequential_plain": round(seq_plain * 1e3 / out.elapsed_ms, 2)}


def bench_krylov(args, can128, log):
    """Krylov drivers on the same preconditioned operator (complex128, 256^3, tol as the
    main solve): BiCGSTAB (true residual checked every 5), GMRES(20), GMRES(5), beside the
    plain complex128 fixed point (the headline alpha) -- the comparison of Table 1b."""
    import torch
    from paper_2207_14222_amd import solver
    op = solver.Operator(can128.symbol, can128.B)
    y = can128.y
    N = y.numel()
    out = {}
    runs = [("bicgstab", dict(method="bicgstab", check_every=5)), ("gmres20", dict(method="gmres", restart=20)),
            ("gmres5", dict(method="gmres", restart=5))]
    for name, kw in runs:
        op.krylov(y, tol=args.tol, maxit=3000, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.krylov(y, tol=args.tol, maxit=3000, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        applies = 2 * r.iterations if name == "bicgstab" else r.iterations
        out[name] = {"time_ms": round(dt * 1e3, 2), "iterations": r.iterations, "operator_applications": applies,
                     "status": r.status_name, "rho": float(r.hist_true[-1, 1]),
                     "ms_per_iteration": round(dt * 1e3 / max(1, r.iterations), 4)}
        if name == "bicgstab":
            # 43 arrays per iteration: two applications of P (13 + 14) and three vector updates (4 + 6 + 6)
            out[name]["GB/s_per_iter"] = round(43 * N * 16 * r.iterations / dt / 1e9, 1)
        log(f"krylov {name}: {out[name]}")
    op.solve(y, alpha=args.alpha, tol=args.tol, maxit=20000, check_every=args.check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.solve(y, alpha=args.alpha, tol=args.tol, maxit=20000, check_every=args.check_every)
    torch.cuda.synchronize()
    out["fixed_point_c128"] = {"time_ms": round((time.perf_counter() - t0) * 1e3, 2), "iterations": r.iterations,
                               "operator_applications": r.iterations, "status": r.status_name}
    op.close()
    return out


def bench_pantograph(args, log):
    """Pantograph (complex128, single workgroup): the direct canonical form and the
    antisymmetrised one on the accretive case (lam 0.5, b 5, N = 1024; tol 1e-9), and
    the antisymmetrised one on the non-accretive case (lam 0.9, a 0.1, b -5), where the
    direct form diverges: tol 1e-8 on a window of 256 samples (the paper reports below
    1e-8 in 125 iterations) and of 1024 samples; derivative symbol with the Nyquist
    mode kept for the antisymmetrised non-accretive runs.  Times include the whole
    solve in one launch."""
    import torch
    from paper_2207_14222_amd import media, solver
    out = {}

    def run(pp, antisym, alpha, tol, maxit, check, nyquist_zero=True):
        can = solver.canonical_pantograph(pp.a, pp.b, pp.lam, pp.t0, pp.h, pp.x0_at_lam_t, pp.x0_t0,
                                          nyquist_zero=nyquist_zero)
        op = solver.Operator(can.symbol, can.B, gather=can.gather, antisym=antisym)
        y = torch.stack([torch.zeros_like(can.y), can.y]).contiguous() if antisym else can.y
        op.solve(y, alpha=alpha, tol=tol, maxit=maxit, check_every=check)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.solve(y, alpha=alpha, tol=tol, maxit=maxit, check_every=check)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"n": int(pp.a.shape[0]), "alpha": alpha, "time_ms": round(dt * 1e3, 3), "iterations": r.iterations,
                "status": r.status_name, "rho": float(r.hist_true[-1, 1]) if len(r.hist_true) else None,
                "us_per_iteration": round(dt * 1e6 / max(1, r.iterations), 2)}

    acc = media.pantograph(n=1024, b_value=5.0)
    out["accretive_direct"] = run(acc, False, 0.9, 1e-9, 20000, 1)
    out["accretive_antisym"] = run(acc, True, 1.0, 1e-9, 200000, 100)
    non = media.pantograph_constant(n=256)
    out["nonaccretive_direct"] = run(non, False, 0.8, 1e-8, 2000, 1)
    out["nonaccretive_antisym"] = run(non, True, 0.8, 1e-8, 5000, 1, nyquist_zero=False)
    non1024 = media.pantograph_constant(n=1024)
    out["nonaccretive_antisym_n1024"] = run(non1024, True, 0.7, 1e-8, 20000, 1, nyquist_zero=False)
    log(f"pantograph: {out}")
    return out


def _flux_refined(p, tol, k, maxit):
    """Refined flux-form solve (complex64 inner iterations, FP64 residual and
    update every k) from x = 0 at alpha = 1 to tol; one untimed run first."""
    import torch
    from paper_2207_14222_amd import solver
    op = solver.FluxOperator(p.mu, p.D, p.source, p.h, refine=True)
    op.solve(alpha=1.0, tol=tol, maxit=maxit, check_every=k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.solve(alpha=1.0, tol=tol, maxit=maxit, check_every=k)
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t0
    rho = op.residual(r.x)
    del op
    torch.cuda.empty_cache()
    return {"time_ms": round(dtm * 1e3, 2), "iterations": r.iterations, "status": r.status_name,
            "cycles": int(r.hist_true.shape[0]), "rho": rho, "refine_every": k}


def bench_flux(args, log):
    """Steady anisotropic diffusion in flux form (Sec. 3.2) on the 256 x 256 ring:
    complex128 and complex64 solves from x = 0 at alpha = 1 to ||r||/||y|| < 1e-3
    (the tolerance of Table 1) and complex128 to 1e-6, the FP64 residual checked
    every 10 iterations, and the refined solve (complex64 inner iterations, FP64
    refinement) to 1e-6.  Bytes per iteration (two launches): the column pass
    reads and writes the 3 planes of t (6 N values); the row pass reads t, x,
    y, b_u, b2 (3+3+3+1+4 N) and writes x and t (6 N)."""
    import torch
    from paper_2207_14222_amd import media, solver
    p = media.diffusion_ring(n=256)
    n = p.mu.size
    out = {}
    for dname, dt, es in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        op = solver.FluxOperator(p.mu, p.D, p.source, p.h, dtype=dt)
        iter_bytes = (6 + 20) * n * es
        for tol in ((1e-3, 1e-6) if dname == "c128" else (1e-3,)):
            op.solve(alpha=1.0, tol=tol, maxit=20000, check_every=10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = op.solve(alpha=1.0, tol=tol, maxit=20000, check_every=10)
            torch.cuda.synchronize()
            dtm = time.perf_counter() - t0
            # iteration cost without the residual checks
            K = 200
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            op.iterate(alpha=1.0, K=K)
            torch.cuda.synchronize()
            us_it = (time.perf_counter() - t1) * 1e6 / K
            out[f"{dname}_tol{tol:g}"] = {
                "time_ms": round(dtm * 1e3, 3), "iterations": r.iterations, "status": r.status_name,
                "rho": float(r.hist_true[-1, 1]), "us_per_iteration": round(us_it, 2),
                "model_GB/s_per_iter": round(iter_bytes / (us_it * 1e-6) / 1e9, 1)}
        del op
    out["refined_tol1e-06"] = _flux_refined(p, 1e-6, args.refine_every, 20000)
    log(f"flux-form diffusion: {out}")
    return out


def bench_flux3d(args, log):
    """Steady anisotropic diffusion in flux form in 3-D (four components [u; Jx;
    Jy; Jz]) on a 128^3 random tensor medium (media.diffusion_tensor_random3,
    seed 7): complex128 solve from x = 0 at alpha = 1 to 1e-6, FP64 residual
    every 20 iterations, the refined solve (complex64 inner iterations, FP64
    refinement) to 1e-6, and the iteration time without checks for complex128
    and complex64.  Bytes per iteration (four launches): the two middle-axis
    passes and the axis-0 pass read and write the 4 planes of t (3 x 8 N
    values); the row pass reads t, x, y (3 x 4 N), b_u (N) and b2 (9 N) and
    writes x and t (8 N): 54 N values."""
    import torch
    from paper_2207_14222_amd import media, solver
    p = media.diffusion_tensor_random3(shape=(128, 128, 128), seed=7, h=0.3)
    n = p.mu.size
    out = {"grid": [128, 128, 128]}
    for dname, dt, es in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        op = solver.FluxOperator(p.mu, p.D, p.source, p.h, dtype=dt)
        iter_bytes = 54 * n * es
        rec = {}
        if dname == "c128":
            op.solve(alpha=1.0, tol=1e-6, maxit=5000, check_every=20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = op.solve(alpha=1.0, tol=1e-6, maxit=5000, check_every=20)
            torch.cuda.synchronize()
            rec.update({"time_ms": round((time.perf_counter() - t0) * 1e3, 2), "iterations": r.iterations,
                        "status": r.status_name, "rho": float(r.hist_true[-1, 1])})
        K = 50
        op.iterate(alpha=1.0, K=5)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        op.iterate(alpha=1.0, K=K)
        torch.cuda.synchronize()
        us_it = (time.perf_counter() - t1) * 1e6 / K
        rec.update({"us_per_iteration": round(us_it, 1),
                    "model_GB/s_per_iter": round(iter_bytes / (us_it * 1e-6) / 1e9, 1)})
        out[dname] = rec
        del op
        torch.cuda.empty_cache()
    out["refined"] = _flux_refined(p, 1e-6, args.refine_every, 5000)
    log(f"flux-form diffusion 3-D: {out}")
    return out


def bench_eigen(args, log):
    """Five lowest modes of the double-ring well (Sec. 4, Eq. schrodinger) on a
    512 x 512 grid, complex128: H + 5 in canonical form, shift-invert Lanczos
    (24 basis vectors, thick restart) with CG inner solves on the preconditioned
    system to 1e-11, Ritz residual 1e-8.  Bytes per CG iteration: k_cg_first reads
    r, p, B and writes p, t (5 arrays), the symbol pass reads and writes t (2),
    k_klast reads t, p, B and writes q (4), k_cg_update reads x, r, p, q and
    writes x, r (6): 17 arrays of N complex128 values."""
    import torch
    from paper_2207_14222_amd import media, solver
    V, h = media.double_ring_well(n=512)
    shift = 5.0
    can = solver.canonical_schrodinger(V, (h, h), shift, dtype=torch.complex128)
    op = solver.Operator(can.symbol, can.B)
    kw = dict(nev=5, ncv=24, tol=1e-8, inner_tol=1e-11, max_restarts=30)
    op.eigs(**kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.eigs(**kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = V.size
    cg_bytes = 17 * n * 16
    energies = (np.real(can.c) * r.evals - shift).tolist()
    out = {"time_ms": round(dt * 1e3, 2), "status": "converged" if r.converged else "maxit",
           "restarts": r.restarts, "cg_iterations": r.inner_iterations,
           "us_per_cg_iteration": round(dt * 1e6 / max(1, r.inner_iterations), 2),
           "model_GB/s_per_cg_iter": round(cg_bytes * r.inner_iterations / dt / 1e9, 1),
           "energies": [round(e, 8) for e in energies], "max_resid": float(np.max(r.resid))}
    op.close()
    log(f"eigenmodes: {out}")
    return out


def bench_learned(args, log):
    """Learned initial guess on 128^3 random-sphere media (shared canonical scaling):
    training data from solves of the method (seeds 0..), Adam training of the
    3-D network, then on held-out media (seeds 10000..) the solve from x0 = 0
    against network inference + residual check + solve from the learned x0,
    and the plain complex128 solve."""
    import torch
    from paper_2207_14222_amd import learned, surrogate
    res, net, _ = learned.run((128, 128, 128), n_train=args.learned_train, n_test=args.learned_test,
                              epochs=args.learned_epochs, lr=2e-3, log=log)
    # GB/s per inner iteration of the refined solver at 128^3 (12 complex64 arrays per iteration)
    wl = learned.Workload((128, 128, 128))
    nre = next(wl.index_maps([10000]))
    op, y = wl.operator(nre)
    r = wl.solve(op, y)
    _, it_ms = op.profile(y, r.x, alpha=wl.alpha, K=50)
    res["ms_per_iter"] = it_ms
    res["GB/s_per_iter"] = 12 * y.numel() * 8 / (it_ms * 1e-3) / 1e9
    op.close()
    # network forward alone: executed matrix-core flops (padded channels) per launch sequence
    flops = 0
    for name, cin, cout, taps in surrogate.LAYERS:
        d, h, w = net.levels[net._level(name)]
        flops += 2 * d * h * w * taps * cin * cout
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.forward()
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    res["forward_ms"] = round(fwd_ms, 3)
    res["forward_TFLOP/s"] = round(flops / (fwd_ms * 1e-3) / 1e12, 1)
    res["forward_frac_bf16_peak"] = round(flops / (fwd_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4)
    res["forward_flops"] = flops
    def rnd(d):
        for k, v in list(d.items()):
            if isinstance(v, float):
                d[k] = float(f"{v:.5g}")
            elif isinstance(v, dict):
                rnd(v)
    rnd(res)
    log(f"learned x0: {res}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shape", default="256,256,256")
    ap.add_argument("--alpha", type=float, default=0.9, help="step size of the headline and comparison solves")
    ap.add_argument("--batch-alpha", type=float, default=0.9, help="step size of the batched 2-D problems")
    ap.add_argument("--batch-refine-every", type=int, default=150,
                    help="refinement interval of the batched schedule and of its one-at-a-time refined comparison")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--refine-every", type=int, default=100,
                    help="refinement interval of the headline solve (its last cycle is shortened to the predicted "
                         "crossing of tol)")
    ap.add_argument("--check-every", type=int, default=20,
                    help="residual check interval of the plain and Krylov comparisons")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the plain complex128/complex64 reference solves")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch plan")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 2-D workload")
    ap.add_argument("--batch-variant", type=int, default=None,
                    help="batched schedule variant (bits 0-1 fused-pass plan, bit 2 persistent); default: autotuned")
    ap.add_argument("--batch-only", action="store_true",
                    help="profiling aid: run only the batched workload's autotuned solve (no headline line)")
    ap.add_argument("--batch-n", type=int, default=96)
    ap.add_argument("--batch-side", type=int, default=0,
                    help="profiling aid: every batched problem of this side instead of the drawn sizes")
    ap.add_argument("--batch-maxit", type=int, default=20000,
                    help="profiling aid: iteration cap of the batched solve (a cap below the iterations to "
                         "tolerance keeps every problem in every launch)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-initial-guess workload")
    ap.add_argument("--no-flux", action="store_true", help="skip the flux-form tensor diffusion workload")
    ap.add_argument("--no-eigen", action="store_true", help="skip the eigenmode workload")
    ap.add_argument("--learned-train", type=int, default=2000, help="training media (the protocol's 2000)")
    ap.add_argument("--learned-test", type=int, default=200, help="held-out media (the protocol's 200)")
    ap.add_argument("--learned-epochs", type=int, default=4)
    ap.add_argument("--plan", default=None,
                    help="force a launch plan 'x_prefetch,w_mid,w_sym,x_stream[,r_load]' (no tuning)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); no multi-GPU path is built "
              "(independent problems and slabs of one grid would shard across GPUs, but that is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    from paper_2207_14222_amd import media, solver

    if args.batch_only:
        out = bench_batch(args, log, sequential=False)
        print(json.dumps({"batched": out}), flush=True)
        return

    shape = tuple(int(s) for s in args.shape.split(","))
    N = int(np.prod(shape))
    log(f"media {shape}")
    prob = media.helmholtz_spheres(shape=shape, seed=2)
    log("canonical form (library)")
    can128 = solver.canonical_helmholtz(prob.k2, prob.source, prob.spacing, dtype=torch.complex128)
    op_ref = solver.Operator(can128.symbol, can128.B, refine=True)
    y = can128.y
    x = torch.zeros_like(y)
    torch.cuda.synchronize()

    def refined_solve():
        return op_ref.solve(y, alpha=args.alpha, tol=args.tol, maxit=20000, check_every=args.refine_every)

    # measured streaming copy bandwidth (read + write bytes) with the library's
    # non-temporal copy kernel, the practical streaming ceiling beside the 8 TB/s peak
    a = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    solver.stream_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncopy = 5 if args.copy_probe else 4
    e0.record()
    for _ in range(ncopy):
        solver.stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 8 * ncopy / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert torch.equal(a, b)
    del a, b
    log(f"copy: {ncopy} x 1 GiB streaming copy kernel, {copy_gbs:.0f} GB/s (read + write)")
    for w in range(args.warmup):
        r = refined_solve()
        log(f"warmup {w + 1}/{args.warmup}: {r.iterations} iterations, status {r.status_name}")
    plan = op_ref.get_plan()
    if args.plan:
        op_ref.set_plan(*[int(v) for v in args.plan.split(",")])
        plan = op_ref.get_plan()
        log(f"plan {plan}")
    elif not args.no_tune:
        r = refined_solve()   # workspace holds a valid inner problem for tuning
        plan = op_ref.autotune(y, x, alpha=args.alpha, reps=5)
        log(f"autotuned plan {plan}")
    times = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = refined_solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {k + 1}/{args.steps}: {times[-1] * 1e3:.1f} ms, {r.iterations} iterations, "
            f"rho {r.hist_true[-1, 1]:.3e}, status {r.status_name}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    t_step = total / args.steps
    iters = r.iterations
    converged = r.converged

    # per-pass timing of the inner complex64 iterations (and one FP64 residual)
    log("per-pass timing")
    pass_ms, iter_ms = op_ref.profile(y, x, alpha=args.alpha, K=50)
    nd = len(shape)
    s64 = 8
    # algorithmic bytes per launch (complex64 inner iteration; FP64 residual passes)
    pass_bytes = {"x_fused": 6 * N * s64, "m_fwd": 2 * N * s64, "sym": 2 * N * s64, "m_inv": 2 * N * s64,
                  "x_first": 2 * N * s64, "r_fwd": 2 * N * 16, "r_mfwd": 2 * N * 16,
                  "r_sym": 2 * N * 16, "r_minv": 2 * N * 16, "r_inv": 4 * N * 16 + N * 8, "reduce": 0}
    iter_bytes = (4 * nd + 2 - 2) * N * s64 if nd >= 2 else 4 * N * s64   # 12 arrays (3-D), 8 (2-D)
    per_iter_kernels = ["x_fused", "sym"] + (["m_fwd", "m_inv"] if nd == 3 else [])
    dom = max(per_iter_kernels, key=lambda k: pass_ms[k])
    ach = pass_bytes[dom] / (pass_ms[dom] * 1e-3) / 1e9
    traffic = recorded_traffic(plan, shape) if dom == "x_fused" else None
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_launch_us": round(pass_ms[dom] * 1e3, 2),
                "bytes_per_launch": pass_bytes[dom]}
    gbs_iter = iter_bytes / (iter_ms * 1e-3) / 1e9
    passes = {k: {"avg_us": round(v * 1e3, 2),
                  "GB/s": round(pass_bytes[k] / (v * 1e-3) / 1e9, 1) if pass_bytes[k] else None}
              for k, v in pass_ms.items() if v > 0}

    extra = {}
    if not args.no_extra:
        log("plain complex128 solve")
        op128 = solver.Operator(can128.symbol, can128.B)
        r128 = op128.solve(y, alpha=args.alpha, tol=args.tol, maxit=20000, check_every=args.check_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r128 = op128.solve(y, alpha=args.alpha, tol=args.tol, maxit=20000, check_every=args.check_every)
        torch.cuda.synchronize()
        t128 = time.perf_counter() - t0
        pm128, it128 = op128.profile(y, r128.x.clone(), alpha=args.alpha, K=20)
        extra["plain_c128"] = {"time_s": round(t128, 4), "iterations": r128.iterations,
                               "status": r128.status_name, "ms_per_iter": round(it128, 4),
                               "GB/s_per_iter": round(2 * iter_bytes / (it128 * 1e-3) / 1e9, 1)}
        del op128, r128
        log("plain complex64 solve (attainable residual)")
        can64 = solver.canonical_helmholtz(prob.k2, prob.source, prob.spacing, dtype=torch.complex64)
        op64 = solver.Operator(can64.symbol, can64.B)
        r64 = op64.solve(can64.y, alpha=args.alpha, tol=args.tol, maxit=6000, check_every=args.check_every)
        extra["plain_c64"] = {"iterations": r64.iterations, "status": r64.status_name,
                              "min_rho": float(np.min(r64.hist_true[:, 1])),
                              "reaches_tol": bool(r64.converged)}
        del op64, r64, can64
        torch.cuda.empty_cache()

    if not args.no_extra:
        log("Krylov drivers (complex128)")
        extra["krylov_c128"] = bench_krylov(args, can128, log)
        torch.cuda.empty_cache()

    if not args.no_extra:
        log("pantograph: direct and antisymmetrised forms")
        extra["pantograph"] = bench_pantograph(args, log)

    if not args.no_extra:
        log("1-D workload (N = 256, complex128, tol 1e-10)")
        extra["config1_1d"] = bench_config1(args, log)

    if not args.no_extra:
        log("diffusion workload")
        extra["diffusion"] = bench_diffusion(args, log)
        torch.cuda.empty_cache()

    if not args.no_flux:
        log("flux-form tensor diffusion (256 x 256 ring)")
        extra["flux_ring256"] = bench_flux(args, log)
        torch.cuda.empty_cache()

    if not args.no_flux:
        log("flux-form tensor diffusion in 3-D (128^3)")
        extra["flux3d_128"] = bench_flux3d(args, log)
        torch.cuda.empty_cache()

    if not args.no_eigen:
        log("eigenmodes of the double-ring well (512 x 512)")
        extra["eigen_ring512"] = bench_eigen(args, log)
        torch.cuda.empty_cache()

    if not args.no_batch:
        log("batched 2-D workload")
        extra["batched"] = bench_batch(args, log)
        torch.cuda.empty_cache()

    if not args.no_learned:
        log("learned initial guess workload (128^3)")
        extra["learned_x0"] = bench_learned(args, log)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        cpu = cpu_baseline(prob, iters, n_iter=args.cpu_iters)

    out = {
        "metric": METRIC,
        "value": round(t_step, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "helmholtz3d_spheres_256" if shape == (256, 256, 256) else
                   "helmholtz3d_spheres_" + "x".join(map(str, shape)),
                   "grid": list(shape), "alpha": args.alpha, "tol": args.tol,
                   "refine_every": args.refine_every, "iterations": iters, "converged": converged,
                   "plan": plan,
                   "mode": "complex64 iterations + FP64 residual refinement"},
        "GB/s_per_iter": round(gbs_iter, 1),
        "copy_GB/s": round(copy_gbs, 1),
        "ms_per_iter": round(iter_ms, 4),
        "iter_model_bytes": iter_bytes,
        "roofline": roofline,
        "passes": passes,
        "modes": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

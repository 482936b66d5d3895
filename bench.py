"""Benchmark of the implicit-MPM hot path on one MI355X.

Workload (default): the 3-D footing cube, 128^3 cells of 1/128 m with the
soil in the lower half on 2x2x2 Gauss points (8,388,608 particles), Hencky +
Drucker-Prager (E = 50 MPa, nu = 0.25, friction uniform in [25, 35] deg per
particle, c = 0, psi = 0), its geostatic load step (gravity).  A step is one
load step: binning and pattern, Newton iterations (residual, Jacobian,
multigrid-preconditioned BiCGStab) to 1e-10, and the particle update; the
input state is kept, so every step repeats it.  --workload c2 runs the
plane-strain footing (256 x 128 cells, 131,072 particles) instead.

Prints one JSON line: the metric is the residual + Jacobian assembly rate
(Mparticles/s); it also carries ms per Newton iteration, the roofline of the
BSR SpMV (the HBM-bound product of the Krylov solve, timed with HIP events
on the library's stream), with the cube the plane-strain footing's figures
under "c2", the batched-vs-sequential comparison and the CPU oracle timed on
a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KRYLOV_NAMES = {0: "block-Jacobi BiCGStab, GMRES(100) fallback", 1: "block-Jacobi GMRES(100)",
                2: "BiCGStab preconditioned by a geometric multigrid V-cycle, GMRES(100) fallback"}


def spmv_bytes(n_row, nnzb, bs):
    """Algorithmic HBM bytes of one BSR SpMV: values + column indices + row
    pointers + one read of x and one write of y."""
    return nnzb * (bs * bs * 8 + 4) + 4 * (n_row + 1) + 2 * n_row * bs * 8


PMC_PROFILES = {"c2": "k_spmv_c2_geostatic_pmc.md", "c3": "k_spmv_c3_cube_pmc.md"}


def spmv_traffic(lanes, workload):
    """HBM bytes per SpMV launch with this many lanes per row on the
    workload's matrix, from the committed counter passes
    (profiles/k_spmv_<workload>_pmc.md), or None when the kernel's source has
    changed since they were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", PMC_PROFILES[workload])
    src = os.path.join(ROOT, "paper_2507_09435_amd", "csrc", "mpm_krylov.hip")
    try:
        text = open(prof).read()
        code = open(src).read()
    except OSError:
        return None
    i = code.find("template <int BS, int LPR, bool TR>")
    j = code.find("// ---------------------------------------------------------- BiCGStab")
    fields = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_", "kernel_")))
    if i < 0 or j < 0 or fields.get("kernel_source_sha1", "").strip() != hashlib.sha1(code[i:j].encode()).hexdigest():
        return None
    key = f"traffic_bytes_per_launch_lanes{lanes}"
    return int(float(fields[key])) if key in fields else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="with the cube: skip the plane-strain footing key")
    ap.add_argument("--krylov-rtol", type=float, default=1e-12)
    ap.add_argument("--krylov-method", type=int, default=None,
                    help="0 block-Jacobi BiCGStab (GMRES fallback), 1 GMRES, 2 multigrid-preconditioned BiCGStab "
                         "(default: the faster on the workload, 0 for c3, 2 for c2)")
    ap.add_argument("--batch-sims", type=int, default=64,
                    help="sims of the batched footing set timed batched and one at a time (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=2, help="load steps of that comparison (incl. geostatic)")
    ap.add_argument("--c5-full", action="store_true",
                    help="only the batched footing set with its adjoint gradient checked by central differences")
    ap.add_argument("--c5-sims", type=int, default=64)
    ap.add_argument("--c5-steps", type=int, default=30)
    ap.add_argument("--c5-fd-steps", type=int, default=10)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only the SpMV launches and a plain copy of known size, for counter passes")
    ap.add_argument("--workload", choices=["c3", "c2"], default="c3",
                    help="c3: the 128^3 footing cube (default); c2: the 256x128 plane-strain footing")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the chip's reachable peaks: HBM copy and triad bandwidth (torch), FP64 "
                         "DGEMM throughput (the vendor BLAS on the FP64 matrix cores); one JSON line")
    ap.add_argument("--c3-probe", action="store_true",
                    help="the 128^3 footing cube: one residual, one Jacobian and timed BSR SpMV launches "
                         "(the HBM-bound regime of the SpMV), one JSON line")
    args = ap.parse_args()
    if args.krylov_method is None:
        # measured on one MI355X: on the cube the multigrid cuts BiCGStab
        # iterations ~6x, but each V-cycle streams the 10 GB fine matrix seven
        # times, so block-Jacobi solves a load step in about half the time;
        # on the plane-strain footing the multigrid is several times faster
        args.krylov_method = 0 if args.workload == "c3" else 2
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU layout is a design "
                                   "(domain slabs with halo exchange), not an implementation"}))
        sys.exit(2)

    import torch

    from paper_2507_09435_amd import mpm as M
    from paper_2507_09435_amd import workloads as W

    if args.pmc_probe:
        pmc_probe(M, W, torch, args.workload)
        return
    if args.c5_full:
        print(json.dumps(c5_full(M, W, torch, args)))
        return
    if args.c3_probe:
        print(json.dumps(c3_probe(M, W, torch)))
        return
    if args.peaks:
        print(json.dumps(peak_probe(torch)))
        return

    if args.workload == "c3":
        w = W.make_c3(n_steps=1)
        label = ("3D footing cube, 128^3 cells (h=1/128 m), soil in the lower half on 2x2x2 Gauss points, "
                 "8388608 particles, Hencky + Drucker-Prager, E=5e7 Pa, nu=0.25, friction U[25,35] deg per "
                 "particle (seed 1003), c=0, geostatic load step")
    else:
        w = W.make_c2(n_steps=1)
        label = ("2D plane-strain Drucker-Prager soil layer of the footing problem, 256x128 cells (h=1/256 m), "
                 "131072 particles, E=1e7 Pa, nu=0.3, friction 30 deg, c=0, geostatic load step")
    P = w.prob
    npart = w.particles.np
    react = np.zeros((P.n_nodes, P.ndof), dtype=np.uint8)
    react[w.footing_nodes(), P.dim - 1] = 1
    stream = torch.cuda.current_stream()
    ctx = M.mpm_create(0, stream.cuda_stream)
    dp = M.make_problem([(P, w.particles)], [w.bc(0)], react_masks=[react])
    print(f"[bench] {args.workload}: {npart} particles on the device", file=sys.stderr, flush=True)
    x_out = torch.empty_like(dp.tensors["x"])
    F_out = torch.empty_like(dp.tensors["F"])
    be_out = torch.empty_like(dp.tensors["be"])

    def load_step(step):
        # one pass of the whole path: binning + pattern, Newton (residual,
        # Jacobian, preconditioned BiCGStab), end-of-step particle update; the
        # input state is left untouched so every step repeats the same work
        n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
        du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
        rep = M.mpm_newton_step(ctx, dp, du, tol=w.tol, max_iter=25, commit=False, krylov_rtol=args.krylov_rtol,
                                time_spmv=4, krylov_method=args.krylov_method)
        M.mpm_update(ctx, dp, du, x_out, F_out, be_out)
        print(f"[bench] step {step}: newton {rep['iters']} krylov {rep['krylov']} "
              f"{rep['ms_total']:.1f} ms (residual {rep['ms_residual']:.1f}, jacobian {rep['ms_jacobian']:.1f}, "
              f"krylov {rep['ms_krylov']:.1f})", file=sys.stderr, flush=True)
        return rep, (n_row, nnzb, nd), du

    for step in range(args.warmup):
        load_step(step)
    torch.cuda.synchronize()

    reps = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        rep, shape, du = load_step(args.warmup + k)
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_res = sum(r["iters"] + 1 for r in reps)
    n_jac = sum(r["iters"] for r in reps)
    ms_res = sum(r["ms_residual"] for r in reps)
    ms_jac = sum(r["ms_jacobian"] for r in reps)
    ms_kry = sum(r["ms_krylov"] for r in reps)
    t_asm_ms = ms_res / n_res + ms_jac / max(n_jac, 1)
    value = npart / (t_asm_ms * 1e-3) / 1e6
    newton_ms = sum(r["ms_total"] for r in reps) / max(n_jac, 1)

    # roofline kernel: the BSR SpMV of the Krylov loop, the path's HBM-bound
    # kernel (the multigrid sweeps take more of the time, bound by launch
    # latency on the coarse levels).  Its average duration is taken with HIP
    # events on the library's stream around 200 back-to-back launches of the
    # same kernel doing the same work as inside BiCGStab (product plus the
    # fused z.y and y.y partial sums) on the converged Jacobian; a sample of
    # in-loop launches is reported beside it.
    n_row, nnzb, nd = shape
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, du, val=val)
    xv = torch.randn(n_row * nd, dtype=torch.float64, device="cuda")
    zv = torch.randn_like(xv)
    yv = torch.empty_like(xv)
    # the autotuner's launch shape for this pattern, then every shape pinned in
    # turn (the same arithmetic): 200 timed launches each after 10 untimed
    lanes = M.mpm_spmv_lanes(ctx)
    nrep = 200
    by_shape = {}
    for lpr in (4, 8, 16):
        M.mpm_spmv_set_lanes(ctx, lpr)
        for _ in range(10):
            M.mpm_spmv(ctx, val, xv, yv, zv)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(nrep):
            M.mpm_spmv(ctx, val, xv, yv, zv)
        e1.record(stream)
        e1.synchronize()
        by_shape[lpr] = e0.elapsed_time(e1) * 1e3 / nrep
    M.mpm_spmv_set_lanes(ctx, 0)
    spmv_us = by_shape[lanes]
    # the matrix-free product on the same tangent tables (reused from the
    # assembly above), same x: the operator a matrix-free Krylov loop applies
    njv = 20 if args.workload == "c3" else 200
    for _ in range(3):
        M.mpm_jv(ctx, dp, None, xv, yv, reuse=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(njv):
        M.mpm_jv(ctx, dp, None, xv, yv, reuse=True)
    e1.record(stream)
    e1.synchronize()
    jv_us = e0.elapsed_time(e1) * 1e3 / njv
    loop_ms = sum(r["spmv_ms"] for r in reps)
    loop_n = sum(r["spmv_launches"] for r in reps)
    nbytes = spmv_bytes(n_row, nnzb, nd)
    achieved = nbytes / (spmv_us * 1e-6) / 1e9

    out = {
        "metric": "Jacobian+residual assembly Mparticles/s",
        "value": round(value, 3),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": label,
                   "particles": npart, "rows": n_row, "bsr_blocks": nnzb, "block": nd,
                   "newton_tol": w.tol, "krylov": KRYLOV_NAMES[args.krylov_method],
                   "krylov_rtol": args.krylov_rtol},
        "newton_step_ms": round(newton_ms, 3),
        "newton_iters_per_step": [r["iters"] for r in reps],
        "krylov_iters_per_step": [r["krylov_iters"] for r in reps],
        "ms_residual_per_eval": round(ms_res / n_res, 4),
        "ms_jacobian_per_eval": round(ms_jac / max(n_jac, 1), 4),
        "ms_krylov_per_newton_iter": round(ms_kry / max(n_jac, 1), 3),
        "roofline": {"kernel": f"k_spmv<{nd},{lanes}> (BSR SpMV in the Krylov loop, lanes per row from the "
                               f"autotuner)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": spmv_traffic(lanes, args.workload),
                     "avg_launch_us": round(spmv_us, 3), "timed_launches": nrep,
                     "avg_launch_us_by_lanes_per_row": {str(k): round(v, 3) for k, v in by_shape.items()},
                     "in_loop_event_us": round(loop_ms * 1e3 / max(loop_n, 1), 3),
                     "algorithmic_bytes_per_launch": nbytes},
        "assembly_roofline": assembly_roofline(npart, nd, ms_jac / max(n_jac, 1), args.workload),
        "matrix_free_jv": {"avg_us": round(jv_us, 3), "timed_calls": njv,
                           "vs_bsr_spmv": round(spmv_us / jv_us, 3),
                           "note": "y = J x from the per-particle tangent tables (no matrix), Dirichlet-modified"},
    }
    if args.workload == "c3" and not args.no_c2:
        M.mpm_destroy(ctx)
        del dp, val, xv, zv, yv
        torch.cuda.empty_cache()
        ctx = M.mpm_create(0, stream.cuda_stream)
        out["c2"] = c2_extra(M, W, torch, ctx, stream, args)
    if args.batch_sims > 0:
        # the plane-strain footings of the batched set: multigrid-preconditioned BiCGStab
        out["batched"] = batched_vs_sequential(ctx, args.batch_sims, args.batch_steps, args.krylov_rtol, 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload)
    M.mpm_destroy(ctx)
    print(json.dumps(out))


FP64_PEAK_TFLOPS = 78.6


def jacobian_source_sha1():
    """SHA-1 of the source the 3-D Jacobian kernels are built from (None if unreadable)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2507_09435_amd", "csrc")
    try:
        code = open(os.path.join(csrc, "mpm_assemble.hip")).read()
        dev = open(os.path.join(csrc, "mpm_device.hpp")).read()
    except OSError:
        return None
    j = code.find("// The FG3 consecutive stencil groups")
    if j < 0:
        return None
    return hashlib.sha1((code[:j] + dev).encode()).hexdigest()


def jacobian_traffic(workload):
    """HBM bytes per 3-D Jacobian evaluation on the cube (its three kernels),
    from the committed counter passes (profiles/k_jac3_cube_pmc.md), or None
    for another workload or when the kernels' source has changed since: the
    device code of mpm_assemble.hip up to the residual's kernels, and the
    constitutive code of mpm_device.hpp."""
    if workload != "c3":
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", "k_jac3_cube_pmc.md")).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_", "jacobian_source_sha1")))
    if fields.get("jacobian_source_sha1", "").strip() != jacobian_source_sha1():
        return None
    v = fields.get("traffic_bytes_per_jacobian")
    return int(float(v)) if v else None


def assembly_roofline(npart, nd, ms_jac, workload):
    """The Jacobian evaluation against the FP64 peak: the local-block
    contraction of each particle, K_ab = sum_ij g_ai T_(r i)(c j) g_bj over
    its 3^d x 3^d node pairs and nd^2 entries with d FMAs each once the
    row side T g_a is formed (2 flop per FMA), per measured evaluation in
    the Newton loop (tangent tables, stencil data and the block sweep).
    traffic: counted HBM bytes of one evaluation, where measured."""
    nn = 3 ** nd
    flop = 2.0 * nn * nn * nd * nd * nd
    achieved = npart * flop / (ms_jac * 1e-3) / 1e12
    return {"kernels": "Jacobian evaluation (increment gradients, tangent tables, block sweep)", "bound": "alu",
            "flop_per_particle": flop, "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": jacobian_traffic(workload)}


def c2_extra(M, W, torch, ctx, stream, args, steps=5, warmup=1):
    """The plane-strain footing (256 x 128 cells, 131,072 particles) beside
    the cube: its geostatic load step with multigrid-preconditioned BiCGStab
    (assembly rate, ms per Newton iteration and per load step) and its SpMV
    (200 back-to-back launches of the autotuner's shape)."""
    w = W.make_c2(n_steps=1)
    P = w.prob
    react = np.zeros((P.n_nodes, P.ndof), dtype=np.uint8)
    react[w.footing_nodes(), P.dim - 1] = 1
    dp = M.make_problem([(P, w.particles)], [w.bc(0)], react_masks=[react])
    x_out = torch.empty_like(dp.tensors["x"])
    F_out = torch.empty_like(dp.tensors["F"])
    be_out = torch.empty_like(dp.tensors["be"])
    reps = []
    torch.cuda.synchronize()
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
        du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
        rep = M.mpm_newton_step(ctx, dp, du, tol=w.tol, max_iter=25, commit=False, krylov_rtol=args.krylov_rtol,
                                krylov_method=2)
        M.mpm_update(ctx, dp, du, x_out, F_out, be_out)
        if k >= warmup:
            reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_res = sum(r["iters"] + 1 for r in reps)
    n_jac = sum(r["iters"] for r in reps)
    t_asm_ms = sum(r["ms_residual"] for r in reps) / n_res + sum(r["ms_jacobian"] for r in reps) / n_jac
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, du, val=val)
    xv = torch.randn(n_row * nd, dtype=torch.float64, device="cuda")
    zv = torch.randn_like(xv)
    yv = torch.empty_like(xv)
    for _ in range(10):
        M.mpm_spmv(ctx, val, xv, yv, zv)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(200):
        M.mpm_spmv(ctx, val, xv, yv, zv)
    e1.record(stream)
    e1.synchronize()
    spmv_us = e0.elapsed_time(e1) * 1e3 / 200
    lanes = M.mpm_spmv_lanes(ctx)
    achieved = spmv_bytes(n_row, nnzb, nd) / (spmv_us * 1e-6) / 1e9
    print(f"[bench] c2: {w.particles.np / t_asm_ms / 1e3:.1f} Mparticles/s, "
          f"{sum(r['ms_total'] for r in reps) / n_jac:.2f} ms per Newton iteration", file=sys.stderr, flush=True)
    return {"workload": "2D plane-strain Drucker-Prager footing layer, 256x128 cells, 131072 particles, geostatic "
                        "load step, multigrid-preconditioned BiCGStab",
            "assembly_mparticles_per_s": round(w.particles.np / t_asm_ms / 1e3, 3),
            "ms_residual_per_eval": round(sum(r["ms_residual"] for r in reps) / n_res, 4),
            "ms_jacobian_per_eval": round(sum(r["ms_jacobian"] for r in reps) / n_jac, 4),
            "newton_step_ms": round(sum(r["ms_total"] for r in reps) / n_jac, 3),
            "ms_per_load_step": round(wall * 1e3 / steps, 3),
            "spmv": {"kernel": f"k_spmv<{nd},{lanes}>", "avg_launch_us": round(spmv_us, 3),
                     "achieved_GBps": round(achieved, 1), "frac_of_hbm_peak": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": spmv_traffic(lanes, "c2")}}


def batched_vs_sequential(ctx, nsims, nsteps, krylov_rtol, krylov_method):
    """Newton iterations per second summed over sims: the first nsims
    footings of the batched set (uneven sizes, E and friction per sim; the
    gradient reading of the footing) solved as one batch, against the same
    sims solved one at a time, same steps and tolerances."""
    import torch
    from paper_2507_09435_amd import adjoint as AD
    from paper_2507_09435_amd import workloads as W
    sims, _ = W.make_c5(nsim=64)
    sims = sims[:nsims]
    E = [float(w.particles.E[0]) for w in sims]
    phi = [float(w.particles.phi[0]) for w in sims]
    steps = list(range(nsteps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dp = AD.make_batch(sims, E, phi)
    run = AD.forward(ctx, dp, sims, steps, krylov_rtol=krylov_rtol, krylov_method=krylov_method, line_search=4,
                     max_iter=50)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    print(f"[bench] batched {nsims} sims x {nsteps} steps: {t_b:.2f} s, newton {run.newton_iters}",
          file=sys.stderr, flush=True)
    iters = 0
    t0 = time.perf_counter()
    for k, w in enumerate(sims):
        d1 = AD.make_batch([w], [E[k]], [phi[k]])
        r1 = AD.forward(ctx, d1, [w], steps, krylov_rtol=krylov_rtol, krylov_method=krylov_method, line_search=4,
                        max_iter=50)
        iters += sum(r1.newton_iters)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    print(f"[bench] sequential: {t_s:.2f} s, {iters} Newton iterations", file=sys.stderr, flush=True)
    particles = sum(w.particles.np for w in sims)
    return {"sims": nsims, "load_steps": nsteps, "particles": particles, "krylov": KRYLOV_NAMES[krylov_method],
            "newton_iters": iters, "batched_s": round(t_b, 3), "sequential_s": round(t_s, 3),
            "newton_iters_per_s_batched": round(iters / t_b, 2),
            "newton_iters_per_s_sequential": round(iters / t_s, 2),
            "speedup": round(t_s / t_b, 3),
            "note": "the same Newton iterations counted on both sides: the sum over sims of each sim's own "
                    "iterations when solved alone"}


def c5_full(M, W, torch, args):
    """The batched footing set at full size: every sim's load steps in one
    batch, the squared misfit of each sim's footing reaction curve against
    the curve of its target (E, friction), and its gradient with respect to
    (E, friction) from the step adjoints behind torch.autograd.  The gradient
    is checked against central differences of the same losses over the first
    --c5-fd-steps steps (all sims perturbed at once: they are independent)."""
    from paper_2507_09435_amd import adjoint as AD
    sims, targets = W.make_c5(nsim=args.c5_sims, n_steps=args.c5_steps)
    ctx = M.mpm_create(0, torch.cuda.current_stream().cuda_stream)

    def progress(step, rep):
        print(f"[c5]   step {step}: newton {rep['iters']} krylov {rep['krylov_iters']} {rep['ms_total']:.0f} ms",
              file=sys.stderr, flush=True)

    def adjoint_progress(step, kit):
        print(f"[c5]   adjoint step {step}: krylov max {max(kit)}", file=sys.stderr, flush=True)

    # backtracking line search: cone/elastic switching can make full Newton steps cycle
    # Newton to 1e-12, stopping at the round-off floor only within 100x of it:
    # central differences with a 1e-5 relative perturbation magnify a
    # residual left at ||r|| / ||r_0|| = e into an error of about e / 1e-5
    opts = dict(tol=1e-12, stall_factor=100.0, krylov_rtol=1e-12, max_iter=50, krylov_method=2, line_search=4,
                progress=progress, adjoint_progress=adjoint_progress)
    E0 = torch.tensor([float(w.particles.E[0]) for w in sims], dtype=torch.float64)
    phi0 = torch.tensor([float(w.particles.phi[0]) for w in sims], dtype=torch.float64)
    Et = torch.tensor([t[0] for t in targets], dtype=torch.float64)
    phit = torch.tensor([t[1] for t in targets], dtype=torch.float64)

    def timed(f, label):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        print(f"[c5] {label}: {dt:.2f} s", file=sys.stderr, flush=True)
        return out, dt

    def gradient(nsteps, label):
        curves = AD.ReactionCurves(ctx, sims, list(range(nsteps + 1)), **opts)
        with torch.no_grad():
            Rt, _ = timed(lambda: curves(Et, phit), f"{label} target curves")
        E = E0.clone().requires_grad_(True)
        phi = phi0.clone().requires_grad_(True)
        R, t_f = timed(lambda: curves(E, phi), f"{label} forward")
        per_sim = ((R - Rt) ** 2).sum(dim=0)
        reached = max(curves.last_run.newton_rel)
        _, t_b = timed(lambda: per_sim.sum().backward(), f"{label} backward")
        return curves, Rt, E.grad.detach(), phi.grad.detach(), t_f, t_b, float(per_sim.sum()), reached

    _, _, _, _, t_fwd, t_bwd, loss_total, reached_full = gradient(args.c5_steps, "full")
    curves, Rt, gE, gphi, _, _, _, reached_fd = gradient(args.c5_fd_steps, "fd horizon")

    def loss(Ev, pv, label):
        with torch.no_grad():
            Rv, _ = timed(lambda: curves(Ev, pv), label)
            return ((Rv - Rt) ** 2).sum(dim=0)

    dE, dphi = 1e-5, 1e-5
    fd_E = (loss(E0 * (1 + dE), phi0, "E+") - loss(E0 * (1 - dE), phi0, "E-")) / (2 * dE * E0)
    fd_phi = (loss(E0, phi0 + dphi, "phi+") - loss(E0, phi0 - dphi, "phi-")) / (2 * dphi)

    def rel(a, b):
        a, b = a.numpy(), b.numpy()
        return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)

    eE, ep = rel(gE, fd_E), rel(gphi, fd_phi)
    M.mpm_destroy(ctx)
    return {"mode": "batched footing set, forward + adjoint gradient", "sims": len(sims),
            "load_steps": args.c5_steps + 1, "particles": sum(w.particles.np for w in sims),
            "newton_tol": opts["tol"], "newton_stall_factor": opts["stall_factor"],
            "newton_reached_max": {"full": reached_full, "fd_horizon": reached_fd},
            "krylov": KRYLOV_NAMES[opts["krylov_method"]],
            "forward_s": round(t_fwd, 3), "backward_s": round(t_bwd, 3), "loss_total": loss_total,
            "grad_vs_central_fd": {"load_steps": args.c5_fd_steps + 1, "dE_rel": dE, "dphi_rad": dphi,
                                   "E_rel_err_max": float(eE.max()), "E_rel_err_median": float(np.median(eE)),
                                   "phi_rel_err_max": float(ep.max()), "phi_rel_err_median": float(np.median(ep)),
                                   "worst_E": {"sim": int(eE.argmax()), "adjoint": float(gE[eE.argmax()]),
                                               "fd": float(fd_E[eE.argmax()])},
                                   "worst_phi": {"sim": int(ep.argmax()), "adjoint": float(gphi[ep.argmax()]),
                                                 "fd": float(fd_phi[ep.argmax()])}}}


def c3_probe(M, W, torch):
    """The 3-D footing cube (128^3 cells, 8388608 particles, geostatic
    load): residual and Jacobian at du = 0 timed with HIP events, then 50
    back-to-back in-loop SpMV launches (product plus the fused partial dot
    products) on that Jacobian, timed the same way.  The 10.6 GB matrix
    streams from HBM on every launch."""
    w = W.make_c3()
    P = w.prob
    stream = torch.cuda.current_stream()
    ctx = M.mpm_create(0, stream.cuda_stream)
    dp = M.make_problem([(P, w.particles)], [w.bc(0)])
    t0 = time.perf_counter()
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    r = torch.zeros_like(du)
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    M.mpm_residual(ctx, dp, du, r)        # warm-up of both assemblies
    M.mpm_jacobian_bsr(ctx, dp, du, val=val)
    e[0].record(stream)
    M.mpm_residual(ctx, dp, du, r)
    e[1].record(stream)
    M.mpm_jacobian_bsr(ctx, dp, du, val=val)
    e[2].record(stream)
    xv = torch.randn(n_row * nd, dtype=torch.float64, device="cuda")
    zv = torch.randn_like(xv)
    yv = torch.empty_like(xv)
    for _ in range(5):
        M.mpm_spmv(ctx, val, xv, yv, zv)
    nrep = 50
    e[3].record(stream)
    for _ in range(nrep):
        M.mpm_spmv(ctx, val, xv, yv, zv)
    e[4].record(stream)
    e[4].synchronize()
    spmv_ms = e[3].elapsed_time(e[4]) / nrep
    lanes = M.mpm_spmv_lanes(ctx)
    nbytes = spmv_bytes(n_row, nnzb, nd)
    achieved = nbytes / (spmv_ms * 1e-3) / 1e9
    M.mpm_destroy(ctx)
    return {"workload": "3D footing cube 128^3 cells, 8388608 particles, friction U[25,35] deg per particle, "
                        "geostatic load, du = 0",
            "particles": w.particles.np, "rows": n_row, "bsr_blocks": nnzb, "block": nd,
            "prepare_s": round(t_prep, 3),
            "ms_residual": round(e[0].elapsed_time(e[1]), 3), "ms_jacobian": round(e[1].elapsed_time(e[2]), 3),
            "spmv": {"kernel": f"k_spmv<3,{lanes}>", "bound": "hbm", "avg_launch_ms": round(spmv_ms, 4),
                     "timed_launches": nrep, "algorithmic_bytes_per_launch": nbytes,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4)}}


def peak_probe(torch):
    """What the chip reaches outside this library, to set the measured
    kernels against: a device-to-device copy and a triad a = b + s c over
    2 GiB FP64 arrays (HBM bytes read + written per second), and an FP64
    matrix product of order 8192 (2 n^3 flop per second; the vendor BLAS
    runs it on the FP64 matrix cores, whose published peak equals the FP64
    vector peak on this chip)."""
    dev = "cuda"
    n = (2 << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.rand(n, dtype=torch.float64, device=dev)
    c = torch.rand(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_copy = timed(lambda: a.copy_(b), 20)
    t_triad = timed(lambda: torch.add(b, c, alpha=1.5, out=a), 20)
    m = 8192
    A = torch.rand(m, m, dtype=torch.float64, device=dev)
    B = torch.rand(m, m, dtype=torch.float64, device=dev)
    C = torch.empty(m, m, dtype=torch.float64, device=dev)
    t_gemm = timed(lambda: torch.matmul(A, B, out=C), 10)
    return {"probe": "peaks", "hbm_copy_GBps": round(2 * 8 * n / t_copy / 1e9, 1),
            "hbm_triad_GBps": round(3 * 8 * n / t_triad / 1e9, 1), "hbm_peak_GBps": HBM_PEAK_GBS,
            "dgemm_TFlops": round(2 * m ** 3 / t_gemm / 1e12, 2), "fp64_peak_TFlops": 78.6,
            "sizes": {"copy_triad_bytes_per_array": 8 * n, "dgemm_order": m}}


def pmc_probe(M, W, torch, workload):
    """For the counter passes: on the workload's geostatic state, one
    residual and one Jacobian (each of their kernels once), 20 SpMV launches
    per launch shape on that Jacobian, 5 matrix-free products, and a plain
    256 MiB copy (the scale of the HBM byte counters)."""
    w = W.make_c3(n_steps=1) if workload == "c3" else W.make_c2(n_steps=1)
    P = w.prob
    ctx = M.mpm_create(0, torch.cuda.current_stream().cuda_stream)
    dp = M.make_problem([(P, w.particles)], [w.bc(0)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    r = torch.zeros_like(du)
    M.mpm_residual(ctx, dp, du, r)
    M.mpm_jacobian_bsr(ctx, dp, du, val=val)
    xv = torch.randn(n_row * nd, dtype=torch.float64, device="cuda")
    zv = torch.randn_like(xv)
    yv = torch.empty_like(xv)
    for lanes in (4, 8, 16):   # every launch shape, 20 dispatches each (same arithmetic)
        M.mpm_spmv_set_lanes(ctx, lanes)
        for _ in range(20):
            M.mpm_spmv(ctx, val, xv, yv, zv)
    M.mpm_spmv_set_lanes(ctx, 0)
    for _ in range(5):
        M.mpm_jv(ctx, dp, None, xv, yv, reuse=True)
    a = torch.randn(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    M.mpm_destroy(ctx)
    print(json.dumps({"pmc_probe": workload, "particles": w.particles.np, "rows": n_row, "bsr_blocks": nnzb,
                      "spmv_algorithmic_bytes": spmv_bytes(n_row, nnzb, nd),
                      "copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))


def cpu_baseline(w, workload, budget_s=12.0):
    """The oracle as it stands: residual + dual-number Jacobian at the
    workload's initial state on the host cores (both OpenMP over particles),
    repeated until about budget_s seconds of work; the rate is the mean over
    the repetitions.  The 3-D cube is sampled: its first 32768 particles in
    input order (the bottom 128 x 32 x 1 cells)."""
    from oracle import oracle as O
    P, st = w.prob, w.particles
    note = f"the full {st.np}-particle workload"
    if workload == "c3":
        n = 32768
        st = W_sub(st, n)
        note = f"the first {n} particles of the cube (cells 128 x 32 x 1 at the base)"
    pat = O.pattern(P, st)
    rng = np.random.default_rng(0)
    dof = np.zeros((P.n_nodes, P.ndof))
    dof[pat.active] = rng.normal(size=(pat.n_row, P.ndof)) * 1e-4 * P.h
    t_res = t_jac = 0.0
    reps = 0
    while reps < 200 and t_res + t_jac < budget_s:
        t0 = time.perf_counter()
        O.forces(P, st, dof)
        t1 = time.perf_counter()
        O.jacobian_bsr(P, st, dof, pat)
        t2 = time.perf_counter()
        t_res += t1 - t0
        t_jac += t2 - t1
        reps += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(reps * st.np / (t_res + t_jac) / 1e6, 4), "unit": "Mparticles/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} repetitions of one residual + one Jacobian (both OpenMP, {threads} threads) of "
                      f"{note}: {t_res:.2f} s + {t_jac:.2f} s"}


def W_sub(st, n):
    """The first n particles of a particle set (a view copy of every array)."""
    from paper_2507_09435_amd import workloads as W
    cut = lambda a: None if a is None else np.ascontiguousarray(a[..., :n])
    return W.Particles(cut(st.x), cut(st.vol0), cut(st.F), cut(st.be), cut(st.fp), cut(st.E), cut(st.phi))


if __name__ == "__main__":
    main()

"""Benchmark: cell-steps/s of the immersed-boundary time step at Poisson
(divergence) residual 1e-6 on one MI355X.

Workload (default): 256^3 uniform cells, 40 seeded overlapping ellipsoids
(semi-axes 4-20 cells, ~2k triangles each, 3% gaps) plus 5 thin plates, inflow
U = 1, Re = 1e4 on the mean ellipsoid diameter, CSM on, CFL 0.3.  A step is one
pass of the whole hot path on this input: eddy viscosity, predictor, face
velocity and right-hand side, pressure solve to relative residual 1e-6,
projection, FP64 divergence check and surface force.  Tagging and the stencil
build happen once per geometry before the timed region (reported as setup).

Prints ONE JSON line.  `python bench.py --gpus N` with N > 1 exits: the library and
this benchmark run on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s at div residual 1e-6: mixed+learned vs plain FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell of the two fused conjugate-gradient passes (FP64
# vectors, 1-byte pressure code): A reads z, d, x, code and writes x, d; B reads d, r,
# code and writes r, z
SWEEP_BYTES = {"pcg_a": 41, "pcg_b": 33, "unused": 0}
SWEEP_NAMES = ("pcg_a", "pcg_b", "unused")
# kernel names of the double2 passes (grids with an even cell count in x; the scalar
# passes k_pcg_a / k_pcg_b serve odd nx)
# FP32 vectors of the mixed correction solve: A reads z, d, x (4 B), code; writes x, d.
# B reads d, r, code; writes r, z
SWEEP_BYTES_F32 = {"pcg_a": 21, "pcg_b": 17, "unused": 0}
KERNEL_SYMBOL = {"pcg_a": "k_pcg_a_v<double, false>", "pcg_b": "k_pcg_b_v<double>", "unused": ""}
# the FP32 correction sweeps of the mixed solve (nx divisible by 4)
KERNEL_SYMBOL_F32 = {"pcg_a": "k_pcg_a_f4<false>", "pcg_b": "k_pcg_b_f4", "unused": ""}
# algorithmic FLOPs of one network application per cell: 2 * 27 * (16 + 256 + 256 + 16)
CNN_FLOP_PER_CELL = 29376
# Whole-step model (algorithmic bytes of the kernels a step runs, per cell; the same
# per-kernel figures as the roofline records): the eddy viscosity, predictor,
# right-hand side and projection sweeps (FP64 fields: 33 + 129 + 57 + 105 B; FP32
# fields: 17 + 77 + 45 + 81 B), the FP64 divergence check (U read, 24 B) and the choice
# of the pressure guess (2 p - p_prev formed 24 B, two residual passes 17 B each, the
# pick 32 B); per solver iteration the two CG passes (FP64 41 + 33 B, FP32 21 + 17 B; the
# learned FCG 21 + 13 B plus the network application, 38 + 66 + 45 B and 29,376 FLOP,
# and with the smoothing steps around it the pre-smoothing pass (r and code read, r1
# written: 9 B) and the post-smoothing pass (z2, r, r_prev, code read, z written: 17 B));
# per FP64 refinement sweep of the mixed paths the residual and the accumulation (45 B).
STEP_BYTES_FIXED = {"f64": 33 + 129 + 57 + 105 + 24, "f32": 17 + 77 + 45 + 81 + 24}
GUESS_BYTES = 24 + 17 + 17 + 32
ITER_BYTES = {"pcg_fp64": 41 + 33, "mixed": 21 + 17, "mixed_learned": 21 + 13 + 38 + 66 + 45}
SMOOTH_BYTES = 9 + 17
REFINE_BYTES = 45
BF16_PEAK_TFLOPS = 2500.0
# dominant kernel of the learned preconditioner: the fused forward half y = K x (the
# gated 1 -> 16 layer recomputed on the halo region in LDS, then the 16 -> 16 layer):
# 2*27*16 (W1) + 2*27*16 (gate) + 2*27*16*16 (W2) FLOP per cell (algorithmic: no halo
# recompute, no padding); reads r (4 B) and the geometry input (2 B), writes y (32 B)
CONV_KERNEL = "k_mfwd<true>"
CONV_NAME = "fused_forward"
CONV_FLOP_PER_CELL = 2 * 27 * 16 + 2 * 27 * 16 + 2 * 27 * 16 * 16
CONV_BYTES_PER_CELL = 38


def workload(name):
    from paper_2002_06206_amd import inputs
    if name == "ellipsoids256":
        return inputs.case_ellipsoids256(0)
    if name == "dirty_sphere128":
        return inputs.case_dirty_sphere128(0)
    if name == "sphere32":
        return inputs.case_sphere32(0)
    if name == "plate256":
        return inputs.case_plate256(0)
    if name == "vehicle1024":
        # 1024^3 cells, ~1M-triangle vehicle-like assembly, dead-end filter on; run as
        #   python bench.py --workload vehicle1024 --steps 2 --warmup 1 --no-cpu-baseline
        return inputs.case_vehicle(1024, 0)
    raise SystemExit("unknown workload %s" % name)


def kernel_source_hash():
    """Hash of the sources of every kernel with a committed counter summary."""
    h = hashlib.sha256()
    for f in ("poisson.hip", "cnn.hip", "common.h", "momentum.hip", "shepard.hip", "step.hip", "bcm.hip"):
        with open(os.path.join(ROOT, "paper_2002_06206_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, wl):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, when it was
    taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel, wl))
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if line.startswith("{"):
            try:
                d = json.loads(line)
            except ValueError:
                return None
            if d.get("source_sha256") == kernel_source_hash():
                return d.get("hbm_bytes_per_launch")
    return None


CPU_PCG_ITERS = 50


def cpu_worker(workload_name, n_pcg):
    """One oracle process (one thread) on the workload: set-up untimed, then one FP64
    time step's eddy viscosity, predictor, face velocity + right-hand side and
    projection timed in full, and n_pcg conjugate-gradient iterations of its pressure
    solve timed.  Prints one JSON line."""
    import numpy as np

    from oracle import flow, tagging
    case = workload(workload_name)
    g = flow.Grid(case.n, case.dx, case.origin, case.bc, case.u_in)
    b, th = tagging.tag(case.tri, case.n, case.dx, case.origin)
    st = flow.build_stencils(g, b, th, case.deadend)
    u, U, p, h = flow.init_state(st, case.u_in)
    t0 = time.perf_counter()
    nut = flow.csm_nut(st, u) if case.csm else np.zeros(g.shape)
    us, H = flow.predictor(st, u, U, h, nut, case.nu, case.dt, (0.0, 0.0, 0.0), 0, None)
    Us = flow.face_predicted(st, us, None)
    rhs = flow.poisson_rhs(st, Us, case.dt)
    t1 = time.perf_counter()
    x, it = flow.pcg(st, rhs, p, 1e-30, n_pcg)
    t2 = time.perf_counter()
    flow.project(st, us, Us, x, case.dt)
    t3 = time.perf_counter()
    print(json.dumps({"t_fixed": (t1 - t0) + (t3 - t2), "t_pcg": t2 - t1, "pcg_iters": int(it),
                      "cells": g.ncell}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_samples(workload_name, workers, n_pcg=CPU_PCG_ITERS):
    """Runs `workers` oracle processes at once, one thread each (the host's cores), each
    on its own copy of the workload; started before this process touches the GPU.
    Returns their measurements and the wall time of the whole sample."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, "-c", "import bench; bench.cpu_worker(%r, %d)" % (workload_name, n_pcg)]
    t0 = time.perf_counter()
    procs = [subprocess.Popen(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for _ in range(workers)]
    res = []
    for pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            raise SystemExit("cpu baseline worker failed (rc %d): %s" % (pr.returncode, err[-2000:]))
        res.append(json.loads(out.strip().splitlines()[-1]))
    return res, time.perf_counter() - t0


def cpu_baseline(case, samples, wall_s, gpu_iters_per_step):
    """The oracle on all host cores: P concurrent single-thread oracle processes, each
    solving its own copy of the same workload (independent problems, so the job's
    throughput is P cells x steps over the time of one step).  Per process, the
    non-solver parts of a step are measured in full and CPU_PCG_ITERS conjugate-gradient
    iterations are measured; the remaining iterations of the step (the GPU plain solve's
    count per step, same algorithm and stopping rule) are extrapolated at the measured
    rate.  The slowest process sets the step time."""
    P = len(samples)
    N = samples[0]["cells"]
    t_fixed = max(r["t_fixed"] for r in samples)
    t_iter = max(r["t_pcg"] / max(r["pcg_iters"], 1) for r in samples)
    t_step = t_fixed + gpu_iters_per_step * t_iter
    one = samples[0]
    t_one = one["t_fixed"] + gpu_iters_per_step * one["t_pcg"] / max(one["pcg_iters"], 1)
    return {
        "value": float(P * N / t_step),
        "unit": "cell-steps/s",
        "cores": P,
        "kind": "oracle",
        "sample": ("%d concurrent 1-thread numpy oracle processes, one %dx%dx%d step each: CSM, predictor, RHS, "
                   "projection measured (%.1f s); %d PCG iterations measured (%.2f s each), the other %.0f of the "
                   "step extrapolated" % (P, case.n[0], case.n[1], case.n[2], t_fixed, samples[0]["pcg_iters"],
                                          t_iter, max(gpu_iters_per_step - samples[0]["pcg_iters"], 0))),
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
        "threads_per_process": 1,
        "single_process_value": float(N / t_one),
        "measured_pcg_iters": samples[0]["pcg_iters"],
        "extrapolated_pcg_iters": max(gpu_iters_per_step - samples[0]["pcg_iters"], 0.0),
        "sample_wall_s": round(wall_s, 1),
    }


def run_solver(case, solver, args, ibm, torch, weights=None):
    """Set-up, warm-up and timed steps of one solver configuration.  Returns a dict.
    weights: trained preconditioner weights for the learned solver."""
    N = case.n[0] * case.n[1] * case.n[2]
    precision = ibm.FP64 if solver == "pcg_fp64" else ibm.MIXED
    kind = {"pcg_fp64": ibm.SOLVER_PCG_JACOBI, "mixed": ibm.SOLVER_FCG_JACOBI,
            "mixed_learned": ibm.SOLVER_FCG_CNN}[solver]
    t0 = time.perf_counter()
    s = ibm.Solver(case.n, case.dx, case.origin, case.bc, case.u_in, precision)
    blocked, _ = s.tag(case.tri, want_theta=False)
    s.build(blocked, None, case.deadend)
    net = None
    if solver == "mixed_learned":
        net = ibm.Network(N, weights, inference_only=True)
        net.attach(s)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    st = s.new_state(case.u_in)
    # pressure history for the solve's initial guess (the better of p^n and
    # 2 p^n - p^{n-1}; at the first step p_prev = p, so the guess is p)
    p_prev = st["p"].clone() if args.p_guess == "extrapolate" else None
    # device memory in use with the context, the state (and the network) resident: the
    # whole device's figure after torch's cache is released, of which torch_live are
    # this process's live torch tensors (the state, the inputs)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free_b, total_b = torch.cuda.mem_get_info()
    torch_live_b = torch.cuda.memory_allocated()
    # time step: CFL 0.3 on the largest face velocity of the previous step, capped at
    # the configured dt (= CFL 0.3 on the inflow velocity); variable-step AB2
    ctl = {"dt_prev": 0.0, "umax": max(abs(v) for v in case.u_in)}

    def params(step, tol=None):
        dt = min(case.dt, 0.3 * case.dx / max(ctl["umax"], 1e-30))
        p = ibm.step_params(dt, case.nu, csm=case.csm, step=step, dt_prev=ctl["dt_prev"],
                            tol=args.tol if tol is None else tol,
                            max_iter=20000, check_every=16, kind=kind,
                            inner_tol=args.inner_tol_learned if solver == "mixed_learned" else args.inner_tol,
                            inner_max_iter=2000, inner_restart=args.inner_restart, p_prev=p_prev,
                            omega=args.smooth if solver == "mixed_learned" else 0.0)
        ctl["dt_prev"] = dt
        return p

    # progress lines on stderr for workloads whose steps take many seconds
    verbose = N >= 512 ** 3

    def progress(msg):
        if verbose:
            print("[bench] %s: %s (%.0f s)" % (solver, msg, time.perf_counter() - t0), file=sys.stderr, flush=True)

    progress("set-up done")
    cb = None
    if verbose:
        last = [time.perf_counter()]

        def on_poll(iters, rr):
            if rr < 0.0:   # an FP64 residual check of the mixed solve
                progress("FP64 relative residual %.3e after %d iterations" % (-rr, iters))
            elif time.perf_counter() - last[0] > 20.0:
                last[0] = time.perf_counter()
                progress("solving, %d iterations" % iters)
        cb = ibm.ibm_set_progress(s.ctx, on_poll)
    step = 0
    for _ in range(args.warmup):
        rc, stats = s.step(st, params(step, args.warmup_tol))
        ctl["umax"] = stats["umax"]
        step += 1
        progress("warm-up step %d: %d iterations" % (step, stats["iters_inner"]))
    ibm.ibm_timing_enable(s.ctx, True)
    ibm.ibm_timing_read(s.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, outers, fallbacks, fb_iters = [], [], 0, []
    worst_res = 0.0
    worst_div = 0.0
    forces = None
    for _ in range(args.steps):
        rc, stats = s.step(st, params(step))
        ctl["umax"] = stats["umax"]
        forces = s.forces(st, case.nu)
        step += 1
        iters.append(stats["iters_inner"])
        outers.append(stats["iters_outer"])
        fallbacks += stats["fallback_used"]
        fb_iters.append(stats["iters_fallback"])
        worst_res = max(worst_res, stats["rel_residual"])
        worst_div = max(worst_div, stats["div_linf"])
        progress("timed step %d: %d iterations" % (step, stats["iters_inner"]))
        if rc != 0:
            raise SystemExit("%s: step %d did not converge (rc=%d)" % (solver, step, rc))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pred = ibm.ibm_timing_slot(s.ctx, 9, reset=True)
    tim = ibm.ibm_timing_read(s.ctx, reset=True)
    ibm.ibm_timing_enable(s.ctx, False)
    if cb is not None:
        ibm.ibm_set_progress(s.ctx, None)
    elapsed = t1 - t0
    bytes_tab = SWEEP_BYTES if precision == ibm.FP64 else SWEEP_BYTES_F32
    k_dom = max(range(3), key=lambda k: tim["ms"][k])
    name = SWEEP_NAMES[k_dom]
    real = tim["real_iters"]
    avg_s = tim["ms"][k_dom] / 1e3 / max(real, 1)
    achieved = bytes_tab[name] * N / avg_s / 1e9
    Fp, Fv = forces
    # whole-step roofline: the step's algorithmic bytes (and the network's FLOPs) per cell
    # at the measured iterations, against 8 TB/s and 2.5 PFLOP/s
    it_step = sum(iters) / len(iters)
    sweeps = sum(outers) / len(outers)
    step_bytes = (STEP_BYTES_FIXED["f64" if precision == ibm.FP64 else "f32"]
                  + (GUESS_BYTES if p_prev is not None else 0)
                  + (ITER_BYTES[solver] + (SMOOTH_BYTES if solver == "mixed_learned" and args.smooth > 0 else 0))
                  * it_step
                  + (REFINE_BYTES * sweeps if solver != "pcg_fp64" else 0))
    step_flop = CNN_FLOP_PER_CELL * it_step if solver == "mixed_learned" else 0.0
    bound_value = min(HBM_PEAK_GBS * 1e9 / step_bytes,
                      BF16_PEAK_TFLOPS * 1e12 / step_flop if step_flop > 0 else float("inf"))
    value = N * args.steps / elapsed
    step_roofline = {"bytes_per_cell_step": round(step_bytes, 1), "flop_per_cell_step": round(step_flop, 1),
                     "bound": "hbm" if step_flop == 0 or step_bytes / (HBM_PEAK_GBS * 1e9) >= step_flop /
                     (BF16_PEAK_TFLOPS * 1e12) else "mfma",
                     "roofline_value": round(bound_value, 1), "frac": round(value / bound_value, 4)}
    out = {"solver": solver, "value": value, "ms_per_step": elapsed / args.steps * 1e3,
           "step_roofline": step_roofline,
           "iters_per_step": sum(iters) / len(iters), "refinement_sweeps_per_step": sum(outers) / len(outers),
           "fallbacks": fallbacks, "fp64_fallback_iters_per_step": sum(fb_iters) / len(fb_iters),
           "max_rel_residual": worst_res, "max_div_linf": worst_div,
           "setup_s": round(t_setup, 3), "cuts": s.ncut, "dt_last": ctl["dt_prev"],
           "device_gib_in_use": round((total_b - free_b) / 2 ** 30, 2),
           "torch_live_gib": round(torch_live_b / 2 ** 30, 2),
           "force_last_step": [a + b for a, b in zip(Fp, Fv)],
           "dominant": {"name": name, "kernel": (KERNEL_SYMBOL if precision == ibm.FP64 else KERNEL_SYMBOL_F32)[name],
                        "bytes_per_cell": bytes_tab[name], "avg_s": avg_s, "achieved_gbs": achieved,
                        "launches": tim["launches"][k_dom], "launches_with_work": real,
                        "sweeps_ms": {SWEEP_NAMES[k]: round(tim["ms"][k], 2) for k in range(3)}}}
    if solver == args.solver:
        out["surface_force"] = shepard_timing(case, s, st, torch)
    if solver == "pcg_fp64":
        out["predictor"] = predictor_record(case, pred, "central")
        if args.quick_steps > 0:
            out["hybrid_quick"] = quick_timing(case, s, st, ctl, step, args, ibm, torch)
            step += 2 + args.quick_steps
    if solver == "pcg_fp64" and args.bcm:
        out["building_cubes"] = bcm_timing(case, blocked, args, ibm, torch)
    if solver == "pcg_fp64" and args.sor:
        out["red_black_sor"] = sor_timing(case, s, args, ibm, torch)
    if solver == "pcg_fp64" and args.cn_steps > 0:
        out["crank_nicolson"] = cn_timing(case, s, st, ctl, step, args, ibm, torch)
    if solver == "mixed_learned":
        # slot 0: whole preconditioner applications (three marching MFMA kernels and the
        # relay of the dot products); slot 1: the fused FCG passes; slot 2: the dominant
        # kernel (fused forward half)
        apply_s = tim["ms"][0] / 1e3 / max(real, 1)
        conv_s = tim["ms"][2] / 1e3 / max(real, 1)
        out["cnn"] = {"flop_per_cell": CNN_FLOP_PER_CELL, "avg_apply_us": round(apply_s * 1e6, 2),
                      "apply_tflops": round(CNN_FLOP_PER_CELL * N / apply_s / 1e12, 2),
                      "fcg_passes_ms": round(tim["ms"][1], 2)}
        out["dominant"] = {"name": CONV_NAME, "kernel": CONV_KERNEL, "bound": "mfma",
                           "flop_per_launch": CONV_FLOP_PER_CELL * N, "bytes_per_cell": CONV_BYTES_PER_CELL,
                           "avg_s": conv_s, "achieved_tflops": CONV_FLOP_PER_CELL * N / conv_s / 1e12,
                           "achieved_gbs": CONV_BYTES_PER_CELL * N / conv_s / 1e9,
                           "launches": tim["launches"][2], "launches_with_work": real,
                           "sweeps_ms": {"preconditioner": round(tim["ms"][0], 2), "fcg_passes": round(tim["ms"][1], 2),
                                         CONV_NAME: round(tim["ms"][2], 2)}}
        net.close()
    s.close()
    torch.cuda.synchronize()
    return out


# near-field surface force (eq. (force)): per triangle 72 B of vertices read, 16 B of
# front/back pressure written and 24 pressure gathers of 8 B (no reuse counted)
SHEPARD_BYTES_PER_TRIANGLE = 72 + 16 + 24 * 8


def shepard_timing(case, s, st, torch, calls=20):
    """Times ibm_shepard_force on the workload's triangles and the final pressure of the
    run, without and with the thin-plate filter Z (the filtered call includes building
    its triangle bins): whole calls (kernels, block-partial sum, copy of the three
    doubles to the host; each call synchronises), host clock."""
    tri = torch.as_tensor(case.tri, dtype=torch.float64).cuda().contiguous()
    side = torch.empty((tri.shape[0], 2), dtype=torch.float64, device="cuda")
    ntri = int(tri.shape[0])
    out = {"triangles": ntri, "bytes_per_triangle": SHEPARD_BYTES_PER_TRIANGLE}
    for key, flt in (("", False), ("filtered_", True)):
        for _ in range(3):
            s.shepard_force(tri, st["p"], side, flt)
        t0 = time.perf_counter()
        for _ in range(calls):
            f = s.shepard_force(tri, st["p"], side, flt)
        per = (time.perf_counter() - t0) / calls
        out[key + "us_per_call"] = round(per * 1e6, 2)
        out[key + "pressure_force"] = f
    out["achieved_gbs_per_call"] = round(SHEPARD_BYTES_PER_TRIANGLE * ntri / (out["us_per_call"] * 1e-6) / 1e9, 1)
    return out


# momentum predictor, FP64 (timing slot 9 brackets both of its parts: the plain sweep
# k_predict_fast<double, 2> over the cells without a blocked or domain face and the
# per-cell form k_fix<PredictOp<double>> over the others; with the hybrid QUICK face
# value the per-cell form k_all<PredictOp<double>> covers every cell): reads u, U, H^{n-1}
# (24 B each), nu_t (8 B) and the mask, writes u* and H (24 B each)
PREDICT_BYTES_PER_CELL = 129


def predictor_record(case, slot, face):
    N = case.n[0] * case.n[1] * case.n[2]
    ms, launches = slot
    avg = ms / 1e3 / max(launches, 1)
    kern = ("k_predict_fast<double, 2> + k_fix<PredictOp<double>>" if face == "central"
            else "k_all<PredictOp<double>>")
    return {"kernel": kern, "face_value": face, "launches": launches,
            "avg_launch_us": round(avg * 1e6, 2), "bytes_per_cell": PREDICT_BYTES_PER_CELL,
            "achieved_gbs": round(PREDICT_BYTES_PER_CELL * N / avg / 1e9, 1) if avg > 0 else None,
            "frac": round(PREDICT_BYTES_PER_CELL * N / avg / 1e9 / HBM_PEAK_GBS, 4) if avg > 0 else None}


def quick_timing(case, s, st, ctl, step, args, ibm, torch):
    """The hybrid face value of Sec. 3 (central blended with args.quick of QUICK) on the
    developed plain FP64 state, explicit scheme at the benchmark's CFL 0.3: whole steps
    by the host clock and the predictor kernel by dispatch events (slot 9)."""
    N = case.n[0] * case.n[1] * case.n[2]

    def prm(k):
        dt = min(case.dt, 0.3 * case.dx / max(ctl["umax"], 1e-30))
        p = ibm.step_params(dt, case.nu, csm=case.csm, step=k, dt_prev=ctl["dt_prev"], tol=args.tol, max_iter=20000,
                            check_every=16, quick=args.quick)
        ctl["dt_prev"] = dt
        return p
    for _ in range(2):
        rc, stats = s.step(st, prm(step))
        ctl["umax"] = stats["umax"]
        step += 1
    ibm.ibm_timing_enable(s.ctx, True)
    ibm.ibm_timing_read(s.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.quick_steps):
        rc, stats = s.step(st, prm(step))
        if rc != 0:
            raise SystemExit("hybrid QUICK step did not converge (rc=%d)" % rc)
        ctl["umax"] = stats["umax"]
        step += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pred = ibm.ibm_timing_slot(s.ctx, 9, reset=True)
    ibm.ibm_timing_read(s.ctx, reset=True)
    ibm.ibm_timing_enable(s.ctx, False)
    rec = predictor_record(case, pred, "central + %g QUICK" % args.quick)
    return {"weight": args.quick, "steps": args.quick_steps, "ms_per_step": round(elapsed / args.quick_steps * 1e3, 2),
            "value": N * args.quick_steps / elapsed, "predictor": rec,
            "roofline": {"bound": "hbm", "achieved": rec["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": rec["frac"], "traffic": committed_traffic("predict", args.workload),
                         "kernel": rec["kernel"], "algorithmic_bytes_per_launch": PREDICT_BYTES_PER_CELL * N,
                         "avg_launch_us": rec["avg_launch_us"]}}


# one red-black SOR half sweep (one colour): x read at every cell (8 B), b and the
# code byte at the cells of the colour (4 + 0.5 B), x written there (4 B)
SOR_BYTES_PER_CELL = 16.5


def sor_timing(case, s, args, ibm, torch):
    """Red-black SOR (Sec. 2.1) against the plain FP64 PCG on the same right-hand side
    (the last step's compatible b), both from x = 0 to the benchmark tolerance: whole
    solves by the host clock, the half sweeps by dispatch events (slot 0)."""
    N = case.n[0] * case.n[1] * case.n[2]
    b = s.rhs()
    out = {}
    for name, kw in (("pcg_fp64", dict(kind=ibm.SOLVER_PCG_JACOBI)),
                     ("rbsor", dict(kind=ibm.SOLVER_RBSOR, omega=args.sor_omega))):
        x = torch.zeros_like(b)
        ibm.ibm_timing_enable(s.ctx, True)
        ibm.ibm_timing_read(s.ctx, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, stats = s.poisson(b, x, tol=args.tol, max_iter=200000, check_every=16, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tim = ibm.ibm_timing_read(s.ctx, reset=True)
        ibm.ibm_timing_enable(s.ctx, False)
        rec = {"rc": rc, "iterations": stats["iters_inner"], "ms": round(el * 1e3, 2),
               "rel_residual": stats["rel_residual"]}
        if name == "rbsor":
            half = tim["ms"][0] / 1e3 / max(tim["launches"][0], 1)
            rec.update({"omega": args.sor_omega if args.sor_omega > 0 else "2/(1+sin(pi/n))",
                        "kernel": "k_sor", "half_sweep_us": round(half * 1e6, 2),
                        "bytes_per_cell": SOR_BYTES_PER_CELL,
                        "achieved_gbs": round(SOR_BYTES_PER_CELL * N / half / 1e9, 1) if half > 0 else None})
            rec["roofline"] = {"bound": "hbm", "achieved": rec["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(rec["achieved_gbs"] / HBM_PEAK_GBS, 4) if rec["achieved_gbs"] else None,
                               "traffic": committed_traffic("sor_half_sweep", args.workload), "kernel": "k_sor",
                               "algorithmic_bytes_per_launch": SOR_BYTES_PER_CELL * N,
                               "avg_launch_us": rec["half_sweep_us"]}
        out[name] = rec
    return out


def bcm_solve_timing(G, case, n, ibm, torch):
    """The pressure solve on the cubes (ibm_bcm_solve) with the geometry set: b = L u for
    a smooth u sampled at the cube cell centres (a consistent right-hand side), from
    x = 0 to a relative residual of 1e-6, by BiCGStab and by red-black SOR (capped at 4,000
    sweeps), timed by the host clock (the call synchronises)."""
    L = [case.n[a] * case.dx for a in range(3)]
    org = torch.from_numpy(G.origins).cuda().to(torch.float64)            # fine-cell units
    w = torch.where(torch.from_numpy(G.levels).cuda() == 1, 1.0, 2.0).to(torch.float64)
    ar = torch.arange(n, dtype=torch.float64, device="cuda") + 0.5
    side = n + 4
    u = torch.zeros(G.size, dtype=torch.float64, device="cuda")
    ui = u.view(G.ncubes, side, side, side)[:, 2:2 + n, 2:2 + n, 2:2 + n]
    fine_dx = 0.5 * 2.0 * case.dx
    xc = case.origin[0] + (org[:, 0, None] + ar[None, :] * w[:, None]) * fine_dx
    yc = case.origin[1] + (org[:, 1, None] + ar[None, :] * w[:, None]) * fine_dx
    zc = case.origin[2] + (org[:, 2, None] + ar[None, :] * w[:, None]) * fine_dx
    ui.copy_(torch.sin(3.0 * xc[:, None, None, :] / L[0]) * torch.cos(2.0 * yc[:, None, :, None] / L[1])
             + 0.5 * zc[:, :, None, None] / L[2])
    G.exchange(u)
    b = torch.zeros_like(u)
    G.laplacian(u, b)
    out = {}
    for name, kw in (("bicgstab", dict(kind=ibm.BCM_BICGSTAB, max_iter=20000, check_every=16)),
                     ("rbsor", dict(kind=ibm.BCM_SOR, omega=1.95, max_iter=4000, check_every=100))):
        x = torch.zeros_like(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, it, rel = G.solve(b, x, tol=1e-6, **kw)
        el = time.perf_counter() - t0
        out[name] = {"rc": rc, "iterations": it, "ms": round(el * 1e3, 2), "rel_residual": rel,
                     "us_per_iteration": round(el * 1e6 / max(it, 1), 1)}
    return out


def bcm_timing(case, blocked, args, ibm, torch, reps=20):
    """The building-cube grid (Sec. 2.2) over the workload's domain: coarse cubes of 16^3
    cells of twice the workload's cell size, refined (8 cubes of 16^3 cells at the
    workload's cell size) wherever the geometry cuts a grid line inside them; the halo
    exchange, the 7-point operator and red-black SOR sweeps (two exchanges and two half
    sweeps each) timed with events on the stream they run on; then the operator and the
    sweeps again with the workload's geometry on both levels (ibm_bcm_set_blocked), and the
    pressure solve on the cubes with that geometry (bcm_solve_timing)."""
    n = 16
    N = case.n
    if any(v % (2 * n) for v in N):
        return None
    K = tuple(v // (2 * n) for v in N)
    b = blocked.reshape(N[2], N[1], N[0]).to(torch.bool)
    refine = b.reshape(K[2], 2 * n, K[1], 2 * n, K[0], 2 * n).any(dim=5).any(dim=3).any(dim=1).cpu().numpy()
    G = ibm.BCM(K, n, 2.0 * case.dx, case.origin, refine)
    x = torch.randn(G.size, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    for _ in range(3):
        G.exchange(x)
        G.laplacian(x, y)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        G.exchange(x)
    ev[1].record()
    for _ in range(reps):
        G.laplacian(x, y)
    ev[2].record()
    ev.append(torch.cuda.Event(enable_timing=True))
    G.sor(y, x, 1.8, reps)
    ev[3].record()
    torch.cuda.synchronize()
    ex_us = ev[0].elapsed_time(ev[1]) / reps * 1e3
    lap_us = ev[1].elapsed_time(ev[2]) / reps * 1e3
    sor_us = ev[2].elapsed_time(ev[3]) / reps * 1e3
    # immersed geometry on the cubes: level 1 takes the workload's own tagging, level 0 a
    # tagging of the same triangles on the grid of twice the cell size
    coarse = ibm.Solver(tuple(v // 2 for v in N), 2.0 * case.dx, case.origin, case.bc, case.u_in)
    cb, _ = coarse.tag(case.tri, want_theta=False)
    G.set_blocked(0, cb)
    G.set_blocked(1, blocked.reshape(N[2], N[1], N[0]).contiguous())
    coarse.close()
    del cb
    for _ in range(2):
        G.laplacian(x, y)
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev2[0].record()
    for _ in range(reps):
        G.laplacian(x, y)
    ev2[1].record()
    G.sor(y, x, 1.8, reps)
    ev2[2].record()
    torch.cuda.synchronize()
    mlap_us = ev2[0].elapsed_time(ev2[1]) / reps * 1e3
    msor_us = ev2[1].elapsed_time(ev2[2]) / reps * 1e3
    solve = bcm_solve_timing(G, case, n, ibm, torch)
    cells = G.ncubes * n ** 3
    fine = int(refine.sum())
    # algorithmic bytes: operator 16 B per cell (x read once, y written); exchange per
    # halo cell the destination, two offsets and one source index (16 B), the value
    # read and written (16 B), plus 7 more source reads and indices for a mean
    lap_bytes = 16 * cells
    out = {"coarse_cubes": math.prod(K), "refined": fine, "cubes": int(G.ncubes), "cells": int(cells),
           "halo_cells": int(G.nhalo), "exchange_us": round(ex_us, 2), "laplacian_us": round(lap_us, 2),
           "sor_sweep_us": round(sor_us, 2),
           "with_geometry": {"laplacian_us": round(mlap_us, 2), "sor_sweep_us": round(msor_us, 2),
                             "mask_bytes_per_cell": 1, "solve": solve},
           "laplacian_bytes_per_cell": 16,
           "laplacian_achieved_gbs": round(lap_bytes / (lap_us * 1e-6) / 1e9, 1),
           "roofline": {"bound": "hbm", "achieved": round(lap_bytes / (lap_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(lap_bytes / (lap_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": committed_traffic("bcm_laplacian", args.workload), "kernel": "k_bcm_lap",
                        "algorithmic_bytes_per_launch": lap_bytes, "avg_launch_us": round(lap_us, 2)}}
    G.close()
    return out


# Crank-Nicolson predictor (eq. (crank-nicolson)), three velocity components of FP64:
# algorithmic bytes per cell of each BiCGStab pass, as stated in momentum.hip (timing
# slots 4-8 in this order)
CN_PASSES = ("cn_direction", "cn_apply_p", "cn_stabilise", "cn_apply_s", "cn_update")
CN_KERNELS = {"cn_direction": "k_cn_dir<double>", "cn_apply_p": "k_cn_ap<double>", "cn_stabilise": "k_cn_s<double>",
              "cn_apply_s": "k_cn_as<double>", "cn_update": "k_cn_x<double>"}
CN_BYTES_PER_CELL = {"cn_direction": 96, "cn_apply_p": 105, "cn_stabilise": 72, "cn_apply_s": 81,
                     "cn_update": 168}


def cn_timing(case, s, st, ctl, step, args, ibm, torch):
    """Crank-Nicolson steps on the developed plain FP64 state at twice the explicit CFL
    (0.6): whole steps timed by the host clock, the five BiCGStab passes by dispatch
    events (timing slots 4-8).  A pass launched after its solve converged returns at
    once; the per-launch figures divide by the passes that did work (iterations made,
    the largest component count per solve)."""
    N = case.n[0] * case.n[1] * case.n[2]
    dt = min(2.0 * case.dt, 0.6 * case.dx / max(ctl["umax"], 1e-30))
    prm = lambda k: ibm.step_params(dt, case.nu, csm=case.csm, step=k, tol=args.tol, max_iter=20000,  # noqa: E731
                                    check_every=16, scheme="cn", mom_tol=args.mom_tol)
    for _ in range(2):
        rc, stats = s.step(st, prm(step))
        step += 1
    ibm.ibm_timing_enable(s.ctx, True)
    for k in (4, 5, 6, 7, 8):
        ibm.ibm_timing_slot(s.ctx, k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, worked = [], 0
    for _ in range(args.cn_steps):
        rc, stats = s.step(st, prm(step))
        if rc != 0:
            raise SystemExit("crank-nicolson step did not converge (rc=%d)" % rc)
        step += 1
        its.append(stats["iters_momentum"])
        worked += max(stats["iters_momentum"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    slots = {name: ibm.ibm_timing_slot(s.ctx, k, reset=True) for name, k in zip(CN_PASSES, (4, 5, 6, 7, 8))}
    ibm.ibm_timing_enable(s.ctx, False)
    passes = {}
    for name, (ms, launches) in slots.items():
        avg = ms / 1e3 / max(worked, 1)
        passes[name] = {"kernel": CN_KERNELS[name], "ms_total": round(ms, 3), "launches": launches,
                        "launches_with_work": worked, "avg_launch_us": round(avg * 1e6, 2),
                        "bytes_per_cell": CN_BYTES_PER_CELL[name],
                        "achieved_gbs": round(CN_BYTES_PER_CELL[name] * N / avg / 1e9, 1) if avg > 0 else None}
    dom = max(CN_PASSES, key=lambda n: slots[n][0])
    d = passes[dom]
    traffic = committed_traffic(dom, args.workload)
    return {"dt": dt, "cfl": 0.6, "mom_tol": args.mom_tol, "steps": args.cn_steps,
            "ms_per_step": round(elapsed / args.cn_steps * 1e3, 2),
            "value": N * args.cn_steps / elapsed,
            "iters_per_component": its,
            "predictor_ms_per_step": round(sum(v[0] for v in slots.values()) / args.cn_steps, 3),
            "passes": passes,
            "roofline": {"bound": "hbm", "achieved": d["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(d["achieved_gbs"] / HBM_PEAK_GBS, 4) if d["achieved_gbs"] else None,
                         "traffic": traffic, "kernel": d["kernel"],
                         "algorithmic_bytes_per_launch": d["bytes_per_cell"] * N,
                         "avg_launch_us": d["avg_launch_us"]}}


def train_network(args, ibm, torch):
    """Trains the learned preconditioner on the GPU (library forward/backward kernels,
    Adam) on (b, p) pairs of the plain FP64 solver from seeded 64^3 windows of the
    ellipsoid field, disjoint from the benchmark geometry (seed 0).  Untimed set-up."""
    from paper_2002_06206_amd import inputs, train
    t0 = time.perf_counter()
    # 20 windows x 100 steps, every step from the third on: 1,960 (b, p) pairs
    seeds = tuple(range(train.TRAIN_SEEDS[0], train.TRAIN_SEEDS[0] + args.train_windows))   # disjoint from EVAL_SEEDS
    data = train.build_dataset(seeds, 64, steps=100, every=1,
                               depths=tuple(int(k) for k in args.train_depths.split(",")))
    held = train.build_dataset(train.EVAL_SEEDS, 64, steps=24, every=3)
    t1 = time.perf_counter()
    net = ibm.Network(64 ** 3, inputs.cnn_init_weights(0))
    om = getattr(args, "train_smooth", 0.0)
    before = train.mean_loss(net, held, om)
    train.train(net, data, args.train_iters, args.train_lr, omega=om)
    after = train.mean_loss(net, held, om)
    w = net.weights
    net.close()
    for s_, _ in data + held:
        s_.close()
    torch.cuda.synchronize()
    info = {"pairs": sum(len(p) for _, p in data), "data_s": round(t1 - t0, 2),
            "train_s": round(time.perf_counter() - t1, 2), "iters": args.train_iters,
            "depths": args.train_depths, "loss_smoothing_omega": round(om, 6),
            "heldout_loss_before": round(before, 4), "heldout_loss_after": round(after, 4)}
    return w, info


def probe(ibm, torch, n=384, reps=10):
    """Practical bandwidth ceilings and the counter calibration kernel.  Two plain
    streaming kernels of the library on n^3 doubles: the cell copy (ibm_get_rhs, k_copy:
    8 B read and 8 B written per cell) and the FP64 7-point operator (ibm_apply_laplacian:
    x and the code byte read, y written; 17 B per cell), each launched on buffers rotated
    over three pairs (3 x 2 x 432 MiB at n = 384, beyond the 256 MB Infinity Cache) and
    timed with events on the stream they run on.  Under rocprofv3 --pmc the k_copy
    dispatches calibrate FETCH_SIZE / WRITE_SIZE against their known 2 x 8 B per cell."""
    torch.cuda.set_device(0)
    bc = (ibm.INFLOW, ibm.OUTFLOW) + (ibm.SLIP,) * 4
    s = ibm.Solver((n, n, n), 1.0, (0.0, 0.0, 0.0), bc, (1.0, 0.0, 0.0))
    s.build(torch.zeros((n, n, n), dtype=torch.uint8, device="cuda"),
            torch.full((n, n, n, 6), 2.0, dtype=torch.float64, device="cuda"))
    bufs = [(torch.randn((n, n, n), dtype=torch.float64, device="cuda"),
             torch.empty((n, n, n), dtype=torch.float64, device="cuda")) for _ in range(3)]
    out = {"cells": n ** 3}
    for name, bytes_per_cell in (("copy", 16), ("laplacian", 17)):
        def run(k):
            x, y = bufs[k % 3]
            if name == "copy":
                ibm.ibm_get_rhs(s.ctx, y)   # the context's right-hand side buffer into y (values unused)
            else:
                ibm.ibm_apply_laplacian(s.ctx, x, y)
        for k in range(3):
            run(k)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        stream = torch.cuda.current_stream()
        ev[0].record(stream)
        for k in range(reps):
            run(k)
        ev[1].record(stream)
        torch.cuda.synchronize()
        us = ev[0].elapsed_time(ev[1]) / reps * 1e3
        out[name] = {"us_per_launch": round(us, 2), "bytes_per_cell": bytes_per_cell,
                     "gbs": round(bytes_per_cell * n ** 3 / (us * 1e-6) / 1e9, 1)}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ellipsoids256")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--warmup-tol", type=float, default=None,
                    help="Poisson tolerance of the untimed warm-up steps (default: --tol)")
    ap.add_argument("--inner-tol", type=float, default=1e-1,
                    help="mixed solve: residual reduction of each FP32 segment between FP64 replacements")
    ap.add_argument("--inner-tol-learned", type=float, default=1e-5,
                    help="mixed+learned solve: the same per segment (flexible CG restarts at each "
                         "replacement, so it favours fewer, longer segments)")
    ap.add_argument("--inner-restart", type=int, default=0,
                    help="mixed solve: 1 = start every FP32 segment from a fresh search direction")
    ap.add_argument("--p-guess", default="extrapolate", choices=["extrapolate", "previous"],
                    help="initial guess of each step's pressure solve: the better of p^n and "
                         "2 p^n - p^{n-1} (by residual), or p^n")
    ap.add_argument("--solver", default="mixed_learned", choices=["mixed", "mixed_learned", "pcg_fp64"],
                    help="headline solver (the metric names mixed+learned); plain FP64 and mixed always run")
    ap.add_argument("--smooth", type=float, default=6.0 / 7.0,
                    help="damped Jacobi weight of the smoothing steps around the network in the learned solve "
                         "(0: the network's map alone)")
    ap.add_argument("--train-smooth", type=float, default=0.0,
                    help="train the network through the smoothed preconditioner with this weight "
                         "(0: as the network's map alone)")
    ap.add_argument("--no-learned", action="store_true", help="skip training and the learned solver")
    ap.add_argument("--train-iters", type=int, default=2000)
    ap.add_argument("--train-lr", type=float, default=2e-3)
    ap.add_argument("--train-windows", type=int, default=20, help="64^3 training windows (98 pairs each)")
    ap.add_argument("--train-depths", default="0,32",
                    help="Krylov depths of the training pairs, cycled (0: the step's (b, p) itself)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes of the CPU baseline (0: min(16, host CPUs))")
    ap.add_argument("--cn-steps", type=int, default=5,
                    help="Crank-Nicolson steps timed after the plain FP64 run (0: none)")
    ap.add_argument("--mom-tol", type=float, default=1e-10, help="Crank-Nicolson momentum solve tolerance")
    ap.add_argument("--quick-steps", type=int, default=5,
                    help="explicit steps with the hybrid central/QUICK face value timed after the plain run (0: none)")
    ap.add_argument("--quick", type=float, default=0.1, help="QUICK weight of the hybrid face value")
    ap.add_argument("--sor", type=int, default=1, help="time red-black SOR against PCG on one right-hand side")
    ap.add_argument("--bcm", type=int, default=1, help="time the building-cube halo exchange and operator")
    ap.add_argument("--sor-omega", type=float, default=0.0, help="SOR relaxation (0: 2/(1+sin(pi/n)))")
    ap.add_argument("--probe", action="store_true",
                    help="only measure the copy and 7-point-operator bandwidth ceilings (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library and this benchmark run on one GPU only (collectives and sharding are "
              "not part of them); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.probe:
        import torch

        from paper_2002_06206_amd import ibm
        print(json.dumps({"probe": probe(ibm, torch)}))
        return
    case = workload(args.workload)
    N = case.n[0] * case.n[1] * case.n[2]
    # the CPU sample runs first, before this process touches the GPU, on the host's cores
    # (at most 16: the CPU share of one GPU on the benchmark hosts)
    cpu_runs = None
    if not args.no_cpu_baseline and N <= 512 ** 3:
        workers = args.cpu_workers if args.cpu_workers > 0 else min(16, os.cpu_count() or 1)
        cpu_runs = cpu_samples(args.workload, workers)

    import torch

    from paper_2002_06206_amd import ibm
    torch.cuda.set_device(0)

    # the plain FP64 context and state (~330 B per cell) do not fit one GPU at 1024^3
    plain = run_solver(case, "pcg_fp64", args, ibm, torch) if N <= 512 ** 3 else None
    runs = {"mixed": run_solver(case, "mixed", args, ibm, torch)}
    if plain is not None:
        runs["pcg_fp64"] = plain
    train_info = None
    if not args.no_learned or args.solver == "mixed_learned":
        w, train_info = train_network(args, ibm, torch)
        runs["mixed_learned"] = run_solver(case, "mixed_learned", args, ibm, torch, w)
    head = runs[args.solver]
    dom = head["dominant"]
    sweep = runs["mixed"]["dominant"]
    sweep_traffic = committed_traffic(sweep["name"] + "_f32", args.workload)
    roofline_sweeps = {"bound": "hbm", "achieved": round(sweep["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(sweep["achieved_gbs"] / HBM_PEAK_GBS, 4),
                       "traffic": sweep_traffic, "kernel": sweep["kernel"],
                       "algorithmic_bytes_per_launch": sweep["bytes_per_cell"] * N,
                       "avg_launch_us": round(sweep["avg_s"] * 1e6, 2), "sweeps_ms": sweep["sweeps_ms"]}
    if dom.get("bound") == "mfma":
        traffic = committed_traffic(CONV_NAME, args.workload)
        roofline = {"bound": "mfma", "achieved": round(dom["achieved_tflops"], 1), "peak": BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(dom["achieved_tflops"] / BF16_PEAK_TFLOPS, 4),
                    "traffic": traffic, "kernel": dom["kernel"], "flop_per_launch": dom["flop_per_launch"],
                    "algorithmic_bytes_per_launch": dom["bytes_per_cell"] * N,
                    "achieved_algorithmic_gbs": round(dom["achieved_gbs"], 1),
                    "avg_launch_us": round(dom["avg_s"] * 1e6, 2), "launches": dom["launches"],
                    "launches_with_work": dom["launches_with_work"], "sweeps_ms": dom["sweeps_ms"]}
    else:
        traffic = committed_traffic(dom["name"] + ("" if args.solver == "pcg_fp64" else "_f32"), args.workload)
        roofline = {"bound": "hbm", "achieved": round(dom["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": dom["kernel"], "algorithmic_bytes_per_launch": dom["bytes_per_cell"] * N,
                    "avg_launch_us": round(dom["avg_s"] * 1e6, 2), "launches": dom["launches"],
                    "launches_with_work": dom["launches_with_work"], "sweeps_ms": dom["sweeps_ms"]}
    cpu = None
    if cpu_runs is not None and plain is not None:
        cpu = cpu_baseline(case, cpu_runs[0], cpu_runs[1], plain["iters_per_step"])
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"pcg_fp64": "f64", "mixed": "f32+f64", "mixed_learned": "bf16+f32+f64"}[args.solver],
        "data": "synthetic",
        "config": {"workload": case.name, "cells": list(case.n), "triangles": int(len(case.tri)),
                   "cuts": head["cuts"], "solver": head["solver"], "tol": args.tol, "inner_tol": args.inner_tol,
                   "inner_tol_learned": args.inner_tol_learned,
                   "preconditioner_smoothing_omega": round(args.smooth, 6),
                   "nu": case.nu, "dt_max": case.dt, "cfl": 0.3, "csm": case.csm,
                   "pressure_guess": ("p^n or 2p^n - p^(n-1), the smaller residual" if args.p_guess == "extrapolate"
                                      else "p^n")},
        "plain_fp64_value": plain["value"] if plain else None,
        "speedup_vs_plain_fp64": head["value"] / plain["value"] if plain else None,
        "solvers": {k: {kk: vv for kk, vv in v.items()
                        if kk not in ("dominant", "crank_nicolson", "hybrid_quick", "predictor", "red_black_sor",
                                      "building_cubes")}
                    for k, v in runs.items()},
        "speedups_vs_plain_fp64": {k: round(v["value"] / plain["value"], 4) for k, v in runs.items()} if plain else None,
        "training": train_info,
        "roofline": roofline,
        "roofline_sweeps": roofline_sweeps,
        "step_roofline": head["step_roofline"],
        "surface_force": head.get("surface_force"),
        "crank_nicolson": plain.get("crank_nicolson") if plain else None,
        "hybrid_quick": plain.get("hybrid_quick") if plain else None,
        "red_black_sor": plain.get("red_black_sor") if plain else None,
        "building_cubes": plain.get("building_cubes") if plain else None,
        "predictor": plain.get("predictor") if plain else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

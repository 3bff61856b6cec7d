#!/usr/bin/env python3
"""Throughput of the meshfree ALE BGK time step on one MI355X.

One "step" is one full bgk_step (neighbour search, least-squares operators,
upwind transport, moments + implicit relaxation, walls, motion) over every
particle and velocity of the workload, with all inputs resident in HBM.  The
metric is particle x velocity updates per second: N * N_v / t_step (a Chu
pair g1, g2 counts once).

Default workload: the 3D cavity with 48^3 particles and 20^3 velocities on
[-4, 4]^3 (full BGK, h = 2.2 dx, Kn = 1, lid 0.1, moving cloud), FP64.  The
same run is repeated in FP32 and BF16-operand modes; each precision then
continues untimed to the workload's 200 steps, and the errors of rho, u, T
against the FP64 run are reported there, at Kn = 1 and (unless
--no-kn-sweep) at Kn = 0.1 and 10.

Printed: one JSON line (the benchmark contract), with the roofline of the
dominant kernel (the transport, timed with HIP events on the library's
stream inside the timed region) and the CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
# VALU lane-operation issue rate, FP64 and unpacked FP32 alike:
# 256 CUs x 4 SIMDs x 16 lanes/clock x 2.4 GHz = 39.3e12 lane-ops/s
# (= the 78.6 TFLOP/s FP64 vector peak with an FMA counted as 2 flops).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources the fused kernel's machine code depends on: a traffic figure measured
# with counters is reported only while these are unchanged.
TRAFFIC_SOURCES = ("paper_2408_02350_amd/csrc/k_fused.hip",
                   "paper_2408_02350_amd/csrc/device_common.h",
                   "paper_2408_02350_amd/csrc/bgk_internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, precision):
    """HBM bytes per launch of the fused kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    there is none for this workload or the kernel source changed since."""
    import glob
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md"))):
        with open(path) as fh:
            m = re.search(r"<!--\s*traffic:\s*(\{.*?\})\s*-->", fh.read(), flags=re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("workload") == workload and rec.get("precision") == precision:
            if rec.get("source_sha256") == kernel_source_hash():
                return float(rec["bytes_per_launch"])
    return None


def transport_algorithmic(cav, edges, prec):
    """Algorithmic work of one transport launch.

    bytes: read every f row once, write every interior f-tilde row once, read
    the d*d upwind vectors of every edge once.  ops: k VALU lane-ops per
    (particle, neighbour, velocity) with k = 5 + 2 n_c (2D Chu: two
    incremental projections, two min(0, .), one add, per component one
    subtract and one FMA) or 8 + 2 n_c (3D: three projections, three mins,
    two adds, subtract and FMA)."""
    s = 8 if prec == "fp64" else 4
    NV, nc, d = cav.n_velocities, cav.n_comp, cav.dim
    N = cav.n_particles
    n_wall = N - cav_interior(cav)
    bytes_ = N * NV * nc * s + (N - n_wall) * NV * nc * s + edges * d * d * s
    k = (5 + 2 * nc) if d == 2 else (8 + 2 * nc)
    ops = edges * NV * k
    return bytes_, ops, k


def cav_interior(cav):
    return (cav.n - 2) ** cav.dim


def run_gpu(cav, precision, steps, warmup, timing=True, total_steps=None):
    """Time `steps` full steps after `warmup`; then (untimed) continue to
    total_steps.  Returns the timing and (rho, U, T) at the last step; diag
    also holds the state check of the last state (smallest f, negative and
    non-finite counts, moment residuals) and the drift of total mass and
    energy since the initial state."""
    import torch

    import paper_2408_02350_amd.bgk as bgk

    sim = bgk.Simulation(cav, precision=precision, device="cuda:0")
    log(f"[bench] {cav.name} {precision}: N={cav.n_particles} NV={cav.n_velocities} "
        f"warmup={warmup} steps={steps}")
    s0 = bgk.bgk_state_check(sim.ctx, sim.f, sim.rho, sim.U, sim.T)
    sim.step(warmup)
    bgk.bgk_check(sim.ctx)
    torch.cuda.synchronize()
    if timing:
        bgk.bgk_timing_enable(sim.ctx, True)
        bgk.bgk_timing_read(sim.ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bgk.bgk_check(sim.ctx)
    ktime = bgk.bgk_timing_read(sim.ctx) if timing else (0.0, 0)
    diag = bgk.bgk_diagnostics(sim.ctx)
    cnt, _ = bgk.bgk_build_neighbors(sim.ctx, sim.x)
    interior = sim.wall_id == 0
    edges = int((cnt[interior] - 1).sum().item())
    ms = (t1 - t0) * 1e3 / steps
    log(f"[bench] {precision}: {ms:.4f} ms/step, transport {ktime[0] / max(ktime[1], 1):.4f} ms "
        f"x {ktime[1]}, edges {edges}, diag {diag}")
    done = warmup + steps
    if total_steps is not None and total_steps > done:
        sim.step(total_steps - done)
        bgk.bgk_check(sim.ctx)
        done = total_steps
    torch.cuda.synchronize()
    s1 = bgk.bgk_state_check(sim.ctx, sim.f, sim.rho, sim.U, sim.T)
    diag["state"] = {k: s1[k] for k in ("min_f", "negatives", "nonfinite", "rho_residual",
                                        "U_residual", "T_residual")}
    diag["state"].update({"mass_drift": (s1["mass"] - s0["mass"]) / s0["mass"],
                          "energy_drift": (s1["energy"] - s0["energy"]) / s0["energy"],
                          "after_steps": done})
    state = (sim.rho.cpu().numpy(), sim.U.cpu().numpy(), sim.T.cpu().numpy())
    del sim
    torch.cuda.empty_cache()
    return ms, ktime, edges, state, diag, done


def follow_run(cav, precision, steps, follow=None, record=None):
    """Untimed run of `steps` steps.  record: a list that receives the
    positions before every step; follow: positions to take before every step
    (another run's cloud).  Returns (rho, U, T) after the last step."""
    import torch

    import paper_2408_02350_amd.bgk as bgk

    sim = bgk.Simulation(cav, precision=precision, device="cuda:0")
    for s in range(steps):
        if record is not None:
            record.append(sim.x.clone())
        if follow is not None:
            sim.x.copy_(follow[s])
        sim.step(1)
    bgk.bgk_check(sim.ctx)
    torch.cuda.synchronize()
    state = (sim.rho.cpu().numpy(), sim.U.cpu().numpy(), sim.T.cpu().numpy())
    del sim
    torch.cuda.empty_cache()
    return state


def time_particle_management(cav, reps):
    """Wall time of one plan (with its host read of the counts) and one
    apply on a disturbed cloud of the workload's lattice (interior particles
    displaced by up to 0.45 dx, 20% removed), FP64 state at the rest
    Maxwellian, mean over reps after one warm-up."""
    import torch

    import paper_2408_02350_amd.bgk as bgk
    from paper_2408_02350_amd.inputs import disturbed_cloud

    x, wid = disturbed_cloud(cav.dim, cav.n, 0)
    N = x.shape[1]
    cfg = bgk.config_from(cav, cav.precision, n_particles=N, flags=bgk.BGK_FLAG_PARTICLES)
    dev = torch.device("cuda:0")
    ctx = bgk.bgk_init(cfg, torch.from_numpy(wid).to(dev))
    xt = torch.from_numpy(x).to(dev)
    rho = torch.ones(N, dtype=torch.float64, device=dev)
    U = torch.zeros((cav.dim, N), dtype=torch.float64, device=dev)
    T = torch.ones(N, dtype=torch.float64, device=dev)
    f = bgk.bgk_maxwellian(ctx, rho, U, T)
    plan_ms, apply_ms = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pairs, holes = bgk.bgk_pm_plan(ctx, xt)
        t1 = time.perf_counter()
        out = bgk.bgk_pm_apply(ctx, xt, f, rho, U, T, N - pairs + holes)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        bgk.bgk_check(ctx)
        del out
        if r > 0:
            plan_ms.append((t1 - t0) * 1e3)
            apply_ms.append((t2 - t1) * 1e3)
    log(f"[bench] particle management {cav.name}: N={N} pairs={pairs} holes={holes}")
    return {"workload": cav.name + "_disturbed", "n_particles": N, "n_velocities": cav.n_velocities,
            "pairs": pairs, "holes": holes, "plan_ms": sum(plan_ms) / len(plan_ms),
            "apply_ms": sum(apply_ms) / len(apply_ms), "reps": reps, "precision": cav.precision}


def time_adjoint(cav, precision, nsteps, every, reps):
    """The reverse mode on one GPU: wall time of one checkpointed rollout
    (forward pass, then backward pass: segment recomputation keeping each
    step's state, plus the reverse steps on them), the device time of one
    reverse step alone (bgk_adjoint_step, which recomputes its forward step;
    HIP events on the library stream, mean over reps), and that of the
    reverse kernels alone (bgk_adjoint_step_kept on a kept state).

    Roofline of the reverse step: bytes = 3 n_c N N_v s (read the adjoint
    of f-tilde and f^n, write lam_f; s = 8 in FP64, 4 in FP32 storage);
    ops = 2 k per (particle, neighbour, velocity) with k the forward count
    (the flux and its U-derivative)."""
    import torch

    import paper_2408_02350_amd.bgk as bgk
    from paper_2408_02350_amd.adjoint import FrozenCavity, rollout_objective

    dev = torch.device("cuda:0")
    problem = FrozenCavity(cav, device=dev, precision=precision)
    f0 = problem.rest_state()
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=dev, requires_grad=True)
    walls = []
    for r in range(2):
        f0g = f0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = rollout_objective(problem, f0g, lid, nsteps, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        walls.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    fwd_ms, bwd_ms = walls[-1]
    # one reverse step alone, on the state after the rollout
    (f, rho, U, T), _ = problem.forward(f0, cav.lid, 5)
    c = problem.ctx
    lam_f = torch.rand_like(f)
    lam_U = torch.zeros_like(U)
    out_f, out_U = torch.empty_like(f), torch.empty_like(U)
    bgk.bgk_adjoint_step(c, f, U, problem.x, lam_f, lam_U, None, None, out_f, out_U)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    stream = c.stream
    ev[0].record(stream)
    for _ in range(reps):
        bgk.bgk_adjoint_step(c, f, U, problem.x, lam_f, lam_U, None, None, out_f, out_U)
    ev[1].record(stream)
    torch.cuda.synchronize()
    bgk.bgk_check(c)
    step_ms = ev[0].elapsed_time(ev[1]) / reps
    # the reverse kernels alone, on the state bgk_step_keep kept
    f1, ft, U1 = torch.empty_like(f), torch.empty_like(f), U.clone()
    rho1, T1 = torch.empty_like(rho), torch.empty_like(T)
    bgk.bgk_step_keep(c, f, f1, problem.x, U1, rho1, T1, ft)
    kept = (ft, f1, rho1, U1, T1)
    bgk.bgk_adjoint_step_kept(c, f, U, problem.x, kept, lam_f, lam_U, None, None, out_f, out_U)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        bgk.bgk_adjoint_step_kept(c, f, U, problem.x, kept, lam_f, lam_U, None, None, out_f, out_U)
    ev[1].record(stream)
    torch.cuda.synchronize()
    bgk.bgk_check(c)
    kern_ms = ev[0].elapsed_time(ev[1]) / reps
    del f1, ft, kept
    cnt, _ = bgk.bgk_build_neighbors(c, problem.x)
    edges = int((cnt[problem.wall_id == 0] - 1).sum().item())
    s = 8 if precision == "fp64" else 4
    nc, NV, N = cav.n_comp, cav.n_velocities, cav.n_particles
    k = (5 + 2 * nc) if cav.dim == 2 else (8 + 2 * nc)
    bytes_, ops = 3 * nc * N * NV * s, edges * NV * 2 * k
    return {"workload": cav.name, "precision": precision, "steps": nsteps,
            "checkpoint_every": every, "rollout_forward_ms": fwd_ms,
            "rollout_backward_ms": bwd_ms, "reverse_step_ms": step_ms,
            "reverse_step_hbm_frac": bytes_ / (step_ms * 1e-3) / (PEAK_HBM_GBS * 1e9),
            "reverse_step_alu_frac": ops / (step_ms * 1e-3) / (PEAK_VALU_TOPS * 1e12),
            "reverse_kernels_ms": kern_ms,
            "reverse_kernels_alu_frac": ops / (kern_ms * 1e-3) / (PEAK_VALU_TOPS * 1e12),
            "algorithmic_bytes": bytes_, "algorithmic_ops": ops}


def moment_errors(state, ref, lid):
    import numpy as np

    rho, U, T = state
    r0, U0, T0 = ref
    e_rho = float(np.max(np.abs(rho - r0)) / np.max(np.abs(r0)))
    e_T = float(np.max(np.abs(T - T0)) / np.max(np.abs(T0)))
    e_u = float(np.max(np.sqrt(((U - U0) ** 2).sum(axis=0))) / abs(lid))
    return e_rho, e_u, e_T


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cav, budget_s):
    """The CPU oracle on the host cores, on a bounded sample of the workload.

    The oracle's full step at the 3D sizes takes minutes, so the sample is
    the per-particle work of one step (neighbour row by the oracle's O(N)
    scan, least-squares row, transport of the row over all velocities, its
    moments and relaxation: S1-S6, the same row functions the oracle's full
    step runs) for a window of consecutive interior particles of the
    workload's cloud, sized to about budget_s seconds; the rate is that
    window's particle x velocity updates per second (walls and motion, a
    few percent of a step, are not in the sample).  Timed once on all the
    OpenMP threads and once on one thread."""
    import numpy as np

    import oracle
    from paper_2408_02350_amd.inputs import cloud_for

    c = oracle.config(cav)
    x, wid = cloud_for(cav)
    N = cav.n_particles
    interior = np.nonzero(wid == 0)[0]
    start = len(interior) // 4
    kmax = min(20000, len(interior) - 1 - start)      # window limit, interior rows
    # timing input: a constant f and a resting gas (the row work does not
    # depend on the values).  Only the rows a window can read are filled:
    # the window and its neighbours, which lie within 3 lattice layers.
    margin = 4 * cav.n ** (cav.dim - 1)
    lo = max(0, int(interior[start]) - margin)
    hi = min(N, int(interior[start + kmax]) + 1 + margin)
    f = np.empty((cav.n_comp, N, cav.n_velocities))
    f[:, lo:hi] = 0.01
    U = np.zeros((cav.dim, N))

    def sample(threads):
        k, sec, rows = 64, 0.0, 0
        i0 = int(interior[start])
        while True:     # grow the window until it takes about budget_s
            i1 = int(interior[start + k]) + 1
            _, sec, rows = oracle.step_rows(c, wid, x, f, U, i0, i1, threads)
            if sec >= 0.25 * budget_s or k >= kmax:
                break
            k = min(kmax, int(k * min(16.0, max(2.0, budget_s / max(sec, 1e-3)))))
        if sec < 0.5 * budget_s and k < kmax:
            k = min(kmax, int(k * budget_s / max(sec, 1e-3)))
            i1 = int(interior[start + k]) + 1
            _, sec, rows = oracle.step_rows(c, wid, x, f, U, i0, i1, threads)
        log(f"[bench] oracle sample, {threads or oracle.num_threads()} thread(s): {rows} rows "
            f"in {sec:.2f} s")
        return rows * cav.n_velocities / sec, rows, sec

    cores = oracle.num_threads()
    v_all, r_all, s_all = sample(0)
    v_one, r_one, s_one = sample(1)
    return {"value": v_all, "unit": "particle-velocity updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "single_thread": {"value": v_one, "cores": 1, "rows": r_one, "seconds": s_one},
            "sample": f"S1-S6 of {r_all} consecutive interior particles ({r_one} on one thread) "
                      f"of {cav.name} ({cav.n_particles} particles x {cav.n_velocities} "
                      f"velocities, FP64; the oracle's row functions: O(N) neighbour scan, "
                      f"least-squares row, transport of the row, moments + relaxation), "
                      f"{s_all:.1f} s on {cores} threads, {s_one:.1f} s on one thread"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5", help="c1..c5 (default c5)")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 runs")
    ap.add_argument("--no-kn-sweep", action="store_true",
                    help="report the FP32/BF16 errors at the workload's Kn only")
    ap.add_argument("--error-steps", type=int, default=None,
                    help="steps after which the FP32/BF16 errors are taken (default: the "
                         "workload's step count, at least warmup + steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="CPU seconds of each oracle sample (all threads, then one thread)")
    ap.add_argument("--paper-scales", action="store_true",
                    help="only time the paper's own cavity sizes (20 velocity points per "
                         "axis, h = 3.1 dx, first-derivative least squares) and print one "
                         "JSON line with the per-step times")
    ap.add_argument("--particle-management", action="store_true",
                    help="only time bgk_pm_plan + bgk_pm_apply on a disturbed cloud of the "
                         "workload's size and print one JSON line")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time the reverse mode (checkpointed rollouts of the 100^2 x 24^2 "
                         "cavity, FP64, and of a 20-step window of the 48^3 x 20^3 cavity, FP32 "
                         "storage; --workload c4 or c5 for one of them) and print one JSON line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.rand(n, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB x 5")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU velocity-sharded design is not built)", file=sys.stderr)
        sys.exit(2)

    from paper_2408_02350_amd.inputs import CONFIGS, PAPER_SCALES

    if args.paper_scales:
        rows = []
        for key, pc in PAPER_SCALES.items():
            pc = pc.replace(precision=args.precision)
            ms, ktime, edges, *_ = run_gpu(pc, args.precision, args.steps, args.warmup)
            interior = cav_interior(pc)
            rows.append({"workload": pc.name, "n_particles": pc.n_particles,
                         "n_velocities": pc.n_velocities, "h_over_dx": pc.h_factor,
                         "wls": "first-derivative fit", "mean_neighbours": edges / interior + 1,
                         "ms_per_step": ms,
                         "transport_ms": ktime[0] / max(ktime[1], 1),
                         "updates_per_s": pc.n_particles * pc.n_velocities / (ms * 1e-3)})
        print(json.dumps({"paper_scales": rows, "precision": args.precision,
                          "steps": args.steps, "warmup": args.warmup}), flush=True)
        return

    if args.adjoint:
        rows = []
        if args.workload in ("c2", "c4"):
            rows.append(time_adjoint(CONFIGS["c4"], "fp64", 50, 10, 10))
        if args.workload in ("c2", "c5"):
            rows.append(time_adjoint(CONFIGS["c5"].replace(move=0), "fp32", 20, 5, 3))
        print(json.dumps({"adjoint": rows}), flush=True)
        return

    if args.particle_management:
        print(json.dumps({"particle_management": time_particle_management(
            CONFIGS[args.workload].replace(precision=args.precision), args.steps)}), flush=True)
        return

    cav = CONFIGS[args.workload].replace(precision=args.precision)
    mixed_on = not args.no_mixed and args.precision == "fp64"
    err_steps = args.error_steps if args.error_steps is not None else cav.steps
    err_steps = max(err_steps, args.warmup + args.steps)
    ms, ktime, edges, state, diag, _ = run_gpu(cav, args.precision, args.steps, args.warmup,
                                               total_steps=err_steps if mixed_on else None)
    updates = cav.n_particles * cav.n_velocities
    value = updates / (ms * 1e-3)

    k_ms = ktime[0] / max(ktime[1], 1)
    bytes_, ops, k = transport_algorithmic(cav, edges, args.precision)
    t_alu = ops / (PEAK_VALU_TOPS * 1e12)
    t_hbm = bytes_ / (PEAK_HBM_GBS * 1e9)
    ach_gbs = bytes_ / (k_ms * 1e-3) / 1e9
    ach_tops = ops / (k_ms * 1e-3) / 1e12
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": ach_tops, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                "frac": ach_tops / PEAK_VALU_TOPS}
    else:
        roof = {"bound": "hbm", "achieved": ach_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach_gbs / PEAK_HBM_GBS}
    roof.update({"traffic": measured_traffic(cav.name, args.precision), "kernel": "k_fused",
                 "kernel_ms": k_ms, "kernel_updates_per_s": updates / (k_ms * 1e-3),
                 "algorithmic_bytes": bytes_, "algorithmic_ops": ops, "ops_per_update": k,
                 "hbm_frac": ach_gbs / PEAK_HBM_GBS, "alu_frac": ach_tops / PEAK_VALU_TOPS,
                 "step_share": k_ms / ms})

    out = {
        "metric": "particle×velocity updates/sec per step (FP64 vs mixed) at stated moment error",
        "value": value,
        "unit": "particle-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16xf32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": cav.name, "dim": cav.dim, "n_particles": cav.n_particles,
                   "n_velocities": cav.n_velocities, "n_comp": cav.n_comp, "kn": cav.kn,
                   "h_over_dx": cav.h_factor, "wls_degree": cav.wls_degree,
                   "precision": args.precision, "move": cav.move,
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "state": diag["state"],
    }

    if mixed_on:
        # FP32 and BF16 operands: timed like the FP64 run.  Their errors of
        # rho, u (over the lid speed) and T against FP64 after err_steps steps
        # are taken along the FP64 run's cloud (the run takes the FP64 run's
        # positions before every step: two free runs a rounding apart cross
        # the weight's truncation r = h at different steps, a discontinuity
        # of the method rather than an error of the arithmetic), and, as
        # "free", from the free-running timed run continued to err_steps.
        mixed = {}
        xs = []
        ref = follow_run(cav, "fp64", err_steps, record=xs)
        for p in ("fp32", "bf16"):
            ms_p, kt_p, _, st_free, _, n_p = run_gpu(cav.replace(precision=p), p, args.steps,
                                                     args.warmup, total_steps=err_steps)
            st_p = follow_run(cav.replace(precision=p), p, err_steps, follow=xs)
            e_rho, e_u, e_T = moment_errors(st_p, ref, cav.lid)
            f_rho, f_u, f_T = moment_errors(st_free, state, cav.lid)
            log(f"[bench] {p} vs fp64 after {err_steps} steps: e_rho {e_rho:.2e} e_u {e_u:.2e} "
                f"e_T {e_T:.2e} (free-running: {f_rho:.2e} {f_u:.2e} {f_T:.2e})")
            mixed[p] = {"value": updates / (ms_p * 1e-3), "ms_per_step": ms_p,
                        "transport_ms": kt_p[0] / max(kt_p[1], 1),
                        "speedup_vs_fp64": ms / ms_p, "e_rho": e_rho, "e_u": e_u, "e_T": e_T,
                        "free": {"e_rho": f_rho, "e_u": f_u, "e_T": f_T},
                        "after_steps": err_steps, "kn": cav.kn}
        del xs
        out["mixed"] = mixed
        if not args.no_kn_sweep:
            # the same errors at the workload's other Knudsen numbers
            sweep = {}
            for kn in (0.1, 10.0):
                if kn == cav.kn:
                    continue
                ck = cav.replace(kn=kn)
                xs = []
                ref = follow_run(ck, "fp64", err_steps, record=xs)
                row = {}
                for p in ("fp32", "bf16"):
                    st_p = follow_run(ck.replace(precision=p), p, err_steps, follow=xs)
                    e_rho, e_u, e_T = moment_errors(st_p, ref, cav.lid)
                    log(f"[bench] Kn {kn} {p} vs fp64 after {err_steps} steps: e_rho {e_rho:.2e} "
                        f"e_u {e_u:.2e} e_T {e_T:.2e}")
                    row[p] = {"e_rho": e_rho, "e_u": e_u, "e_T": e_T, "after_steps": err_steps}
                del xs
                sweep[f"kn_{kn:g}"] = row
            out["mixed_kn"] = sweep

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cav.replace(precision="fp64"), args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

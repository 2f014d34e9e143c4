"""Benchmark: FR-SG SSP-RK3 steps on one MI355X.

Workload: the 2D Euler shock-vortex problem, 256 x 128 quadrilateral elements,
FR degree 3 (4 x 4 Legendre-Gauss points), total-degree-4 Legendre chaos in two
random dimensions (15 modes), 5 x 5 Gauss nodes, L2 filter switched by the
modal-decay detector, positivity limiter, CFL 0.3; FP64.  Inputs are synthetic
(analytic initial data projected by the library) and resident in HBM before the
timed region.  One step = the whole hot path: three right-hand sides, the
stage combinations, the CFL reduction, the limiter after each stage and the
detector-switched filter plus limiter at the end of the step.

Prints one JSON line.  `value` = DOF-updates/s, DOF = S * M * E * N_sp stored
coefficients advanced by one full step.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FR-SG DOF-updates/s, FP64 vs FP32-mixed at stated L2 err; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
# algorithmic flops per DOF of one stage launch on the shock-vortex workload:
# right-hand side 195 (chaos expansion and projection 2 x 2 N_q = 100, face
# traces and Lax-Friedrichs fluxes 59, physical fluxes 12.5, derivative with the
# Radau corrections 24) plus the stage combination (2 in stage 1, 5 in stages
# 2-3: 4 on average)
SV_FLOP_PER_DOF_LAUNCH = 199.0
# symbol of the stage kernel for the shock-vortex sizes (15 modes, 25 nodes), per precision
# the stage kernel's instances for the headline workload (Lax-Friedrichs flux)
KERNEL_NAME = {"fp64": "k_stage2d<15, 25, double, 0>", "fp32": "k_stage2d<15, 25, float, 0>"}


def traffic_for(kernel, alg_bytes):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters (FETCH_SIZE, WRITE_SIZE,
    scaled by a copy kernel's readings), if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))["kernels"].get(kernel)
        src = os.path.join(ROOT, rec["source"])
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if digest != rec["source_sha256"]:
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(cfg_full):
    """Oracle timed on the host: one SSP-RK3 step of the same problem on a quarter-size mesh."""
    import numpy as np  # noqa: F401
    from oracle.initial import project_initial
    from oracle.problem import Problem
    from oracle.stepper import step
    from oracle.tables import build_tables
    from paper_2112_05946_amd import inputs

    cfg = inputs.small(cfg_full, cfg_full["nx"] // 2, cfg_full.get("ny", 1) // 2 if cfg_full.get("ny") else None)
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    u = project_initial(prob, cfg["ic"], (T, R))
    t0, c0 = time.perf_counter(), time.process_time()
    step(prob, u, None, (T, R))
    el, cpu = time.perf_counter() - t0, time.process_time() - c0
    dof = prob.S * R.M * prob.E * prob.nsp
    # threads actually used: process CPU time over wall time (NumPy's own threading)
    cores = max(1, int(round(cpu / el)))
    return {"value": dof / el, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": "1 SSP-RK3 step of the same problem on a %dx%d mesh (%d DOF), %.1f s wall, %.1f s CPU" %
                      (prob.nx, prob.ny, dof, el, cpu)}


def timed_steps(torch, sol, u, steps, warmup):
    """W untimed steps, then K timed steps bracketed by device synchronisation.

    The library launches on the default stream, which is torch's current stream
    here, so torch events bracket its kernels."""
    dt_used = torch.empty(1, dtype=torch.float64, device=u.device)
    flags = torch.empty(4 * sol.E, dtype=torch.uint8, device=u.device)
    for _ in range(warmup):
        sol.step(u, None, dt_used, flags)
    sol.sync()
    dts = torch.empty(steps, dtype=torch.float64, device=u.device)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    # K whole steps in one call: the CFL maximum of step n+1 is reduced in the
    # end-of-step epilogue of step n (the first step reduces it separately)
    sol.steps(u, steps, dts)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def pass_times(sol, u, steps):
    """Per-pass device times (events recorded on the library's stream around each launch)."""
    import torch
    dts = torch.empty(steps, dtype=torch.float64, device=u.device)
    sol.timing(True)
    sol.steps(u, steps, dts)
    passes = sol.timing_read()
    sol.timing(False)
    sol.sync()
    return passes


STAGES = ("stage1", "stage2", "stage3")


def roofline_for(passes, precision, kern=None, name="stage kernel (stages 1-3)"):
    """Roofline of the dominant kernel from the library's per-pass event timings.

    On the fused path the three SSP-RK3 stages are launches of one kernel (the
    stage kernel); its algorithmic bytes per launch are the per-stage figures
    (stage 1: read u, write w1; stages 2, 3: read u and w, write) averaged over
    its launches, divided by its average launch duration."""
    if all(k in passes for k in STAGES):
        launches = sum(passes[k][0] for k in STAGES)
        tot_ms = sum(passes[k][1] for k in STAGES)
        alg = sum(passes[k][0] * passes[k][2] for k in STAGES) / launches
        kern = kern or KERNEL_NAME[precision]
    else:
        dom = max(passes, key=lambda k: passes[k][1])
        launches, tot_ms, alg = passes[dom]
        name = dom
        kern = dom
    avg_s = tot_ms / launches / 1e3
    achieved = alg / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(kern, alg), "kernel": name,
            "alg_bytes_per_launch": alg, "avg_launch_ms": avg_s * 1e3, "launches": launches}


def alu_roofline(roof, flop_per_dof, dof, precision):
    """The same launches against the vector ALU peak: algorithmic flops per launch
    (right-hand side plus stage combination, per DOF) over the average launch time."""
    flops = flop_per_dof * dof
    achieved = flops / (roof["avg_launch_ms"] / 1e3) / 1e12
    peak = FP64_VECTOR_TFLOPS if precision == "fp64" else FP32_VECTOR_TFLOPS
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "flop_per_dof_per_launch": flop_per_dof}


# the triangle path's stage (trace pass + fused stage kernel) for the vortex workload
TRI_KERNEL = "k_stage_tri<3, 15, 25>"


def other_workloads(torch, Solver, inputs, steps, names=None):
    """DOF-updates/s of the other workloads (FP64, CFL steps in one call): the cache-resident 1D
    problems, with the Lasso filter, the HLL flux and the Bogacki-Shampine integrator, the
    shock-vortex problem with HLL, alone and with Bogacki-Shampine, the vortex on 32768
    perturbed triangles (p = 3, 15 modes, 25 nodes) and the shock-vortex problem (filter and
    limiter) on 16384 triangles."""
    out = {}
    for name in names or ("advection_sine", "burgers_sine", "sod_interface", "burgers_lasso", "sod_lasso", "sod_hll",
                          "shock_vortex_hll", "sod_hll_bs3", "shock_vortex_hll_bs3", "tri_vortex",
                          "tri_shock_vortex"):
        cfg = (inputs.tri_vortex(128) if name == "tri_vortex" else
               inputs.tri_shock_vortex(64) if name == "tri_shock_vortex" else inputs.CONFIGS[name])
        sol = Solver(cfg)
        u = sol.initial_state()
        dts = torch.empty(steps, dtype=torch.float64, device=u.device)
        sol.steps(u, 10, dts)
        sol.sync()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sol.steps(u, steps, dts)
        e1.record()
        torch.cuda.synchronize()
        sol.sync()
        ms = e0.elapsed_time(e1) / steps
        dof = int(sol.info["n_dof"])
        out[name] = {"dof": dof, "ms_per_step": ms, "dof_updates_per_s": dof / (ms / 1e3),
                     "shape": "%s, p=%d, %d modes, %d nodes, %d states" % (
                         "%d triangles" % sol.E if cfg.get("element") == "tri" else "%s el" % (
                         "%dx%d" % (cfg["nx"], cfg["ny"]) if cfg["equation"] == "euler2d" else str(cfg["nx"])),
                         cfg["p"], sol.shape[1], sol.info["n_nodes"], sol.shape[0])}
        if cfg.get("element") == "tri":
            passes = pass_times(sol, u, 20)
            out[name]["passes_ms_per_step"] = {k: v[1] / 20 for k, v in passes.items()}
            # counter traffic is on record for the vortex workload's stage only
            out[name]["roofline"] = roofline_for(passes, "fp64", TRI_KERNEL if name == "tri_vortex" else name,
                                                 "trace pass + stage kernel (stages 1-3)")
        sol.close()
    return out


def convergence_study():
    """The wave-propagation study of Sec. 5.1 on the library (RK4, dt = 0.1 dx, t = 2): errors of
    the expectation and orders per norm for N_p = 3 and 4 on 4..64 elements, the largest
    deviation from the paper's Tables 2-3, and the step time on 64 elements."""
    from paper_2112_05946_amd.convergence import NORMS, PAPER, wave_table
    out = {"t": 2.0, "integrator": "rk4", "dt": "0.1 dx"}
    for n in (3, 4):
        tab = wave_table(n)
        dev = max(abs(tab[nm][i] / PAPER[n][nm][i] - 1.0) for nm in NORMS for i in range(len(tab["dx"])))
        out["np%d" % n] = {"dx": tab["dx"], "l1": tab["l1"], "l1_order": tab["l1_order"],
                           "l2_order": tab["l2_order"], "linf_order": tab["linf_order"],
                           "max_rel_dev_from_paper": dev, "ms_per_step_64el": tab["ms_per_step"][-1],
                           "dof_64el": tab["dof"][-1]}
    return out


def precision_at_horizon(torch, Solver, cfg, rel, std):
    """FP32-mixed against FP64 at the workload's end time: both run the same number of CFL
    steps from the same initial state, as many as FP64 needs to reach t_end; relative L2
    distance of the modal state, of E[u] (mode 0) and of Std[u].  For scale, the same
    distances for FP64 started from the initial state perturbed by 1e-7 relative noise
    (seeded): how far FP32-level perturbations carry on this problem in FP64."""
    states, times = {}, {}
    nsteps = None
    for prec in ("fp64", "fp32", "fp64_perturbed"):
        sol = Solver(cfg, precision="fp32" if prec == "fp32" else "fp64")
        u = sol.initial_state()
        if prec == "fp64_perturbed":
            gen = torch.Generator(device=u.device)
            gen.manual_seed(0)
            u.mul_(1.0 + 1e-7 * torch.randn(u.shape, generator=gen, device=u.device, dtype=u.dtype))
        dts = torch.empty(10, dtype=torch.float64, device=u.device)
        t, n = 0.0, 0
        while (nsteps is None and t < cfg["t_end"]) or (nsteps is not None and n < nsteps):
            k = 10 if nsteps is None else min(10, nsteps - n)
            sol.steps(u, k, dts)
            t += float(dts[:k].sum())
            n += k
        sol.sync()
        nsteps = n
        states[prec], times[prec] = u, t
        sol.close()
    a, b, c = states["fp32"], states["fp64"], states["fp64_perturbed"]
    return {"t_end": cfg["t_end"], "steps": nsteps, "t_fp64": times["fp64"], "t_fp32": times["fp32"],
            "rel_l2_vs_fp64": rel(a, b), "rel_l2_mean_vs_fp64": rel(a[:, 0], b[:, 0]),
            "rel_l2_std_vs_fp64": rel(std(a), std(b)),
            "fp64_from_1e-7_perturbed_start": {"rel_l2": rel(c, b), "rel_l2_mean": rel(c[:, 0], b[:, 0]),
                                               "rel_l2_std": rel(std(c), std(b))}}


def adjoint_cost(torch, Solver, inputs):
    """Adjoint/forward cost on the 4096-element Burgers problem (p = 3, 9 modes, 16 nodes):
    500 steps at the CFL step of the initial state, held fixed."""
    from paper_2112_05946_amd.adjoint import AdjointSolve, mean_square
    cfg = inputs.BURGERS_ADJOINT
    n, k = int(cfg["n_steps"]), int(cfg["checkpoint_every"])
    sol = Solver(cfg)
    u0 = sol.initial_state()
    u = u0.clone()
    dtd, flags = sol.step(u)
    dt = float(dtd.item())
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    dts = torch.empty(1, dtype=torch.float64, device=u.device)
    fl = torch.empty(4 * sol.E, dtype=torch.uint8, device=u.device)

    def fwd():
        for _ in range(n):
            sol.step(u, dt, dts, fl)
    fwd()  # warm-up
    u.copy_(u0)
    t_fwd = timed(fwd) / n
    lam = torch.randn_like(u0)

    def adj():
        for _ in range(n):
            sol.adjoint_step(u0, flags, dt, lam)
    adj()
    t_adj = timed(adj) / n
    params = torch.tensor([0.0, float(cfg["gamma"]) if "gamma" in cfg else 1.4], dtype=torch.float64)

    def grad():
        x = u0.clone().requires_grad_(True)
        J = mean_square(AdjointSolve.apply(x, params, sol, n, dt, k), sol)
        J.backward()
    grad()
    t_grad = timed(grad) / n
    sol.close()
    dof = int(sol.info["n_dof"])
    return {"workload": "burgers_adjoint %d elements, p=%d, %d modes, %d nodes, %d DOF, %d steps, checkpoint every %d"
                        % (cfg["nx"], cfg["p"], sol.shape[1], sol.info["n_nodes"], dof, n, k),
            "forward_ms_per_step": t_fwd, "adjoint_step_ms": t_adj, "adjoint_over_forward": t_adj / t_fwd,
            "gradient_ms_per_step": t_grad, "gradient_over_forward": t_grad / t_fwd,
            "note": "gradient = forward with checkpoints + backward (segment recompute + adjoint steps), per step"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="shock_vortex")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed comparison run")
    ap.add_argument("--no-horizon", action="store_true",
                    help="skip the FP32-mixed against FP64 comparison at the workload's end time")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost run")
    ap.add_argument("--no-others", action="store_true", help="skip the 1D workloads")
    ap.add_argument("--no-convergence", action="store_true", help="skip the wave-propagation convergence study")
    ap.add_argument("--profile-workload", default=None,
                    help="run only this one of the other workloads (for profiling) and print its record")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the multi-GPU halo exchange is not built); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_05946_amd import inputs
    from paper_2112_05946_amd.binding import FrsgError, Solver

    torch.cuda.set_device(0)
    if args.profile_workload:
        print(json.dumps(other_workloads(torch, Solver, inputs, args.steps, [args.profile_workload])), flush=True)
        return
    cfg = inputs.CONFIGS[args.config]
    sol = Solver(cfg, precision=args.precision)
    u = sol.initial_state()
    ms, wall = timed_steps(torch, sol, u, args.steps, args.warmup)
    snapshot = u.clone()
    n_dof = int(sol.info["n_dof"])
    value = n_dof / (ms / 1e3)

    # per-pass device times over a second run of K steps (events around each launch)
    passes = pass_times(sol, u, args.steps)
    roofline = roofline_for(passes, args.precision)
    roof_alu = alu_roofline(roofline, SV_FLOP_PER_DOF_LAUNCH, int(sol.info["n_dof"]), args.precision) \
        if args.config == "shock_vortex" else None
    sol.close()

    # the other precision on the same workload: throughput and the L2 distance of
    # its state from this run's after the same W + K steps
    other = None
    if args.precision == "fp64" and not args.no_fp32:
        try:
            sol32 = Solver(cfg, precision="fp32")
        except FrsgError as e:  # FP32-mixed exists on the fused 2D Euler path only
            sol32 = None
            other = {"precision": "fp32_mixed", "skipped": str(e)}
    if other is None and args.precision == "fp64" and not args.no_fp32:
        u32 = sol32.initial_state()
        ms32, _ = timed_steps(torch, sol32, u32, args.steps, args.warmup)
        p32 = pass_times(sol32, u32.clone(), args.steps)
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        err = rel(u32, snapshot)
        # moments of the gPC expansion (orthonormal chaos): E[u] = mode 0, Std[u]^2 = sum of the others squared
        std = lambda x: torch.sqrt(torch.sum(x[:, 1:] ** 2, dim=1))
        other = {"precision": "fp32_mixed", "value": n_dof / (ms32 / 1e3), "ms_per_step": ms32,
                 "speedup_vs_fp64": ms / ms32, "rel_l2_vs_fp64": err,
                 "rel_l2_mean_vs_fp64": rel(u32[:, 0], snapshot[:, 0]),
                 "rel_l2_std_vs_fp64": rel(std(u32), std(snapshot)), "steps_compared": args.warmup + args.steps,
                 "roofline": roofline_for(p32, "fp32"),
                 "passes_ms_per_step": {k: v[1] / args.steps for k, v in p32.items()}}
        sol32.close()
        if not args.no_horizon:
            other["at_t_end"] = precision_at_horizon(torch, Solver, cfg, rel, std)

    adjoint = None if args.no_adjoint else adjoint_cost(torch, Solver, inputs)
    others = None if args.no_others else other_workloads(torch, Solver, inputs, 200)
    convergence = None if args.no_convergence else convergence_study()

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32 node loop, f64 state", "data": "synthetic",
        "config": {"workload": "%s %dx%d elements, p=%d, %d gPC modes (rdim %d), %d random nodes, %d states, "
                               "%d DOF" % (args.config, cfg["nx"], cfg.get("ny", 1), cfg["p"], sol.shape[1],
                                           cfg.get("rdim", 1), sol.info["n_nodes"], sol.shape[0], n_dof),
                   "precision": args.precision, "wall_s_timed": wall},
        "roofline": roofline,
        "roofline_alu": roof_alu,
        "passes_ms_per_step": {k: v[1] / args.steps for k, v in passes.items()},
        "fp32_mixed": other,
        "adjoint": adjoint,
        "other_workloads": others,
        "wave_propagation_convergence": convergence,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
KERNEL_NAME = {"fp64": "k_stage2d<15, 25, double, 0>", "fp32": "k_stage2d<15, 25, float, 0>",
               "bf16": "k_quad_stage<15, 25, 1, 0>"}
# arithmetic the path computes in, per precision
DTYPE = {"fp64": "f64", "fp32": "f32 node loop, f64 state", "bf16": "bf16 hi+lo transforms (f32 accumulation), f64 state"}


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


CPU_SAMPLE_MESH = (128, 64)  # quarter of the shock-vortex mesh: one oracle step is a few seconds of one core


def cpu_sample_child(nx, ny):
    """Child process: one oracle SSP-RK3 step of the shock-vortex problem on an nx x ny
    mesh; prints {"dof", "wall", "cpu"} as JSON.  Touches no GPU."""
    from oracle.initial import project_initial
    from oracle.problem import Problem
    from oracle.stepper import step
    from oracle.tables import build_tables
    from paper_2112_05946_amd import inputs

    cfg = inputs.small(inputs.SHOCK_VORTEX, nx, ny)
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    u = project_initial(prob, cfg["ic"], (T, R))
    t0, c0 = time.perf_counter(), time.process_time()
    step(prob, u, None, (T, R))
    el, cpu = time.perf_counter() - t0, time.process_time() - c0
    print(json.dumps({"dof": prob.S * R.M * prob.E * prob.nsp, "wall": el, "cpu": cpu}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The oracle timed on the host, before anything touches the GPU: one SSP-RK3 step of the
    shock-vortex problem on a 128 x 64 mesh in one process pinned to one thread, then the same
    sample in P concurrent single-threaded processes (P = the cores this process may run on, at
    most 16), whose aggregate DOF-updates/s is the all-cores figure."""
    import subprocess
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample-child", "%dx%d" % CPU_SAMPLE_MESH]

    def run(nproc):
        t0 = time.perf_counter()
        procs = [subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
                 for _ in range(nproc)]
        res = []
        for pr in procs:
            out, err = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError("oracle sample failed: " + err[-400:])
            res.append(json.loads(out.strip().splitlines()[-1]))
        return res, time.perf_counter() - t0

    one, _ = run(1)
    r1 = one[0]
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    P = max(1, min(16, ncores))
    many, wall = run(P)
    dof_all = sum(r["dof"] for r in many)
    sample = "1 oracle SSP-RK3 step of the shock-vortex problem on a %dx%d mesh (%d DOF) per process" % (
        CPU_SAMPLE_MESH + (r1["dof"],))
    return {"value": dof_all / wall, "unit": "DOF-updates/s", "cores": P, "kind": "oracle",
            "sample": sample + ", %d single-threaded processes at once, %.1f s wall, %.1f s CPU" % (
                P, wall, sum(r["cpu"] for r in many)),
            "cpu_model": cpu_model(), "host_cores_visible": ncores,
            "single_core": {"value": r1["dof"] / r1["wall"], "unit": "DOF-updates/s", "cores": 1,
                            "sample": sample + ", one process, %.1f s wall, %.1f s CPU" % (r1["wall"], r1["cpu"])}}


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Bandwidth of the library's streaming copy kernel (fr_sg_copy) on 1 GiB: 2 nbytes of HBM
    traffic per copy, timed with events on the stream it is enqueued on."""
    from paper_2112_05946_amd.binding import device_copy
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        device_copy(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        device_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    gbs = 2 * nbytes / (ms / 1e3) / 1e9
    return {"kernel": "k_copy (fr_sg_copy)", "bytes_per_copy": 2 * nbytes, "ms_per_copy": ms, "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "result_checked": ok}


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
        dts = torch.empty(max(steps, 10), dtype=torch.float64, device=u.device)
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


def _rel(torch):
    return lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _std(torch):
    # Std[u] of the orthonormal chaos expansion: the root sum of squares of the modes k >= 1
    return lambda x: torch.sqrt(torch.sum(x[:, 1:] ** 2, dim=1))


def precision_at_horizon(torch, Solver, cfg, precs):
    """Each reduced precision against FP64 at the workload's end time: every run takes the
    same number of CFL steps from the same initial state, as many as FP64 needs to reach
    t_end; relative L2 distance of the modal state, of E[u] (mode 0) and of Std[u].  For
    scale, the same distances for FP64 started from the initial state perturbed by 1e-7
    relative noise (seeded; then limited where the problem has the limiter): how far FP32-level
    perturbations carry on this problem."""
    rel, std = _rel(torch), _std(torch)
    states, times = {}, {}
    nsteps = None
    for prec in ("fp64",) + tuple(precs) + ("fp64_perturbed",):
        sol = Solver(cfg, precision="fp64" if prec == "fp64_perturbed" else prec)
        u = sol.initial_state()
        if prec == "fp64_perturbed":
            gen = torch.Generator(device=u.device)
            gen.manual_seed(0)
            u.mul_(1.0 + 1e-7 * torch.randn(u.shape, generator=gen, device=u.device, dtype=u.dtype))
            if cfg.get("limiter"):
                # the projected data leaves some nodal pressures near zero (Gibbs points of the
                # interface); the noise can push them below, so the start is limited first
                sol.limit(u)
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
    b = states["fp64"]
    out = {"t_end": cfg["t_end"], "steps": nsteps, "t_fp64": times["fp64"]}
    for prec in tuple(precs) + ("fp64_perturbed",):
        a = states[prec]
        out[prec] = {"t": times[prec], "rel_l2_vs_fp64": rel(a, b), "rel_l2_mean_vs_fp64": rel(a[:, 0], b[:, 0]),
                     "rel_l2_std_vs_fp64": rel(std(a), std(b))}
    return out


def reduced_precisions(torch, Solver, FrsgError, cfg, ms64, ref_state, steps, warmup, horizon=True,
                       kernel_names=None):
    """FP32-mixed and BF16-split on one workload: throughput, speed-up over FP64, the distance
    of the state from FP64's after the same W + K steps, the dominant kernel's roofline, and
    the distances at the end time.  A precision the workload's path does not provide is
    reported as skipped with the library's reason."""
    rel, std = _rel(torch), _std(torch)
    out, ran = {}, []
    for prec in ("fp32", "bf16"):
        try:
            sol = Solver(cfg, precision=prec)
        except FrsgError as e:
            out[prec] = {"skipped": str(e)}
            continue
        u = sol.initial_state()
        ms, _ = timed_steps(torch, sol, u, steps, warmup)
        passes = pass_times(sol, u.clone(), steps)
        n_dof = int(sol.info["n_dof"])
        rec = {"value": n_dof / (ms / 1e3), "ms_per_step": ms, "speedup_vs_fp64": ms64 / ms,
               "rel_l2_vs_fp64": rel(u, ref_state), "rel_l2_mean_vs_fp64": rel(u[:, 0], ref_state[:, 0]),
               "rel_l2_std_vs_fp64": rel(std(u), std(ref_state)), "steps_compared": warmup + steps,
               "passes_ms_per_step": {k: v[1] / steps for k, v in passes.items()}}
        if kernel_names and prec in kernel_names:
            rec["roofline"] = roofline_for(passes, prec, kernel_names[prec])
        else:
            rec["roofline"] = roofline_for(passes, prec, "-")
        out[prec] = rec
        ran.append(prec)
        sol.close()
    if horizon and ran:
        out["at_t_end"] = precision_at_horizon(torch, Solver, cfg, ran)
    return out


def precision_1d(torch, Solver, FrsgError, inputs, steps=200, warmup=10):
    """The 1D workloads (Burgers, Sod) in FP64, FP32-mixed and BF16-split: ms per step and the
    distances from FP64 at the end time.  They are cache resident, so their step time is
    launch-bound and the reduced precisions are there for their accuracy, not their speed."""
    out = {}
    for name in ("burgers_sine", "sod_interface"):
        cfg = inputs.CONFIGS[name]
        sol = Solver(cfg)
        u = sol.initial_state()
        ms, _ = timed_steps(torch, sol, u, steps, warmup)
        ref = u.clone()
        sol.close()
        rec = {"fp64_ms_per_step": ms, "dof": int(sol.info["n_dof"]),
               "fp64_dof_updates_per_s": int(sol.info["n_dof"]) / (ms / 1e3)}
        rec.update(reduced_precisions(torch, Solver, FrsgError, cfg, ms, ref, steps, warmup))
        out[name] = rec
    return out


def adjoint_cost(torch, Solver, inputs):
    """Adjoint/forward cost on the 4096-element Burgers problem (p = 3, 9 modes, 16 nodes):
    500 steps at the CFL step of the initial state, held fixed, in FP64 and FP32-mixed; the
    FP32-mixed gradient's distance from the FP64 one."""
    from paper_2112_05946_amd.adjoint import AdjointSolve, mean_square
    cfg = inputs.BURGERS_ADJOINT
    n, k = int(cfg["n_steps"]), int(cfg["checkpoint_every"])
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    res, grads = {}, {}
    for prec in ("fp64", "fp32"):
        sol = Solver(cfg, precision=prec)
        u0 = sol.initial_state()
        u = u0.clone()
        dtd, flags = sol.step(u)
        dt = float(dtd.item())
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
        # the adjoint step from kept stage states (what the checkpointed gradient uses)
        w1, w2 = torch.empty_like(u0), torch.empty_like(u0)
        sol.step_stages(u0.clone(), w1, w2, dt)

        def adj_kept():
            for _ in range(n):
                sol.adjoint_step_stages(u0, w1, w2, flags, dt, lam)
        adj_kept()
        t_adj_kept = timed(adj_kept) / n
        params = torch.tensor([0.0, 1.4], dtype=torch.float64)
        box = {}

        def grad():
            x = u0.clone().requires_grad_(True)
            J = mean_square(AdjointSolve.apply(x, params, sol, n, dt, k), sol)
            J.backward()
            box["g"] = x.grad
        grad()
        t_grad = timed(grad) / n
        grads[prec] = box["g"]

        # every step's states kept from the forward run (k = 0): nothing recomputed
        def grad_all():
            x = u0.clone().requires_grad_(True)
            J = mean_square(AdjointSolve.apply(x, params, sol, n, dt, 0), sol)
            J.backward()
            box["g0"] = x.grad
        grad_all()
        t_grad_all = timed(grad_all) / n
        dof = int(sol.info["n_dof"])
        res[prec] = {"forward_ms_per_step": t_fwd, "adjoint_step_ms": t_adj, "adjoint_over_forward": t_adj / t_fwd,
                     "adjoint_step_from_kept_stages_ms": t_adj_kept,
                     "gradient_ms_per_step": t_grad, "gradient_over_forward": t_grad / t_fwd,
                     "gradient_keep_all_ms_per_step": t_grad_all, "gradient_keep_all_over_forward": t_grad_all / t_fwd,
                     "gradient_keep_all_equal": bool(torch.equal(box["g0"], box["g"])),
                     "gradient_keep_all_state_bytes": 3 * n * int(u0.numel()) * 8}
        shape = (sol.shape[1], sol.info["n_nodes"])
        sol.close()
    res["fp32"]["gradient_rel_l2_vs_fp64"] = _rel(torch)(grads["fp32"], grads["fp64"])
    res["fp32"]["speedup_vs_fp64_gradient"] = res["fp64"]["gradient_ms_per_step"] / res["fp32"]["gradient_ms_per_step"]
    out = {"workload": "burgers_adjoint %d elements, p=%d, %d modes, %d nodes, %d DOF, %d steps, checkpoint every %d"
                       % (cfg["nx"], cfg["p"], shape[0], shape[1], dof, n, k),
           "note": "gradient = forward with checkpoints + backward (segment recompute keeping the stage states + adjoint steps from them), per step; "
                   "gradient_keep_all: every step's start and stage states kept from the forward run (3 states per step), adjoint steps only"}
    out.update(res["fp64"])
    out["fp32_mixed"] = res["fp32"]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="shock_vortex")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the FP32-mixed and BF16-split runs (c4 and the 1D workloads)")
    ap.add_argument("--no-horizon", action="store_true",
                    help="skip the reduced-precision against FP64 comparison at the workload's end time")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost run")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-convergence", action="store_true", help="skip the wave-propagation convergence study")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-kernel bandwidth reference")
    ap.add_argument("--profile-workload", default=None,
                    help="run only this one of the other workloads (for profiling) and print its record")
    ap.add_argument("--cpu-sample-child", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_sample_child:
        nx, ny = (int(v) for v in args.cpu_sample_child.split("x"))
        cpu_sample_child(nx, ny)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the multi-GPU halo exchange is not built); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the oracle's host timing runs in child processes before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.profile_workload:
        cpu = cpu_baseline()

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
    # the same K-step call five more times, the state marching on: the spread of the timing
    repeats = [timed_steps(torch, sol, u, args.steps, 0)[0] for _ in range(5)]

    # per-pass device times over a second run of K steps (events around each launch)
    passes = pass_times(sol, u, args.steps)
    roofline = roofline_for(passes, args.precision)
    roof_alu = alu_roofline(roofline, SV_FLOP_PER_DOF_LAUNCH, int(sol.info["n_dof"]), args.precision) \
        if args.config == "shock_vortex" and args.precision != "bf16" else None
    sol.close()

    copy = None if args.no_copy else copy_bandwidth(torch)
    if copy:  # the same launches against the copy kernel's measured bandwidth
        roofline["copy_GBs"] = copy["achieved"]
        roofline["frac_of_copy"] = roofline["achieved"] / copy["achieved"]
    reduced = None
    if args.precision == "fp64" and not args.no_precisions:
        reduced = reduced_precisions(torch, Solver, FrsgError, cfg, ms, snapshot, args.steps, args.warmup,
                                     horizon=not args.no_horizon, kernel_names=KERNEL_NAME)
    prec1d = None if args.no_precisions else precision_1d(torch, Solver, FrsgError, inputs)
    adjoint = None if args.no_adjoint else adjoint_cost(torch, Solver, inputs)
    others = None if args.no_others else other_workloads(torch, Solver, inputs, 200)
    convergence = None if args.no_convergence else convergence_study()

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": "%s %dx%d elements, p=%d, %d gPC modes (rdim %d), %d random nodes, %d states, "
                               "%d DOF" % (args.config, cfg["nx"], cfg.get("ny", 1), cfg["p"], sol.shape[1],
                                           cfg.get("rdim", 1), sol.info["n_nodes"], sol.shape[0], n_dof),
                   "precision": args.precision, "wall_s_timed": wall},
        "roofline": roofline,
        "roofline_alu": roof_alu,
        "ms_per_step_repeats": {"runs": repeats, "median": sorted(repeats)[len(repeats) // 2],
                                "min": min(repeats), "max": max(repeats)},
        "passes_ms_per_step": {k: v[1] / args.steps for k, v in passes.items()},
        "copy_bandwidth": copy,
        "reduced_precision": reduced,
        "precision_1d": prec1d,
        "adjoint": adjoint,
        "other_workloads": others,
        "wave_propagation_convergence": convergence,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

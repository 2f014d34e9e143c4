"""BF16-split precision (FRSG_BF16_SPLIT) and the FP64 matrix-core path of the 2D
Euler stage kernel, against the FP64 oracle.

In BF16-split every operand of the chaos expansion and projection is split into
a high and a low bfloat16 part, x = hi + lo + d with |d| <= 2^-16 |x| (each
part carries 8 significant bits and the low part rounds the remainder of the
high one), and the matrix cores form hi*hi + hi*lo + lo*hi in FP32, dropping
lo*lo (also <= 2^-16 of the product).  A transform therefore has a relative
error of order 2^-16 = 1.5e-5 of its largest terms; the right-hand side, a
difference of fluxes over the element width, keeps that order up to the
cancellation of its terms (a factor of a few), so its bar is 1e-4 relative L2.
A step moves the state by dt R, with dt |R| / |u| <= 0.1 here, which gives the
step bar 1e-5.  Switch decisions (FP64, on the BF16-perturbed state) may differ
from the oracle's only where the oracle's own margin is below 1e-3.

The mean mode's projection is accumulated in FP64, and every face flux is formed
from bit-identical traces on its two sides, so the total of each conserved
variable's mean mode over a periodic mesh changes only by the FP32 rounding of
the nodal residuals: at most 1e-6 of that total per step is asserted.

The FP64 matrix-core path (FP64 problems on meshes that the VALU kernel's 4 x 2
tiles do not cover, nx = 2 mod 4) is held to the FP64 parity bar.
"""

import numpy as np
import pytest

from gpu_util import (ELEM_RTOL, RTOL_FP64, announce, check_flags, elem_max_rel, oracle_for, rel_l2, solver_for,
                      to_dev, to_np)
from oracle import fr as ofr
from oracle import stabilize as ost
from oracle import stepper as ostep
from oracle.initial import project_initial
from oracle.problem import Problem
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

BF16_RHS_TOL = 1e-4
BF16_STEP_TOL = 1e-5
BF16_DT_TOL = 1e-5
BF16_TIE = 1e-3

CASES = [
    ("sv_16x8", inputs.small(inputs.SHOCK_VORTEX, 16, 8)),
    ("sv_6x4_tile_rows", inputs.small(inputs.SHOCK_VORTEX, 6, 4)),
    ("sv_periodic_m10q16", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 8), gpc_order=3, nq1d=4,
                                bc=["periodic"] * 4, sensor="always", filter="l2")),
    ("sv_m6q9_hll", dict(inputs.small(inputs.SHOCK_VORTEX, 10, 6), gpc_order=2, nq1d=3, flux="hll")),
    ("sv_m3q4", dict(inputs.small(inputs.SHOCK_VORTEX, 4, 2), gpc_order=1, nq1d=2, rdim=2)),
]


def _flags_close(prob, T, R, gflags, rflags, record, tie):
    for pas in range(4):
        bad = np.nonzero(gflags[pas] != rflags[pas])[0]
        if len(bad) == 0:
            continue
        if pas == 2:
            se, thr = ost.sensor_margin(prob, T, R, record[pas])
            rel = np.abs(se[bad] - thr) / thr
        else:
            m, scale = ost.limiter_margin(prob, T, R, record[pas])
            rel = np.abs(m[bad]) / scale[bad]
        assert np.all(rel <= tie), ("decision differs away from a tie", pas, bad[:5], rel[:5])


@pytest.mark.parametrize("label,cfg", CASES)
@pytest.mark.parametrize("seed", [0, 1])
def test_bf16_rhs_error(label, cfg, seed):
    announce("bf16_rhs", label, seed)
    prob, (T, R) = oracle_for(cfg)
    u = inputs.fuzz_euler(2, R.M, prob.E, 16, seed)
    ref = ofr.rhs(prob, T, R, u)
    sol = solver_for(cfg, "bf16")
    got = to_np(sol.rhs(to_dev(u)))
    sol.sync()
    err = rel_l2(got, ref)
    print("[bf16 rhs]", label, seed, "%.2e" % err, flush=True)
    assert err < BF16_RHS_TOL


@pytest.mark.parametrize("label,cfg", CASES)
def test_bf16_steps_error(label, cfg):
    announce("bf16_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    for i in range(4):
        # one oracle step from the GPU's own state: the per-step error, not its growth
        start = to_np(ud)
        rec = []
        ref, rdt, rfl = ostep.step(prob, start, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        gdt = float(to_np(dtd)[0])
        assert abs(gdt / rdt - 1.0) < BF16_DT_TOL, (i, gdt, rdt)
        err = rel_l2(to_np(ud), ref)
        print("[bf16 step]", label, i, "%.2e" % err, flush=True)
        assert err < BF16_STEP_TOL, (i, err)
        _flags_close(prob, T, R, to_np(flags).reshape(4, prob.E), rfl, rec, BF16_TIE)


def test_bf16_full_size_step_and_steps():
    """The shock-vortex workload at full size: one step from the initial state within the
    step bar on 16 sampled patches (the oracle's step of each element's 7 x 7 patch), and
    a four-step call equal to four single steps up to the time-step rounding."""
    import torch
    from gpu_util import quad_patch
    cfg = inputs.SHOCK_VORTEX
    announce("bf16_full_size")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    dtd, flags = sol.step(ud)
    sol.sync()
    got = to_np(ud)
    gdt = float(to_np(dtd)[0])
    assert abs(gdt / ostep.cfl_dt(prob, T, R, u0) - 1.0) < BF16_DT_TOL
    rng = np.random.default_rng(9)
    picks = [(0, 0), (255, 127), (32, 64), (64, 64), (31, 60)] + \
        [(int(a), int(b)) for a, b in zip(rng.integers(0, 256, 11), rng.integers(0, 128, 11))]
    g, w = [], []
    for (cx, cy) in picks:
        pcfg, ids, c = quad_patch(cfg, cx, cy)
        ref, _, _ = ostep.step(Problem.from_config(pcfg), u0[:, :, ids].copy(), gdt, (T, R))
        g.append(got[:, :, cy * cfg["nx"] + cx])
        w.append(ref[:, :, c])
    err = rel_l2(np.array(g), np.array(w))
    print("[bf16 full size] sampled step error %.2e" % err, flush=True)
    assert err < BF16_STEP_TOL
    u4 = to_dev(u0)
    d4 = torch.empty(4, dtype=torch.float64, device=u4.device)
    sol.steps(u4, 4, dt_used=d4)
    for _ in range(3):
        sol.step(ud)
    sol.sync()
    assert rel_l2(to_np(u4), to_np(ud)) < 1e-10


def test_bf16_conserves_the_mean_mode():
    """Periodic mesh, no limiter, filter on every element: the mesh total of every
    variable's mean mode (sum_e J sum_j w_j u_{e,j,0}) moves by at most 1e-6 of the mesh
    integral of its magnitude (sum_e J sum_j w_j |u_{e,j,0}|) per step (the y-momentum
    total itself is near zero, so it is measured against that scale)."""
    cfg = dict(inputs.small(inputs.SHOCK_VORTEX, 8, 8), gpc_order=3, nq1d=4, bc=["periodic"] * 4,
               sensor="always", filter="l2", limiter=False)
    announce("bf16_conservation")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    w2 = np.outer(T.w, T.w).ravel()
    J = prob.dx * prob.dy / 4.0

    def totals(u):
        return J * np.einsum("sej,j->s", u[:, 0], w2)

    t0 = totals(u0)
    scale = J * np.einsum("sej,j->s", np.abs(u0[:, 0]), w2)
    for i in range(6):
        sol.step(ud)
        sol.sync()
        t = totals(to_np(ud))
        drift = np.abs(t - t0) / scale
        print("[bf16 conservation] step", i, drift, flush=True)
        assert np.all(drift <= 1e-6 * (i + 1)), (i, drift)


@pytest.mark.parametrize("label,cfg", [("sv_6x4", inputs.small(inputs.SHOCK_VORTEX, 6, 4)),
                                       ("sv_10x6_periodic_m10q16",
                                        dict(inputs.small(inputs.SHOCK_VORTEX, 10, 6), gpc_order=3, nq1d=4,
                                             bc=["periodic"] * 4, sensor="always", filter="l2")),
                                       ("sv_6x4_m6q9_hll", dict(inputs.small(inputs.SHOCK_VORTEX, 6, 4), gpc_order=2,
                                                                nq1d=3, flux="hll"))])
def test_fp64_matrix_core_path_parity(label, cfg):
    """FP64 on the matrix-core kernel: RHS of a fuzzed state, six steps and the limiter on
    near-vacuum states at the FP64 parity bar, switch decisions equal up to ties."""
    announce("fp64_mfma", label)
    prob, (T, R) = oracle_for(cfg)
    u = inputs.fuzz_euler(2, R.M, prob.E, 16, 4)
    sol = solver_for(cfg)
    got = to_np(sol.rhs(to_dev(u)))
    sol.sync()
    assert rel_l2(got, ofr.rhs(prob, T, R, u)) < RTOL_FP64
    for start, dt in (("initial", None), ("vacuum", 1e-5)):
        if start == "initial":
            v = project_initial(prob, cfg["ic"], (T, R))
        else:
            v, _ = ost.limit(prob, T, R, inputs.fuzz_euler(2, R.M, prob.E, 16, 6, vacuum_frac=0.2))
        ud = to_dev(v)
        for i in range(3):
            rec = []
            v, rdt, rfl = ostep.step(prob, v, dt, (T, R), record=rec)
            dtd, flags = sol.step(ud, dt)
            sol.sync()
            assert abs(float(to_np(dtd)[0]) / rdt - 1.0) < 1e-13
            check_flags(prob, T, R, to_np(flags).reshape(4, prob.E), rfl, rec)
            gv = to_np(ud)
            assert rel_l2(gv, v) < RTOL_FP64, (start, i, rel_l2(gv, v))
            assert elem_max_rel(gv, v) < ELEM_RTOL

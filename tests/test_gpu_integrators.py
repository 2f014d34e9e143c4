"""The paper's explicit integrators (RK4, Bogacki-Shampine 3(2), Tsitouras
5(4)) at the CFL step on the GPU against the oracle: every right-hand-side
path (fused 1D, multi-pass 1D, fused 2D, generic 2D), with filters, the
limiter and the HLL flux."""

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    ("burgers_rk4_fused", dict(inputs.small(inputs.BURGERS, 24), integrator="rk4")),
    ("burgers_tsit5_multipass", dict(inputs.small(inputs.BURGERS, 10), integrator="tsit5", nq1d=100)),
    ("sod_bs3_hll_fused", dict(inputs.small(inputs.SOD, 40), integrator="bs3", flux="hll")),
    ("sod_tsit5_lasso", dict(inputs.small(inputs.SOD, 30), integrator="tsit5", filter="lasso", sensor="always")),
    ("sv_bs3_hll_fused", dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), integrator="bs3", flux="hll")),
    ("sv_tsit5_fused", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 6), integrator="tsit5")),
    ("sv_rk4_generic", dict(inputs.small(inputs.SHOCK_VORTEX, 7, 5), integrator="rk4")),
    ("advection_tsit5", dict(inputs.small(inputs.ADVECTION, 16), integrator="tsit5")),
]


@pytest.mark.parametrize("label,cfg", CASES)
def test_integrator_steps_match_oracle(label, cfg):
    announce("integrator_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u0)
    ref = u0.copy()
    for i in range(3):
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R))
        dtd, flags = sol.step(ud)
        sol.sync()
        g = to_np(flags).reshape(4, prob.E)
        assert abs(to_np(dtd)[0] - rdt) <= 1e-13 * rdt
        assert np.array_equal(g[2], rflags[2]) and np.array_equal(g[3], rflags[3])
        assert np.array_equal(g[0], rflags[0]) and not g[1].any()
        err = rel_l2(to_np(ud), ref)
        print("[rk] %s step %d rel-L2 %.2e" % (label, i, err), flush=True)
        assert err < RTOL_FP64


@pytest.mark.parametrize("label,cfg,dt", [
    ("sod_rk4_fixed", dict(inputs.small(inputs.SOD, 24), integrator="rk4"), 2e-4),
    ("sv_bs3_fixed", dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), integrator="bs3"), 1e-3),
])
def test_integrator_fixed_dt(label, cfg, dt):
    """A tableau step at a given dt (the first stage kernel publishes it instead of
    deriving it from the CFL maximum) on the fused 1D and 2D paths."""
    announce("integrator_fixed_dt", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u0)
    ref = u0.copy()
    for _ in range(2):
        ref, rdt, rflags = ostep.step(prob, ref, dt, (T, R))
        dtd, flags = sol.step(ud, dt)
        sol.sync()
        assert to_np(dtd)[0] == dt and rdt == dt
        g = to_np(flags).reshape(4, prob.E)
        assert np.array_equal(g[0], rflags[0]) and np.array_equal(g[3], rflags[3]) and not g[1].any()
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_integrator_chained_steps():
    import torch
    cfg = dict(inputs.small(inputs.SOD, 24), integrator="bs3", flux="hll")
    announce("integrator_chained")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref = u0.copy()
    rdts = []
    for _ in range(6):
        ref, rdt, _ = ostep.step(prob, ref, None, (T, R))
        rdts.append(rdt)
    sol = solver_for(cfg)
    ud = to_dev(u0)
    dts = torch.empty(6, dtype=torch.float64, device=ud.device)
    sol.steps(ud, 6, dts)
    sol.sync()
    assert np.allclose(to_np(dts), rdts, rtol=1e-13, atol=0)
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_integrator_chained_steps_2d():
    """fr_sg_steps on the fused 2D path: each stage kernel forms the next stage state in its
    epilogue and writes its face traces for the next launch; later steps take the first
    stage's traces and CFL maximum from the previous step's last launch."""
    import torch
    cfg = dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), integrator="rk4", flux="hll")
    announce("integrator_chained_2d")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref = u0.copy()
    rdts = []
    for _ in range(4):
        ref, rdt, _ = ostep.step(prob, ref, None, (T, R))
        rdts.append(rdt)
    sol = solver_for(cfg)
    ud = to_dev(u0)
    dts = torch.empty(4, dtype=torch.float64, device=ud.device)
    sol.steps(ud, 4, dts)
    sol.sync()
    assert np.allclose(to_np(dts), rdts, rtol=1e-13, atol=0)
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_integrator_full_size_shock_vortex_step():
    """The paper's setting for the 2D problem (Table 6): HLL flux, Bogacki-Shampine."""
    cfg = dict(inputs.SHOCK_VORTEX, integrator="bs3", flux="hll")
    announce("integrator_full_size")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref, rdt, _ = ostep.step(prob, u0, None, (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u0)
    dtd, _ = sol.step(ud)
    sol.sync()
    assert abs(to_np(dtd)[0] - rdt) <= 1e-13 * rdt
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_integrator_has_no_adjoint():
    from paper_2112_05946_amd.binding import FrsgError
    cfg = dict(inputs.small(inputs.BURGERS, 8), integrator="rk4")
    sol = solver_for(cfg)
    u = sol.initial_state()
    flags = sol.step(u.clone(), 1e-4)[1]
    with pytest.raises(FrsgError) as ei:
        sol.adjoint_step(u, flags, 1e-4, u.clone())
    assert ei.value.status == -2


@pytest.mark.parametrize("seed", [3, 4])
def test_fused_limit_pass_matches_oracle(seed):
    """fr_sg_limit on the fused 2D path (element-wise pass with the stage kernel's
    lane layout), near-vacuum elements so that the limiter acts."""
    import torch
    from oracle import stabilize as ost
    cfg = inputs.small(inputs.SHOCK_VORTEX, 12, 8)
    announce("fused_limit_pass", seed)
    prob, (T, R) = oracle_for(cfg)
    u = inputs.fuzz_euler(2, R.M, prob.E, prob.nsp, seed, vacuum_frac=0.25)
    ref, rflags = ost.limit(prob, T, R, u)
    assert rflags.sum() > 0
    sol = solver_for(cfg)
    ud = to_dev(u)
    flags = torch.zeros(prob.E, dtype=torch.uint8, device=ud.device)
    sol.limit(ud, flags)
    sol.sync()
    assert np.array_equal(to_np(flags).astype(bool), rflags)
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


# the reduced precisions under the tableau integrators: every right-hand side of the
# tableau runs in the precision's arithmetic, the combinations stay FP64; the step bars of
# the precision tests hold (a step still moves the state by dt sum_i b_i K_i with
# dt |K| / |u| <= 0.1): FP32-mixed 1e-6, BF16-split 1e-5 per step
REDUCED = [
    ("sod_rk4_fp32", dict(inputs.small(inputs.SOD, 40), integrator="rk4"), "fp32", 1e-6),
    ("burgers_bs3_bf16", dict(inputs.small(inputs.BURGERS, 24), integrator="bs3"), "bf16", 1e-5),
    ("sv_bs3_fp32", dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), integrator="bs3"), "fp32", 1e-6),
    ("sv_rk4_bf16", dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), integrator="rk4"), "bf16", 1e-5),
]


@pytest.mark.parametrize("label,cfg,prec,bar", REDUCED)
def test_integrators_in_reduced_precision(label, cfg, prec, bar):
    from oracle import stabilize as ost
    announce("integrator_reduced", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, prec)
    ud = to_dev(u0)
    ref = u0.copy()
    for i in range(3):
        rec = []
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= bar * rdt
        g = to_np(flags).reshape(4, prob.E)
        bad = np.nonzero(g[2] != rflags[2])[0]
        if len(bad):  # a filter decision may differ only where the oracle's margin is tiny
            se, thr = ost.sensor_margin(prob, T, R, rec[2])
            assert np.all(np.abs(se[bad] - thr) / thr <= 100 * bar)
        err = rel_l2(to_np(ud), ref)
        print("[rk %s] %s step %d rel-L2 %.2e" % (prec, label, i, err), flush=True)
        assert err < bar * (i + 1)

"""FP32-mixed precision on the fused 1D stage kernel (Burgers, Euler) and on the
fused adjoint kernel, against the FP64 oracle; mean-mode conservation of the
FP64, FP32-mixed and BF16-split paths on periodic meshes.

FP32 changes the result, so the bars are error bounds, set as for the 2D
FP32-mixed path: the node loop rounds every operand to FP32 (unit roundoff
6e-8), a right-hand side is a difference of fluxes over the element width whose
cancellation costs a factor of tens at most, so its relative L2 error stays
below FP32_RHS_TOL = 1e-4; a step moves the state by dt R with dt |R| / |u| at
most 0.1, which gives FP32_STEP_TOL = 1e-6 per step.  The adjoint step is
lam_n = B^T lam with B = I + dt R' + ..., whose FP32 part is dt R'^T lam; dt |R'|
is of the order of the CFL number (0.3), so the FP32 rounding of that part keeps
lam_n within FP32_ADJ_TOL = 1e-5 relative L2 of the oracle's.  Switch decisions
(FP64, on the FP32-perturbed state) may differ from the oracle's only where the
oracle's own margin is below FP32_TIE.

Conservation: with periodic sides the exact scheme keeps sum_e J sum_j w_j
u_{e,j,0} of every conserved variable (the correction derivatives integrate to
-1 and +1 and the modified derivative matrix to 0; the filter and the limiter
keep element means).  In floating point each element's mean residual is a sum
of n + 2 terms no larger than the largest flux magnitude F, each rounded once
with unit roundoff u; summed over the three stages and the E
elements, with a safety factor 8, one step moves the total by at most
3 E dt 8 (n + 2) u F (times the face length dx + dy in 2D).  The tests assert
that bound with u = 2^-53 (FP64) and u = 2^-24 (FP32-mixed, and BF16-split,
whose bfloat16 transforms perturb the nodal values but not the balance of the
fluxes formed from them)."""

import numpy as np
import pytest

from gpu_util import announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import adjoint as oadj
from oracle import fr as ofr
from oracle import stabilize as ost
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

FP32_RHS_TOL = 1e-4
FP32_STEP_TOL = 1e-6
FP32_DT_TOL = 1e-6
FP32_ADJ_TOL = 1e-5
FP32_TIE = 1e-5

BURGERS = inputs.small(inputs.BURGERS, 64)
BURGERS_RAGGED = inputs.small(inputs.BURGERS, 37)
SOD = inputs.small(inputs.SOD, 96)
SOD_HLL = inputs.small(inputs.SOD_HLL, 50)
ADVECTION = dict(inputs.small(inputs.ADVECTION, 13), adv_speed=0.7, filter="exp", alpha=36.0, s=8.0,
                 sensor="detector", s0=-2.0 * np.log10(3.0), kappa=4.0)


def _state(cfg, prob, T, R, seed):
    """Projected initial data with random modal content on every third element
    (so that the detector fires on some elements)."""
    u = project_initial(prob, cfg["ic"], (T, R))
    if prob.S == 1:
        u[:, :, ::3] += inputs.fuzz_scalar(R.M, prob.E, T.n, seed, scale=0.3)[:, :, ::3]
    return u


def _flags_close(prob, T, R, gflags, rflags, record):
    diffs = 0
    for pas in range(4):
        bad = np.nonzero(gflags[pas] != rflags[pas])[0]
        if len(bad) == 0:
            continue
        diffs += len(bad)
        if pas == 2:
            se, thr = ost.sensor_margin(prob, T, R, record[pas])
            rel = np.abs(se[bad] - thr) / thr
        else:
            m, scale = ost.limiter_margin(prob, T, R, record[pas])
            rel = np.abs(m[bad]) / scale[bad]
        assert np.all(rel <= FP32_TIE), ("decision differs away from a tie", pas, bad[:5], rel[:5])
    return diffs


@pytest.mark.parametrize("label,cfg", [("burgers", BURGERS), ("burgers_ragged", BURGERS_RAGGED), ("sod", SOD),
                                       ("sod_hll", SOD_HLL)])
@pytest.mark.parametrize("seed", [0, 1])
def test_fp32_1d_rhs_error(label, cfg, seed):
    announce("fp32_1d_rhs", label, seed)
    prob, (T, R) = oracle_for(cfg)
    if prob.S == 1:
        u = inputs.fuzz_scalar(R.M, prob.E, T.n, seed, offset=1.0)
    else:
        u = inputs.fuzz_euler(1, R.M, prob.E, T.n, seed)
    ref = ofr.rhs(prob, T, R, u)
    sol = solver_for(cfg, "fp32")
    got = to_np(sol.rhs(to_dev(u)))
    sol.sync()
    err = rel_l2(got, ref)
    print("[fp32 1d] %s rhs rel L2 error %.3e" % (label, err), flush=True)
    assert err < FP32_RHS_TOL


@pytest.mark.parametrize("label,cfg", [("burgers", BURGERS), ("sod", SOD), ("sod_hll", SOD_HLL),
                                       ("sod_lasso", inputs.small(inputs.SOD_LASSO, 40))])
def test_fp32_1d_steps_error(label, cfg):
    """Four CFL steps of the fused 1D kernel in FP32-mixed against the oracle's FP64
    steps, with the detector, the filter and (Sod) the limiter in the epilogue."""
    announce("fp32_1d_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = _state(cfg, prob, T, R, 3)
    sol = solver_for(cfg, "fp32")
    ud = to_dev(u0)
    ref = u0.copy()
    diffs = fired = 0
    for i in range(4):
        rec = []
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= FP32_DT_TOL * rdt
        gfl = to_np(flags).reshape(4, prob.E)
        diffs += _flags_close(prob, T, R, gfl, rflags, rec)
        fired += int(rflags[2].sum())
        err = rel_l2(to_np(ud), ref)
        print("[fp32 1d] %s step %d rel L2 error %.3e, decisions differing %d" % (label, i, err, diffs), flush=True)
        assert err < FP32_STEP_TOL * (i + 1)
    assert fired > 0  # the filter acted


def test_fp32_1d_limiter_acts():
    """Sod with near-vacuum elements: the FP64 limiter of the FP32 kernel acts and
    keeps every element mean realizable."""
    cfg = SOD
    announce("fp32_1d_vacuum")
    prob, (T, R) = oracle_for(cfg)
    u = inputs.fuzz_euler(1, R.M, prob.E, T.n, 6, vacuum_frac=0.15)
    u, fl = ost.limit(prob, T, R, u)
    assert fl.sum() > 0
    sol = solver_for(cfg, "fp32")
    ud = to_dev(u)
    ref = u.copy()
    for i in range(3):
        rec = []
        ref, _, rflags = ostep.step(prob, ref, 1e-5, (T, R), record=rec)
        _, flags = sol.step(ud, 1e-5)
        sol.sync()
        _flags_close(prob, T, R, to_np(flags).reshape(4, prob.E), rflags, rec)
        err = rel_l2(to_np(ud), ref)
        print("[fp32 1d] vacuum step %d rel L2 error %.3e" % (i, err), flush=True)
        assert err < FP32_STEP_TOL * (i + 1)
    rho = ost.element_mean(prob, T, to_np(ud))
    assert np.all(rho[0] > 0)


def test_fp32_1d_full_size_sod():
    """2048 elements, 11 modes, 24 nodes: ten FP32-mixed CFL steps against the oracle.
    The limiter acts at the Gibbs points of the projected interface and leaves nodal
    pressures at its floor of 1e-8, below the FP32 rounding of the energy; the FP32
    sound speed takes such a pressure as zero instead of returning NaN."""
    cfg = inputs.SOD
    announce("fp32_1d_full_size_sod")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, "fp32")
    ud = to_dev(u0)
    ref = u0.copy()
    limited = 0
    for i in range(10):
        rec = []
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= FP32_DT_TOL * rdt
        _flags_close(prob, T, R, to_np(flags).reshape(4, prob.E), rflags, rec)
        limited += int(rflags[0].sum())
        err = rel_l2(to_np(ud), ref)
        print("[fp32 1d] full-size Sod step %d rel L2 error %.3e" % (i, err), flush=True)
        assert err < FP32_STEP_TOL * (i + 1)
    assert limited > 0


@pytest.mark.parametrize("label,cfg,dt", [("burgers_ragged", BURGERS_RAGGED, 4e-4), ("advection", ADVECTION, 1e-3)])
def test_fp32_adjoint_step_against_oracle(label, cfg, dt):
    """One FP32-mixed adjoint step (the stage states recomputed by the FP32-mixed
    forward kernel) against the oracle's FP64 adjoint step."""
    import torch
    announce("fp32_adjoint_step", label)
    prob, (T, R) = oracle_for(cfg)
    u = _state(cfg, prob, T, R, 11)
    lam = np.random.default_rng(12).standard_normal(u.shape)
    _, _, rflags = ostep.step(prob, u, dt, (T, R))
    ref, rda = oadj.step_vjp(prob, T, R, u, dt, rflags, lam)
    sol = solver_for(cfg, "fp32")
    ud = to_dev(u)
    un = ud.clone()
    _, flags = sol.step(un, dt)
    sol.sync()
    assert np.array_equal(to_np(flags).reshape(4, prob.E), rflags)
    ld = to_dev(lam)
    dp = torch.zeros(2, dtype=torch.float64, device=ud.device)
    sol.adjoint_step(ud, flags, dt, ld, dp)
    sol.sync()
    err = rel_l2(to_np(ld), ref)
    print("[fp32 adjoint] %s rel L2 %.2e, d/da %r vs %r" % (label, err, float(to_np(dp)[0]), rda), flush=True)
    assert err < FP32_ADJ_TOL
    assert abs(float(to_np(dp)[0]) - rda) <= FP32_ADJ_TOL * max(1.0, abs(rda))


def test_fp32_adjoint_full_size_gradient():
    """4096 elements, 500 steps, checkpoints every 25: the FP32-mixed gradient of
    J = int E[u]^2 + Var[u] against the FP64 one (itself held to the oracle and to
    central differences).  Per step the FP32 rounding moves the adjoint by at most
    FP32_ADJ_TOL of its size; over 500 steps that bounds the gradient's relative
    error by 500 FP32_ADJ_TOL = 5e-3."""
    import torch
    from paper_2112_05946_amd.adjoint import AdjointSolve, mean_square
    cfg = inputs.BURGERS_ADJOINT
    announce("fp32_adjoint_full_size")
    grads = {}
    for prec in ("fp64", "fp32"):
        sol = solver_for(cfg, prec)
        u0 = sol.initial_state()
        dtd, _ = sol.step(u0.clone())
        dt = float(to_np(dtd)[0])
        params = torch.tensor([0.0, 1.4], dtype=torch.float64)
        x = u0.clone().requires_grad_(True)
        J = mean_square(AdjointSolve.apply(x, params, sol, cfg["n_steps"], dt, cfg["checkpoint_every"]), sol)
        J.backward()
        grads[prec] = to_np(x.grad)
    err = rel_l2(grads["fp32"], grads["fp64"])
    print("[fp32 adjoint] full size gradient rel L2 vs FP64 %.2e" % err, flush=True)
    assert err < cfg["n_steps"] * FP32_ADJ_TOL


def _mesh_totals(prob, T, u):
    """sum_e J_e sum_j w_j u_{e,j,0} per conserved variable, and the same of |u|."""
    if prob.dim == 1:
        w, J = np.asarray(T.w), prob.dx / 2.0
    else:
        w, J = np.outer(T.w, T.w).ravel(), prob.dx * prob.dy / 4.0
    return J * np.einsum("sej,j->s", u[:, 0], w), J * np.einsum("sej,j->s", np.abs(u[:, 0]), w)


CONSERVATION = [
    ("burgers_fp64", inputs.small(inputs.BURGERS, 64), "fp64"),
    ("burgers_fp32", inputs.small(inputs.BURGERS, 64), "fp32"),
    ("sv_fp64", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 8), gpc_order=3, nq1d=4, bc=["periodic"] * 4,
                     sensor="always", filter="l2", limiter=False), "fp64"),
    ("sv_fp32", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 8), gpc_order=3, nq1d=4, bc=["periodic"] * 4,
                     sensor="always", filter="l2", limiter=False), "fp32"),
    ("sv_bf16", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 8), gpc_order=3, nq1d=4, bc=["periodic"] * 4,
                     sensor="always", filter="l2", limiter=False), "bf16"),
]


@pytest.mark.parametrize("label,cfg,prec", CONSERVATION)
def test_mean_mode_conservation(label, cfg, prec):
    announce("conservation", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = _state(cfg, prob, T, R, 5)
    sol = solver_for(cfg, prec)
    ud = to_dev(u0)
    t0, mag = _mesh_totals(prob, T, u0)
    unit = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    n = prob.p + 1
    grow = 0.0
    worst = 0.0
    for i in range(6):
        u = to_np(ud)
        # a bound on the flux magnitudes of the state at the solution points and
        # nodes: u^2 (Burgers u^2 / 2), or |U|^2 / rho + |U| (Euler m^2 / rho + p)
        nodal = np.einsum("smej,mq->sqej", u, R.Phi)
        big = np.abs(nodal).max()
        F = big ** 2 if prob.S == 1 else big ** 2 / nodal[0].min() + big
        dtd, _ = sol.step(ud)
        sol.sync()
        dt = float(to_np(dtd)[0])
        t, _ = _mesh_totals(prob, T, to_np(ud))
        # faces per element times their length: 1 in 1D, dx + dy in 2D
        face = (prob.dx + prob.dy) if prob.dim == 2 else 1.0
        grow += 3 * prob.E * dt * 8 * (n + 2) * unit * F * face
        bound = grow
        drift = np.abs(t - t0)
        worst = max(worst, float((drift / np.maximum(mag, 1e-300)).max()))
        print("[conservation] %s step %d drift %s bound %.2e" % (label, i, drift, bound), flush=True)
        assert np.all(drift <= bound), (i, drift, bound)
    print("[conservation] %s worst drift / total magnitude %.2e" % (label, worst), flush=True)


def test_fp32_rejected_off_the_fused_paths():
    from paper_2112_05946_amd.binding import FrsgError
    for cfg in (dict(inputs.small(inputs.BURGERS, 9), gpc_order=4, nq1d=100),   # too many nodes for the fused kernel
                inputs.small(inputs.SHOCK_VORTEX, 6, 6)):                      # off the 4 x 2 tiles
        with pytest.raises(FrsgError) as ei:
            solver_for(cfg, "fp32")
        assert ei.value.status == -2

"""BF16-split precision on the 1D stage kernel (chaos expansion and projection on
the matrix cores), against the FP64 oracle.

The bars follow from the split as for the 2D kernel: each operand of the two
transforms is split into high and low bfloat16 parts with |x - hi - lo| <=
2^-16 |x|, and lo*lo (also <= 2^-16 of a product) is dropped, so a transform
has a relative error of order 2^-16 = 1.5e-5 of its largest terms; the
right-hand side keeps that order up to the cancellation of its flux terms (a
factor of a few), so its bar is BF16_RHS_TOL = 1e-4 relative L2; a step moves
the state by dt R with dt |R| / |u| <= 0.1, which gives BF16_STEP_TOL = 1e-5 per
step.  Switch decisions (FP64, on the BF16-perturbed state) may differ from the
oracle's only where the oracle's own margin is below BF16_TIE = 1e-3.
"""

import numpy as np
import pytest

from gpu_util import announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import fr as ofr
from oracle import stabilize as ost
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

BF16_RHS_TOL = 1e-4
BF16_STEP_TOL = 1e-5
BF16_DT_TOL = 1e-5
BF16_TIE = 1e-3

BURGERS = inputs.small(inputs.BURGERS, 64)
BURGERS_RAGGED = inputs.small(inputs.BURGERS, 37)
SOD = inputs.small(inputs.SOD, 96)            # 11 modes, 24 nodes: two blocks of 16 nodes
SOD_HLL = inputs.small(inputs.SOD_HLL, 50)
ADVECTION = inputs.small(inputs.ADVECTION, 20)  # p = 2, 5 modes, 8 nodes
BURGERS_LASSO = inputs.small(inputs.BURGERS_LASSO, 40)


def _state(cfg, prob, T, R, seed):
    u = project_initial(prob, cfg["ic"], (T, R))
    if prob.S == 1:
        u[:, :, ::3] += inputs.fuzz_scalar(R.M, prob.E, T.n, seed, scale=0.3)[:, :, ::3]
    return u


def _flags_close(prob, T, R, gflags, rflags, record):
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
        assert np.all(rel <= BF16_TIE), ("decision differs away from a tie", pas, bad[:5], rel[:5])


@pytest.mark.parametrize("label,cfg", [("burgers", BURGERS), ("burgers_ragged", BURGERS_RAGGED), ("sod", SOD),
                                       ("sod_hll", SOD_HLL), ("advection", ADVECTION)])
@pytest.mark.parametrize("seed", [0, 1])
def test_bf16_1d_rhs_error(label, cfg, seed):
    announce("bf16_1d_rhs", label, seed)
    prob, (T, R) = oracle_for(cfg)
    if prob.S == 1:
        u = inputs.fuzz_scalar(R.M, prob.E, T.n, seed, offset=1.0)
    else:
        u = inputs.fuzz_euler(1, R.M, prob.E, T.n, seed)
    ref = ofr.rhs(prob, T, R, u)
    sol = solver_for(cfg, "bf16")
    got = to_np(sol.rhs(to_dev(u)))
    sol.sync()
    err = rel_l2(got, ref)
    print("[bf16 1d] %s rhs rel L2 error %.3e" % (label, err), flush=True)
    assert err < BF16_RHS_TOL


@pytest.mark.parametrize("label,cfg", [("burgers", BURGERS), ("sod", SOD), ("sod_hll", SOD_HLL),
                                       ("burgers_lasso", BURGERS_LASSO)])
def test_bf16_1d_steps_error(label, cfg):
    """Four CFL steps against the oracle's FP64 steps, with the detector, the filter
    and (Sod) the limiter in the FP64 epilogue."""
    announce("bf16_1d_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = _state(cfg, prob, T, R, 3)
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    ref = u0.copy()
    fired = 0
    for i in range(4):
        rec = []
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= BF16_DT_TOL * rdt
        _flags_close(prob, T, R, to_np(flags).reshape(4, prob.E), rflags, rec)
        fired += int(rflags[2].sum())
        err = rel_l2(to_np(ud), ref)
        print("[bf16 1d] %s step %d rel L2 error %.3e" % (label, i, err), flush=True)
        assert err < BF16_STEP_TOL * (i + 1)
    assert fired > 0


def test_bf16_1d_full_size_burgers():
    """1024 elements, 9 modes, 16 nodes (the Burgers workload): ten BF16-split CFL
    steps against the oracle."""
    cfg = inputs.BURGERS
    announce("bf16_1d_full_size")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    ref = u0.copy()
    for i in range(10):
        rec = []
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= BF16_DT_TOL * rdt
        _flags_close(prob, T, R, to_np(flags).reshape(4, prob.E), rflags, rec)
        err = rel_l2(to_np(ud), ref)
        print("[bf16 1d] full-size Burgers step %d rel L2 error %.3e" % (i, err), flush=True)
        assert err < BF16_STEP_TOL * (i + 1)


def test_bf16_1d_conserves_the_mean():
    """Periodic Burgers: the mesh total of the mean mode moves by at most the rounding
    bound of the FP32 residual (the derivation in test_gpu_fp32_1d)."""
    cfg = BURGERS
    announce("bf16_1d_conservation")
    prob, (T, R) = oracle_for(cfg)
    u0 = _state(cfg, prob, T, R, 5)
    sol = solver_for(cfg, "bf16")
    ud = to_dev(u0)
    J = prob.dx / 2.0
    t0 = J * np.einsum("ej,j->", u0[0, 0], T.w)
    grow = 0.0
    for i in range(6):
        big = np.abs(np.einsum("smej,mq->sqej", to_np(ud), R.Phi)).max()
        dtd, _ = sol.step(ud)
        sol.sync()
        dt = float(to_np(dtd)[0])
        grow += 3 * prob.E * dt * 8 * (T.n + 2) * 2.0 ** -24 * big ** 2
        t = J * np.einsum("ej,j->", to_np(ud)[0, 0], T.w)
        print("[bf16 1d conservation] step %d drift %.3e bound %.3e" % (i, abs(t - t0), grow), flush=True)
        assert abs(t - t0) <= grow


def test_bf16_1d_scope():
    """More than 16 gPC modes: rejected (one block of modes); the adjoint: FP64 and
    FP32-mixed only."""
    import torch
    from paper_2112_05946_amd.binding import FrsgError
    with pytest.raises(FrsgError) as ei:
        solver_for(dict(BURGERS, gpc_order=16, nq1d=17), "bf16")
    assert ei.value.status == -2
    sol = solver_for(BURGERS, "bf16")
    u = sol.initial_state()
    un = u.clone()
    _, flags = sol.step(un, 1e-4)
    lam = torch.ones_like(u)
    with pytest.raises(FrsgError) as ei:
        sol.adjoint_step(u, flags, 1e-4, lam)
    assert ei.value.status == -2

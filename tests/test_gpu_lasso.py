"""Lasso filter (Sec. 4.1.3) on the GPU against the oracle.

Fused 1D stage kernel (end-of-step pass: thread per chaos mode) and the
multi-pass path (node counts the fused kernel does not hold), scalar and
Euler equations, every element filtered or detector-gated; states with every
modal coefficient active (seeded fuzz) so that both branches of the soft
threshold occur.
"""

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    ("burgers_fused", dict(inputs.small(inputs.BURGERS, 20), filter="lasso", sensor="always")),
    ("burgers_fused_detector", dict(inputs.small(inputs.BURGERS, 20), filter="lasso")),
    ("burgers_multipass", dict(inputs.small(inputs.BURGERS, 12), filter="lasso", sensor="always", nq1d=100)),
    ("sod_fused_limiter", dict(inputs.small(inputs.SOD, 24), filter="lasso", sensor="always")),
    ("advection_p2", dict(inputs.small(inputs.ADVECTION, 16), filter="lasso", sensor="always")),
]


def _fuzz(cfg, prob, R, T, seed):
    u = project_initial(prob, cfg["ic"], (T, R))
    if prob.S == 1:
        return u + 0.3 * inputs.fuzz_scalar(R.M, prob.E, T.n, seed)
    return u


@pytest.mark.parametrize("label,cfg", CASES)
def test_lasso_steps_match_oracle(label, cfg):
    announce("lasso_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = _fuzz(cfg, prob, R, T, 11)
    sol = solver_for(cfg)
    ud = to_dev(u0)
    ref = u0.copy()
    for i in range(3):
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R))
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= 1e-13 * rdt
        assert np.array_equal(to_np(flags).reshape(4, prob.E)[2], rflags[2])
        err = rel_l2(to_np(ud), ref)
        print("[lasso] %s step %d rel-L2 %.2e filtered %d/%d" % (label, i, err, rflags[2].sum(), prob.E), flush=True)
        assert err < RTOL_FP64


def test_lasso_chained_steps_match_oracle():
    """fr_sg_steps (CFL maximum passed between steps) with the Lasso filter."""
    import torch
    cfg = dict(inputs.small(inputs.BURGERS, 32), filter="lasso", sensor="always")
    announce("lasso_chained")
    prob, (T, R) = oracle_for(cfg)
    u0 = _fuzz(cfg, prob, R, T, 4)
    ref = u0.copy()
    rdts = []
    for _ in range(8):
        ref, rdt, _ = ostep.step(prob, ref, None, (T, R))
        rdts.append(rdt)
    sol = solver_for(cfg)
    ud = to_dev(u0)
    dts = torch.empty(8, dtype=torch.float64, device=ud.device)
    sol.steps(ud, 8, dts)
    sol.sync()
    assert np.allclose(to_np(dts), rdts, rtol=1e-13, atol=0)
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_lasso_has_no_adjoint():
    from paper_2112_05946_amd.binding import FrsgError
    cfg = dict(inputs.small(inputs.BURGERS, 8), filter="lasso", sensor="always")
    sol = solver_for(cfg)
    u = sol.initial_state()
    lam = u.clone()
    flags = sol.step(u.clone(), 1e-4)[1]
    with pytest.raises(FrsgError) as ei:
        sol.adjoint_step(u, flags, 1e-4, lam)
    assert ei.value.status == -2

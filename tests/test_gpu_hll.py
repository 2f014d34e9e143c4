"""HLL interactive flux on the GPU against the oracle: the fused 1D and 2D stage
kernels, the multi-pass paths, FP32-mixed, and the face-trace hand-over of
fr_sg_steps."""

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import fr as ofr
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

RHS = [
    ("sod_fused", dict(inputs.small(inputs.SOD, 37), flux="hll")),
    ("sod_multipass", dict(inputs.small(inputs.SOD, 9), flux="hll", nq1d=100, gpc_order=6)),
    ("sv_fused", dict(inputs.small(inputs.SHOCK_VORTEX, 12, 8), flux="hll")),
    ("sv_generic", dict(inputs.small(inputs.SHOCK_VORTEX, 7, 5), flux="hll")),      # mesh not in tiles
    ("sv_generic_p2", dict(inputs.small(inputs.SHOCK_VORTEX, 4, 4), flux="hll", p=2)),
]


@pytest.mark.parametrize("label,cfg", RHS)
@pytest.mark.parametrize("seed", [0, 1])
def test_hll_rhs_fuzz(label, cfg, seed):
    announce("hll_rhs", label, seed)
    prob, (T, R) = oracle_for(cfg)
    u = inputs.fuzz_euler(prob.dim, R.M, prob.E, prob.nsp, seed)
    ref = ofr.rhs(prob, T, R, u)
    sol = solver_for(cfg)
    got = to_np(sol.rhs(to_dev(u)))
    sol.sync()
    assert rel_l2(got, ref) < RTOL_FP64


@pytest.mark.parametrize("label,cfg", [RHS[0], RHS[2], RHS[3]])
def test_hll_steps_match_oracle(label, cfg):
    announce("hll_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u0)
    ref = u0.copy()
    for i in range(4):
        ref, rdt, rflags = ostep.step(prob, ref, None, (T, R))
        dtd, flags = sol.step(ud)
        sol.sync()
        assert abs(to_np(dtd)[0] - rdt) <= 1e-13 * rdt
        err = rel_l2(to_np(ud), ref)
        print("[hll] %s step %d rel-L2 %.2e" % (label, i, err), flush=True)
        assert err < RTOL_FP64


def test_hll_fp32_mixed_step():
    cfg = RHS[2][1]
    announce("hll_fp32")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref, rdt, _ = ostep.step(prob, u0, None, (T, R))
    sol = solver_for(cfg, "fp32")
    ud = to_dev(u0)
    dtd, _ = sol.step(ud)
    sol.sync()
    assert abs(to_np(dtd)[0] - rdt) <= 1e-6 * rdt
    assert rel_l2(to_np(ud), ref) < 1e-6


def test_hll_steps_match_single_steps_bitwise():
    import torch
    cfg = RHS[2][1]
    announce("hll_steps_vs_step")
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    ua = to_dev(u0)
    dts = torch.empty(3, dtype=torch.float64, device=ua.device)
    sol.steps(ua, 3, dts)
    sol.sync()
    ub = to_dev(u0)
    for dt in to_np(dts):
        sol.step(ub, float(dt))
    sol.sync()
    assert np.array_equal(to_np(ua), to_np(ub))


@pytest.mark.parametrize("label,cfg", [("sod", dict(inputs.SOD, flux="hll")),
                                       ("shock_vortex", dict(inputs.SHOCK_VORTEX, flux="hll"))])
def test_hll_full_size_step(label, cfg):
    announce("hll_full_size", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref, rdt, _ = ostep.step(prob, u0, None, (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u0)
    dtd, _ = sol.step(ud)
    sol.sync()
    assert abs(to_np(dtd)[0] - rdt) <= 1e-13 * rdt
    assert rel_l2(to_np(ud), ref) < RTOL_FP64

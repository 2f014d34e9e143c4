"""The caller-owned workspace and the exponential filter cutoff on the GPU.

* fr_sg_init, fr_sg_step and fr_sg_destroy allocate no device memory: the free
  device memory is the same before and after each once the caller has
  allocated the state, flags and the workspace fr_sg_workspace_size asked for.
* two contexts on separate workspaces coexist and give the results each gives
  alone.
* the cutoff N* of the exponential filter (Sec. 4.1.1) is honoured on the fused
  1D, generic 1D, fused 2D and fused triangle paths and by the adjoint: steps
  match the oracle to 1e-12 with identical filter decisions.
"""

import ctypes

import numpy as np
import pytest

from gpu_util import ELEM_RTOL, RTOL_FP64, announce, check_flags, elem_max_rel, oracle_for, rel_l2, solver_for, \
    to_dev, to_np
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("label,cfg", [("burgers", inputs.small(inputs.BURGERS, 40)),
                                       ("shock_vortex", inputs.small(inputs.SHOCK_VORTEX, 16, 8))])
def test_init_step_destroy_allocate_no_device_memory(label, cfg):
    import torch
    announce("no_device_allocation", label)
    lib = binding.load_library()
    # warm-up: the same problem once through the binding, so every kernel's code is loaded
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    warm = solver_for(cfg)
    uw = to_dev(u0)
    warm.step(uw)
    warm.sync()
    warm.close()
    P = binding.problem_from_config(cfg)
    n = ctypes.c_int64()
    assert lib.fr_sg_workspace_size(ctypes.byref(P), ctypes.byref(n)) == 0
    stream = torch.cuda.current_stream()
    ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
    u = to_dev(u0)
    dt_used = torch.empty(1, dtype=torch.float64, device="cuda")
    flags = torch.empty(4 * prob.E, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = ctypes.c_void_p()
    assert lib.fr_sg_init(ctypes.byref(P), ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(ws.data_ptr()),
                          n.value, ctypes.byref(ctx)) == 0
    free1 = torch.cuda.mem_get_info()[0]
    assert lib.fr_sg_step(ctx, ctypes.c_void_p(u.data_ptr()), 0.0, ctypes.c_void_p(dt_used.data_ptr()),
                          ctypes.c_void_p(flags.data_ptr())) == 0
    assert lib.fr_sg_sync(ctx) == 0
    free2 = torch.cuda.mem_get_info()[0]
    assert lib.fr_sg_destroy(ctx) == 0
    torch.cuda.synchronize()
    free3 = torch.cuda.mem_get_info()[0]
    print("[free device memory]", free0, free1, free2, free3, flush=True)
    assert free0 == free1 == free2 == free3
    # and the step is the one the binding's solver takes
    assert torch.equal(u, uw)


def test_two_contexts_side_by_side():
    import torch
    announce("two_contexts")
    c1 = inputs.small(inputs.SOD, 33)
    c2 = inputs.small(inputs.SHOCK_VORTEX, 8, 6)
    out = {}
    for cfg in (c1, c2):
        prob, (T, R) = oracle_for(cfg)
        out[cfg["name"]] = project_initial(prob, cfg["ic"], (T, R))
    alone = {}
    for cfg in (c1, c2):
        s = solver_for(cfg)
        u = to_dev(out[cfg["name"]])
        for _ in range(3):
            s.step(u)
        s.sync()
        alone[cfg["name"]] = u
        s.close()
    s1, s2 = solver_for(c1), solver_for(c2)
    a, b = to_dev(out[c1["name"]]), to_dev(out[c2["name"]])
    for _ in range(3):
        s1.step(a)
        s2.step(b)
    s1.sync()
    s2.sync()
    assert torch.equal(a, alone[c1["name"]]) and torch.equal(b, alone[c2["name"]])


NSTAR = [
    ("fused_1d_burgers", dict(inputs.small(inputs.BURGERS, 29), sensor="always", nstar=1.5)),
    ("generic_1d_burgers_100_nodes", dict(inputs.small(inputs.BURGERS, 12), gpc_order=8, nq1d=100,
                                          sensor="always", nstar=2.0)),
    ("fused_2d", dict(inputs.small(inputs.SHOCK_VORTEX, 8, 4), gpc_order=2, nq1d=3, filter="exp", sensor="always",
                      alpha=36.0, s=2.0, nstar=1.0)),
    ("fused_tri", dict(inputs.tri_shock_vortex(4), gpc_order=2, nq1d=3, filter="exp", sensor="always",
                       alpha=36.0, s=2.0, nstar=1.0)),
]


@pytest.mark.parametrize("label,cfg", NSTAR)
def test_exponential_filter_cutoff_steps(label, cfg):
    announce("nstar_steps", label)
    prob, (T, R) = oracle_for(cfg)
    u = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    ud = to_dev(u)
    for i in range(3):
        rec = []
        u, rdt, rfl = ostep.step(prob, u, None, (T, R), record=rec)
        dtd, flags = sol.step(ud)
        sol.sync()
        g = to_np(flags).reshape(4, prob.E)
        assert abs(to_np(dtd)[0] / rdt - 1.0) < 1e-13
        assert rfl[2].all()
        check_flags(prob, T, R, g, rfl, rec)
        got = to_np(ud)
        assert rel_l2(got, u) < RTOL_FP64, (i, rel_l2(got, u))
        assert elem_max_rel(got, u) < ELEM_RTOL


def test_exponential_filter_cutoff_adjoint():
    """The adjoint step with the cutoff filter against the oracle's adjoint."""
    from oracle import adjoint as oadj
    cfg = dict(inputs.small(inputs.BURGERS, 21), sensor="always", nstar=2.0)
    announce("nstar_adjoint")
    prob, (T, R) = oracle_for(cfg)
    u = project_initial(prob, cfg["ic"], (T, R))
    dt = 0.5 * ostep.cfl_dt(prob, T, R, u)
    _, _, rflags = ostep.step(prob, u, dt, (T, R))
    assert rflags[2].all()
    lam = np.random.default_rng(2).standard_normal(u.shape)
    ref, _ = oadj.step_vjp(prob, T, R, u, dt, rflags, lam)
    sol = solver_for(cfg)
    ud = to_dev(u)
    un = ud.clone()
    _, flags = sol.step(un, dt)
    ld = to_dev(lam)
    sol.adjoint_step(ud, flags, dt, ld)
    sol.sync()
    assert np.array_equal(to_np(flags).reshape(4, prob.E), rflags)
    assert rel_l2(to_np(ld), ref) < RTOL_FP64

"""fr_sg_init_static, the entry point for callers that cannot allocate device
memory, against fr_sg_init with a caller-allocated workspace: two problems in a
row on the library's static per-GPU array (the second smaller, so it runs on
what the first left behind), each stepped through the C ABI and compared with
the same steps on a torch-allocated workspace (bit for bit, which is within the
1e-12 parity bar); the calls allocate no device memory; a problem larger than
the array is rejected with a message naming both sizes."""

import ctypes

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, to_dev, to_np
from oracle.initial import project_initial
from paper_2112_05946_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _steps_static(lib, cfg, u0, nsteps):
    import torch
    P = binding.problem_from_config(cfg)
    stream = torch.cuda.current_stream()
    u = to_dev(u0)
    dts = torch.empty(nsteps, dtype=torch.float64, device="cuda")
    E = u.shape[2]
    flags = torch.empty(4 * E * nsteps, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = ctypes.c_void_p()
    st = lib.fr_sg_init_static(ctypes.byref(P), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx))
    assert st == 0, lib.fr_sg_last_error(None).decode()
    assert lib.fr_sg_steps(ctx, ctypes.c_void_p(u.data_ptr()), nsteps, ctypes.c_void_p(dts.data_ptr()),
                           ctypes.c_void_p(flags.data_ptr())) == 0
    assert lib.fr_sg_sync(ctx) == 0
    assert lib.fr_sg_destroy(ctx) == 0
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return u, dts, flags, free0, free1


def _steps_caller_workspace(cfg, u0, nsteps):
    import torch
    from paper_2112_05946_amd.binding import Solver
    sol = Solver(cfg)
    u = to_dev(u0)
    dts = torch.empty(nsteps, dtype=torch.float64, device="cuda")
    flags = torch.empty(4 * sol.E * nsteps, dtype=torch.uint8, device="cuda")
    sol.steps(u, nsteps, dt_used=dts, flags=flags)
    sol.sync()
    sol.close()
    return u, dts, flags


def test_static_workspace_matches_caller_workspace():
    import torch
    lib = binding.load_library()
    big = inputs.small(inputs.SHOCK_VORTEX, 32, 16)
    small = inputs.small(inputs.SHOCK_VORTEX, 12, 8)
    burgers = inputs.small(inputs.BURGERS, 100)
    frees = []
    for label, cfg in (("shock_vortex_32x16", big), ("shock_vortex_12x8", small), ("burgers_100", burgers)):
        announce("static_workspace", label)
        prob, (T, R) = oracle_for(cfg)
        u0 = project_initial(prob, cfg["ic"], (T, R))
        ref_u, ref_dt, ref_fl = _steps_caller_workspace(cfg, u0, 4)
        u, dts, fl, free0, free1 = _steps_static(lib, cfg, u0, 4)
        assert rel_l2(to_np(u), to_np(ref_u)) < RTOL_FP64
        assert torch.equal(u, ref_u) and torch.equal(dts, ref_dt) and torch.equal(fl, ref_fl), label
        frees.append((free0, free1))
    # after the first bind the array is resident: later binds, steps and destroys allocate nothing
    for free0, free1 in frees[1:]:
        assert free0 == free1, frees


def test_static_workspace_rejects_large_problems():
    lib = binding.load_library()
    announce("static_workspace_too_large")
    P = binding.problem_from_config(inputs.SHOCK_VORTEX)
    ctx = ctypes.c_void_p()
    st = lib.fr_sg_init_static(ctypes.byref(P), None, ctypes.byref(ctx))
    msg = lib.fr_sg_last_error(None).decode()
    assert st == -2 and not ctx.value
    assert "static workspace holds 67108864" in msg, msg

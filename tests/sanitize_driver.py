"""Host-side checks run inside a process that preloads the AddressSanitizer
runtime, against the library whose host sources were built with AddressSanitizer
and UndefinedBehaviorSanitizer (paper_2112_05946_amd/build.py, build_sanitized).

Everything here stays on the host: the workspace-size query runs the whole
problem validation, the operator tables (1D, quadrilateral, triangle, every
compiled degree and chaos order), the triangle mesh checks and the workspace
layout; the invalid problems and arguments take the error paths.  No call
reaches the HIP runtime.  A sanitizer finding aborts the process with a report
on stderr; a clean run prints one summary line and exits 0.

usage: python sanitize_driver.py <libfrsg_san.so>
"""

import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2112_05946_amd import binding, inputs  # noqa: E402


def main(path):
    lib = binding.load_library(path)
    n_ok = 0

    def size(cfg, precision="fp64"):
        P = binding.problem_from_config(cfg, precision)
        n = ctypes.c_int64(-1)
        st = lib.fr_sg_workspace_size(ctypes.byref(P), ctypes.byref(n))
        return st, n.value, lib.fr_sg_last_error(None).decode()

    def init_host(cfg, ws, nbytes):
        P = binding.problem_from_config(cfg)
        ctx = ctypes.c_void_p()
        st = lib.fr_sg_init(ctypes.byref(P), None, ws, nbytes, ctypes.byref(ctx))
        return st, ctx.value, lib.fr_sg_last_error(None).decode()

    def expect_ok(cfg, precision="fp64"):
        nonlocal n_ok
        st, n, msg = size(cfg, precision)
        if st != 0 or n <= 0 or n % 256:
            raise SystemExit("size query failed for %s %s: %d %s" % (cfg.get("name"), precision, st, msg))
        n_ok += 1
        return n

    def expect_err(cfg, status, precision="fp64"):
        nonlocal n_ok
        st, n, msg = size(cfg, precision)
        if st != status or n != 0 or not msg:
            raise SystemExit("expected %d for %s, got %d (%s)" % (status, cfg.get("name"), st, msg))
        n_ok += 1

    # every named workload, at its full size where that is a host-only matter
    for cfg in inputs.CONFIGS.values():
        expect_ok(cfg)
    for cfg, precs in ((inputs.BURGERS, ("fp32", "bf16")), (inputs.SOD, ("fp32", "bf16")),
                       (inputs.SHOCK_VORTEX, ("fp32", "bf16")), (inputs.BURGERS_ADJOINT, ("fp32",))):
        for prec in precs:
            expect_ok(cfg, prec)
    # every FR degree and a range of chaos orders in one and two random dimensions
    for p in range(1, 8):
        for order in (0, 1, 4, 8):
            expect_ok(dict(inputs.small(inputs.BURGERS, 12), p=p, gpc_order=order, nq1d=order + 2))
        expect_ok(dict(inputs.small(inputs.SOD, 10), p=p, gpc_order=3, rdim=2, nq1d=4))
    for p in (1, 2, 3):
        expect_ok(dict(inputs.small(inputs.SHOCK_VORTEX, 8, 4), p=p))
    expect_ok(inputs.vortex_convection(8, 2))
    # triangles: every compiled degree, periodic and bounded meshes
    for p in (1, 2, 3, 4):
        expect_ok(inputs.tri_density_wave(3, p=p))
    expect_ok(inputs.tri_vortex(4))
    expect_ok(inputs.tri_shock_vortex(4))

    # invalid problems: the documented status, no size, a message
    base = inputs.BURGERS
    expect_err(dict(base, p=0), -1)
    expect_err(dict(base, p=8), -2)
    expect_err(dict(base, nx=0), -1)
    expect_err(dict(base, nq1d=3), -1)
    expect_err(dict(base, cfl=0.0), -1)
    expect_err(dict(base, limiter=True), -2)
    expect_err(dict(base, filter="exp", nstar=3.0), -1)
    expect_err(dict(base, gpc_order=20, nq1d=21), -2, "bf16")
    expect_err(dict(base, flux="hll"), -2)
    expect_err(dict(inputs.small(inputs.SHOCK_VORTEX, 4, 2), filter="lasso"), -2)
    expect_err(dict(inputs.tri_density_wave(3), p=5), -2)
    bad = {k: v.copy() for k, v in inputs.tri_density_wave(3)["mesh"].items()}
    bad["xy"][4] = bad["xy"][4][::-1]
    expect_err(dict(inputs.tri_density_wave(3), mesh=bad), -1)
    bad = {k: v.copy() for k, v in inputs.tri_density_wave(3)["mesh"].items()}
    bad["nbr_face"][0, 1] = 2
    expect_err(dict(inputs.tri_density_wave(3), mesh=bad), -1)

    # argument checks that end before any device call
    n = expect_ok(base)
    for ws, nbytes, word in ((None, n, "workspace"), (ctypes.c_void_p(1 << 20), n - 256, "workspace"),
                             (ctypes.c_void_p((1 << 20) + 8), n, "aligned")):
        st, ctx, msg = init_host(base, ws, nbytes)
        if st != -1 or ctx or word not in msg:
            raise SystemExit("workspace check: %d %s" % (st, msg))
        n_ok += 1
    checks = [
        lib.fr_sg_init(None, None, None, 0, None) == -1,
        lib.fr_sg_workspace_size(None, None) == -1,
        lib.fr_sg_query(None, None) == -1,
        lib.fr_sg_rhs(None, None, None) == -1,
        lib.fr_sg_step(None, None, 0.0, None, None) == -1,
        lib.fr_sg_steps(None, None, 1, None, None) == -1,
        lib.fr_sg_adjoint_step(None, None, None, 1e-3, None, None) == -1,
        lib.fr_sg_step_stages(None, None, 0.0, None, None, None, None) == -1,
        lib.fr_sg_adjoint_step_stages(None, None, None, None, None, 1e-3, None, None) == -1,
        lib.fr_sg_destroy(None) == 0,
        lib.fr_sg_copy(None, None, 0, None) == 0,
        lib.fr_sg_copy(None, None, -1, None) == -1,
        lib.fr_sg_copy(ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 8), 4, None) == -1,   # misaligned
        lib.fr_sg_copy(ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 16), 4, None) == -1,  # overlap
    ]
    if not all(checks):
        raise SystemExit("argument checks: %s" % checks)
    n_ok += len(checks)
    print("sanitized host checks passed: %d cases" % n_ok, flush=True)


if __name__ == "__main__":
    main(sys.argv[1])

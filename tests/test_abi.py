"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid problems with the documented status before any
device call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr_sg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2112_05946_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2112_05946_amd import build
        build.build()
    return binding.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fr_sg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for need in ("fr_sg_init", "fr_sg_rhs", "fr_sg_step", "fr_sg_destroy", "fr_sg_last_error"):
        assert need in syms


def test_every_declared_symbol_is_exported(lib):
    from paper_2112_05946_amd import binding
    bound = {name for name, _, _ in binding.SYMBOLS}
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert name in bound, "binding lacks " + name


def _init(lib, P, ws=None, nbytes=0):
    ctx = ctypes.c_void_p()
    st = lib.fr_sg_init(ctypes.byref(P), None, ws, nbytes, ctypes.byref(ctx))
    return st, ctx, lib.fr_sg_last_error(None).decode()


def _size(lib, P):
    n = ctypes.c_int64(-1)
    st = lib.fr_sg_workspace_size(ctypes.byref(P), ctypes.byref(n))
    return st, n.value, lib.fr_sg_last_error(None).decode()


@pytest.mark.parametrize("mutate,status", [
    (lambda P: setattr(P, "abi_version", 99), -6),
    (lambda P: setattr(P, "equation", 7), -1),
    (lambda P: setattr(P, "fr_degree", 0), -1),
    (lambda P: setattr(P, "fr_degree", 8), -2),
    (lambda P: setattr(P, "nx", 0), -1),
    (lambda P: setattr(P, "nq1d", 3), -1),
    (lambda P: setattr(P, "rdim", 3), -1),
    (lambda P: setattr(P, "cfl", 0.0), -1),
    (lambda P: setattr(P, "limiter", 1), -2),          # scalar equation
    (lambda P: P.bc.__setitem__(0, 1), -1),            # unpaired periodic side
    (lambda P: P.bc.__setitem__(0, 9), -1),
    (lambda P: setattr(P, "filter", 5), -1),
    (lambda P: setattr(P, "precision", 7), -1),
    (lambda P: (setattr(P, "precision", 2), setattr(P, "gpc_order", 20), setattr(P, "nq1d", 21)), -2),  # 21 modes
    (lambda P: (setattr(P, "filter", 1), setattr(P, "nstar", 3.0)), -1),    # cutoff >= p
    (lambda P: (setattr(P, "filter", 1), setattr(P, "nstar", -0.5)), -1),
    (lambda P: (setattr(P, "filter", 1), setattr(P, "nstar", 2.5), setattr(P, "gpc_order", 2),
                setattr(P, "nq1d", 3)), -1),                                # cutoff >= N_c
])
def test_invalid_problems_rejected_before_launch(lib, mutate, status):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(inputs.BURGERS)
    mutate(P)
    st, ctx, msg = _init(lib, P)
    assert st == status, msg
    assert not ctx.value and msg
    st2, n, msg2 = _size(lib, P)
    assert st2 == status and n == 0 and msg2 == msg


@pytest.mark.parametrize("name,S,nsp", [("BURGERS", 1, 4), ("SOD", 3, 4), ("SHOCK_VORTEX", 4, 16)])
def test_workspace_size_is_a_host_query(lib, name, S, nsp):
    """The size query needs no device; it covers at least the two stage states."""
    from paper_2112_05946_amd import binding, inputs
    cfg = getattr(inputs, name)
    st, n, msg = _size(lib, binding.problem_from_config(cfg))
    assert st == 0, msg
    M = (cfg["gpc_order"] + 1) * (cfg["gpc_order"] + 2) // 2 if cfg.get("rdim", 1) == 2 else cfg["gpc_order"] + 1
    state = 8 * S * M * cfg["nx"] * cfg.get("ny", 1) * nsp
    assert 2 * state < n < 8 * state + (1 << 20)
    assert n % 256 == 0


def test_workspace_argument_checked_before_any_device_call(lib):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(inputs.BURGERS)
    _, n, _ = _size(lib, P)
    st, ctx, msg = _init(lib, P, None, n)
    assert st == -1 and "workspace" in msg and not ctx.value
    st, ctx, msg = _init(lib, P, ctypes.c_void_p(1 << 20), n - 256)       # too short
    assert st == -1 and "workspace" in msg and not ctx.value
    st, ctx, msg = _init(lib, P, ctypes.c_void_p((1 << 20) + 8), n)       # misaligned
    assert st == -1 and "aligned" in msg and not ctx.value


def test_null_arguments(lib):
    assert lib.fr_sg_init(None, None, None, 0, None) == -1
    assert lib.fr_sg_workspace_size(None, None) == -1
    assert lib.fr_sg_query(None, None) == -1
    assert lib.fr_sg_rhs(None, None, None) == -1
    assert lib.fr_sg_step(None, None, 0.0, None, None) == -1
    assert lib.fr_sg_adjoint_step(None, None, None, 1e-3, None, None) == -1
    assert lib.fr_sg_step_stages(None, None, 0.0, None, None, None, None) == -1
    assert lib.fr_sg_adjoint_step_stages(None, None, None, None, None, 1e-3, None, None) == -1
    assert lib.fr_sg_destroy(None) == 0


@pytest.mark.parametrize("base,over", [
    ("SHOCK_VORTEX", dict(filter="lasso", nx=4, ny=2)),     # two physical dimensions
    ("BURGERS", dict(filter="lasso", rdim=2, nq1d=10)),     # two random dimensions
])
def test_lasso_scope_rejected_before_launch(lib, base, over):
    """The Lasso filter is provided for one physical and one random dimension."""
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(dict(getattr(inputs, base), **over))
    st, ctx, msg = _init(lib, P)
    assert st == -2, msg
    assert not ctx.value and "Lasso" in msg


def test_hll_needs_the_euler_equations(lib):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(dict(inputs.BURGERS, flux="hll"))
    st, ctx, msg = _init(lib, P)
    assert st == -2 and "HLL" in msg
    P = binding.problem_from_config(inputs.BURGERS)
    P.flux = 7
    st, ctx, msg = _init(lib, P)
    assert st == -1 and not ctx.value


def test_unknown_integrator_rejected(lib):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(inputs.BURGERS)
    P.integrator = 9
    st, ctx, msg = _init(lib, P)
    assert st == -1 and "integrator" in msg


def _tri_problem(**over):
    from paper_2112_05946_amd import binding, inputs
    cfg = dict(inputs.tri_density_wave(3), **over)
    return binding.problem_from_config(cfg), cfg


@pytest.mark.parametrize("over,status", [
    (dict(equation="burgers"), -2),
    (dict(filter="lasso"), -2),
    (dict(p=5), -2),
])
def test_tri_unsupported_combinations(lib, over, status):
    from paper_2112_05946_amd import binding
    P, _ = _tri_problem(**over)
    assert P.precision == binding.PRECISION["fp64"]
    st, ctx, msg = _init(lib, P)
    assert st == status, msg
    assert not ctx.value and msg


def test_tri_invalid_meshes_rejected_before_launch(lib):
    from paper_2112_05946_amd import binding, inputs
    base = inputs.tri_density_wave(3)

    def try_mesh(mesh, bc=None):
        cfg = dict(base, mesh=mesh)
        if bc:
            cfg["bc"] = bc
        P = binding.problem_from_config(cfg)
        return _init(lib, P)

    m = {k: v.copy() for k, v in base["mesh"].items()}
    m["xy"][4] = m["xy"][4][::-1]                       # clockwise
    st, ctx, msg = try_mesh(m)
    assert st == -1 and "clockwise" in msg and not ctx.value
    m = {k: v.copy() for k, v in base["mesh"].items()}
    m["nbr_face"][0, 1] = 2                              # link not mutual
    st, ctx, msg = try_mesh(m)
    assert st == -1 and "mutual" in msg
    m = inputs.tri_mesh_rectangle(3, 3, periodic=(False, True))
    st, ctx, msg = try_mesh(m, bc=["periodic"] * 4)      # boundary faces on periodic sides
    assert st == -1 and "periodic" in msg
    P, _ = _tri_problem()
    P.n_tri = 0
    st, ctx, msg = _init(lib, P)
    assert st == -1


def test_tri_fp32_mixed_unsupported(lib):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(inputs.tri_density_wave(3), precision="fp32")
    st, ctx, msg = _init(lib, P)
    assert st == -2 and "FP32" in msg


@pytest.mark.parametrize("over,status", [
    (dict(gpc_order=128, nq1d=129), -2),          # 129 modes
    (dict(rdim=2, gpc_order=10, nq1d=17), -2),    # 289 nodes
])
def test_chaos_limits(lib, over, status):
    from paper_2112_05946_amd import binding, inputs
    P = binding.problem_from_config(dict(inputs.BURGERS, **over))
    st, ctx, msg = _init(lib, P)
    assert st == status and "too many" in msg


def test_copy_arguments_checked_before_any_device_call(lib):
    vp = ctypes.c_void_p
    assert lib.fr_sg_copy(None, None, 0, None) == 0                              # nothing to copy
    assert lib.fr_sg_copy(None, None, -1, None) == -1
    assert lib.fr_sg_copy(None, vp(1 << 24), 5, None) == -1
    assert lib.fr_sg_copy(vp((1 << 20) + 8), vp(1 << 24), 4, None) == -1         # misaligned
    assert "aligned" in lib.fr_sg_last_error(None).decode()
    assert lib.fr_sg_copy(vp(1 << 20), vp((1 << 20) + 16), 4, None) == -1        # overlapping
    assert "overlap" in lib.fr_sg_last_error(None).decode()

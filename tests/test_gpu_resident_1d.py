"""Steps of small 1D problems in one one-workgroup launch (fr_sg_steps).

Where every element of a scalar FP64 problem of FR degree <= 3 fits one
workgroup ((E + 2) x N_q <= 1024 threads), fr_sg_steps runs all its steps in one
launch: the three stages of each step are the stage kernel's code separated by
workgroup barriers, and the CFL maximum of each step's output sets the next dt
without leaving the workgroup.  The per-element arithmetic is that of the three
launches per step, so the states, time steps and switch flags must equal those of
fr_sg_step called once per step (whose CFL pass takes the maximum in the same
order) bit for bit; the oracle bounds both at the FP64 parity bar.
"""

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu

ADV = inputs.ADVECTION                                              # 64 elements, p = 2, 8 nodes
ADV_P1 = dict(inputs.small(ADV, 40), p=1, gpc_order=2, nq1d=4)
ADV_OUTFLOW = dict(inputs.small(ADV, 30), bc=["dirichlet", "outflow", "periodic", "periodic"],
                   bc_state=[[0.0] * 4] * 4)
BURG = inputs.small(inputs.BURGERS, 12)                             # detector + exponential filter
BURG_L2 = dict(inputs.small(inputs.BURGERS, 20), filter="l2", sensor="always")
BURG_LASSO = inputs.small(inputs.BURGERS_LASSO, 16)
BURG_ONE = inputs.small(inputs.BURGERS, 1)                          # one element, its own neighbour
# the limits: (E + 2) x N_q threads <= 1024, and 8 bytes x (LDS words of the stage
# over E elements + 2 M N_q for the chaos tables + 16 for the CFL reduction + 256
# for the time steps) <= 64 KB
ADV_MAX = inputs.small(ADV, 126)                                    # (126 + 2) x 8 = 1024 threads
ADV_OVER = inputs.small(ADV, 127)                                   # 1032 threads: launched stages
BURG_MAX = inputs.small(inputs.BURGERS, 56)                         # 64,704 bytes of LDS
BURG_OVER = inputs.small(inputs.BURGERS, 57)                        # 65,760 bytes: launched stages

CASES = [("advection_c1", ADV), ("advection_p1", ADV_P1), ("advection_dirichlet_outflow", ADV_OUTFLOW),
         ("burgers_detector_exp", BURG), ("burgers_l2_always", BURG_L2), ("burgers_lasso", BURG_LASSO),
         ("advection_max_threads", ADV_MAX), ("burgers_max_lds", BURG_MAX), ("burgers_one_element", BURG_ONE)]


def _passes(sol):
    return set(sol.timing_read())


def _resident(passes):
    """'lds' (the states kept in LDS), 'global' (stage states in global memory) or None."""
    if "steps_resident_lds" in passes:
        return "lds"
    return "global" if "steps_resident" in passes else None


# where the three states fit the 64 KB with the stage's LDS they stay there
VARIANT = {"advection_max_threads": "global", "burgers_max_lds": "global"}


def _run_both(cfg, nsteps):
    import torch
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    a = solver_for(cfg)
    a.timing(True)
    ua = to_dev(u0)
    dts = torch.empty(nsteps, dtype=torch.float64, device=ua.device)
    flags = torch.empty(4 * prob.E * nsteps, dtype=torch.uint8, device=ua.device)
    a.steps(ua, nsteps, dts, flags)
    a.sync()
    passes = _passes(a)
    b = solver_for(cfg)
    ub = to_dev(u0)
    dtb, flb = [], []
    for _ in range(nsteps):
        d, f = b.step(ub)
        dtb.append(to_np(d)[0])
        flb.append(to_np(f).copy())
    b.sync()
    return prob, (T, R), u0, (to_np(ua), to_np(dts), to_np(flags)), (to_np(ub), np.array(dtb), np.concatenate(flb)), \
        passes


@pytest.mark.parametrize("label,cfg", CASES)
def test_resident_steps_equal_launched_steps(label, cfg):
    announce("resident_1d", label)
    n = 12
    prob, (T, R), u0, (ua, da, fa), (ub, db, fb), passes = _run_both(cfg, n)
    assert _resident(passes) == VARIANT.get(label, "lds"), passes
    assert np.array_equal(da, db), (da, db)
    assert np.array_equal(fa, fb)
    assert np.array_equal(ua, ub), np.abs(ua - ub).max()
    # the oracle, step by step at the device's time steps
    ref = u0.copy()
    for i in range(n):
        ref, rdt, _ = ostep.step(prob, ref, None, (T, R))
        assert abs(da[i] - rdt) <= 1e-13 * rdt, (i, da[i], rdt)
    assert rel_l2(ua, ref) < RTOL_FP64


def test_filter_fires_in_resident_steps():
    """The detector-switched exponential filter acts in the Burgers run (the oracle's
    detector first fires at step 113 on this mesh, t = 0.42)."""
    announce("resident_1d", "filter_fires")
    cfg = inputs.small(inputs.BURGERS, 24)
    n = 200
    _, _, _, (ua, da, fa), (ub, db, fb), passes = _run_both(cfg, n)
    assert _resident(passes) == "lds"
    fired = fa.reshape(n, 4, -1)[:, 2].sum()
    assert fired > 0
    assert np.array_equal(fa, fb) and np.array_equal(ua, ub) and np.array_equal(da, db)


def test_resident_calls_chain():
    """Two calls of 7 and 5 steps equal one call of 12: the CFL maximum of the
    first call's result is where the second call finds it."""
    import torch
    announce("resident_1d", "chained_calls")
    cfg = BURG
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    s1 = solver_for(cfg)
    u1 = to_dev(u0)
    d1 = torch.empty(12, dtype=torch.float64, device=u1.device)
    s1.steps(u1, 12, d1)
    s2 = solver_for(cfg)
    u2 = to_dev(u0)
    d2 = torch.empty(12, dtype=torch.float64, device=u2.device)
    s2.steps(u2, 7, d2[:7])
    s2.steps(u2, 5, d2[7:])
    s1.sync()
    s2.sync()
    assert np.array_equal(to_np(d1), to_np(d2))
    assert np.array_equal(to_np(u1), to_np(u2))


def test_advection_full_horizon_one_call():
    """The whole c1 run, 320 steps to T = 0.5, in one fr_sg_steps call against the oracle."""
    import torch
    announce("resident_1d", "advection_horizon")
    cfg = ADV
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    ref, t, n = ostep.solve(prob, u0, cfg["t_end"], tables=(T, R))
    sol = solver_for(cfg)
    sol.timing(True)
    ud = to_dev(u0)
    dts = torch.empty(n, dtype=torch.float64, device=ud.device)
    sol.steps(ud, n, dts)
    sol.sync()
    assert _resident(_passes(sol)) == "lds"
    assert abs(float(to_np(dts).sum()) - t) <= 1e-12 * t
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


def test_long_call_is_split_into_launches():
    """5000 steps: two launches (4096 + 904 steps) hand the CFL maximum on; the result equals
    5000 steps taken as 2500 + 2500 in two calls, and the time steps sum to the elapsed time."""
    import torch
    announce("resident_1d", "long_call")
    cfg = ADV
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    n = 5000
    a = solver_for(cfg)
    a.timing(True)
    ua = to_dev(u0)
    da = torch.empty(n, dtype=torch.float64, device=ua.device)
    a.steps(ua, n, da)
    a.sync()
    passes = a.timing_read()
    assert passes["steps_resident_lds"][0] == 2, passes
    b = solver_for(cfg)
    ub = to_dev(u0)
    db = torch.empty(n, dtype=torch.float64, device=ub.device)
    b.steps(ub, n // 2, db[: n // 2])
    b.steps(ub, n // 2, db[n // 2:])
    b.sync()
    assert np.array_equal(to_np(da), to_np(db))
    assert np.array_equal(to_np(ua), to_np(ub))
    assert np.all(to_np(da) > 0)


@pytest.mark.parametrize("label,cfg", [("threads", ADV_OVER), ("lds", BURG_OVER)])
def test_over_the_size_limit_runs_launched_stages(label, cfg):
    """One element past either limit: the steps take the three-launch path, with the oracle's results."""
    import torch
    announce("resident_1d", "over_limit", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    sol = solver_for(cfg)
    sol.timing(True)
    ud = to_dev(u0)
    dts = torch.empty(4, dtype=torch.float64, device=ud.device)
    sol.steps(ud, 4, dts)
    sol.sync()
    passes = _passes(sol)
    assert _resident(passes) is None and "stage1" in passes, passes
    ref = u0.copy()
    for _ in range(4):
        ref, _, _ = ostep.step(prob, ref, None, (T, R))
    assert rel_l2(to_np(ud), ref) < RTOL_FP64


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reduced_precisions_keep_launched_stages(precision):
    announce("resident_1d", "precision", precision)
    cfg = BURG
    prob, tabs = oracle_for(cfg)
    sol = solver_for(cfg, precision)
    sol.timing(True)
    u = to_dev(project_initial(prob, cfg["ic"], tabs))
    sol.steps(u, 2)
    sol.sync()
    assert _resident(_passes(sol)) is None

"""Pins for the oracle's time step, convergence and conservation."""

import math

import numpy as np
import pytest
from scipy.special import spherical_jn

from indep import chaos, dg_weak_rhs_1d, gl, lagrange_matrix
from oracle.fr import euler_pressure, nodal_at_solution_points
from oracle.initial import project_initial, solution_point_coords
from oracle.problem import Problem
from oracle.stepper import cfl_dt, solve, ssprk3, step
from oracle.tables import build_tables
from paper_2112_05946_amd import inputs



def test_ssprk3_amplification_polynomial():
    """u' = lam u: one step multiplies by 1 + z + z^2/2 + z^3/6 (Shu-Osher SSP-RK3)."""
    for lam in (-1.0, -2.5 + 1.0j, 0.3j, -0.1):
        for dt in (0.1, 0.37, 1.0):
            z = lam * dt
            u = np.array([1.0 + 0.5j])
            un, _ = ssprk3(u, dt, lambda w: lam * w)
            assert abs(un[0] - (1 + z + z * z / 2 + z ** 3 / 6) * u[0]) < 1e-14


def _exact_modes(prob, T, R, t):
    """c1 closed form: sin(2 pi (x - t) + 0.2 pi z) projected on Legendre chaos.

    E[e^{i a z} Phi_k] = sqrt(2k+1) i^k j_k(a) for z ~ U(-1, 1) (plane-wave expansion).
    """
    x, _ = solution_point_coords(prob, T)
    a = 0.2 * math.pi
    th = 2 * math.pi * (x - t)
    ex = np.zeros((1, R.M, prob.E, T.n))
    for k in range(R.M):
        c = math.sqrt(2 * k + 1) * spherical_jn(k, a)
        ex[0, k] = c * (-1) ** (k // 2) * (np.sin(th) if k % 2 == 0 else np.cos(th))
    return ex


def test_exact_modes_match_projection_of_initial_data():
    prob = Problem.from_config(inputs.ADVECTION)
    T, R = build_tables(prob)
    u0 = project_initial(prob, "advection_sine", (T, R))
    assert np.max(np.abs(u0 - _exact_modes(prob, T, R, 0.0))) < 5e-15


@pytest.mark.parametrize("p,expect", [(2, 3.0), (3, 4.0)])
def test_advection_closed_form_convergence(p, expect):
    errs = []
    for nx in (16, 32, 64):
        # SSP-RK3 is third order in time: a small CFL keeps its error below the p+1 spatial one
        prob = Problem.from_config(dict(inputs.ADVECTION, nx=nx, p=p, cfl=0.3 if p == 2 else 0.05))
        T, R = build_tables(prob)
        u, t, _ = solve(prob, project_initial(prob, "advection_sine", (T, R)), 0.5, tables=(T, R))
        d = u - _exact_modes(prob, T, R, t)
        errs.append(math.sqrt(np.sum(d * d * (T.w / 2)[None, None, None, :]) / nx))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(orders[-1] - expect) < 0.25, orders


def test_advection_c1_steps_and_dt():
    """CFL 0.3, 64 elements, p = 2: dt = 0.3 / (64 * 3) = 1/640, i.e. 320 steps to T = 0.5."""
    prob = Problem.from_config(inputs.ADVECTION)
    T, R = build_tables(prob)
    u0 = project_initial(prob, "advection_sine", (T, R))
    assert abs(cfl_dt(prob, T, R, u0) - 1.0 / 640.0) < 1e-18
    _, t, n = solve(prob, u0, 0.5, tables=(T, R))
    assert n == 320 and abs(t - 0.5) < 1e-13


def _totals(prob, T, u):
    wts = T.w / 2 if prob.dim == 1 else np.outer(T.w / 2, T.w / 2).ravel()
    return np.einsum("skej,j->sk", u, wts)


def test_conservation_with_filter_active():
    """Burgers past shock formation, periodic: the filter fires, the mean is conserved (lambda_00 = 1)."""
    cfg = inputs.small(inputs.BURGERS, 32)
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    u = project_initial(prob, cfg["ic"], (T, R))
    tot0 = _totals(prob, T, u)[:, 0]
    fired = 0
    for _ in range(400):
        u, dt, flags = step(prob, u, tables=(T, R))
        fired += int(flags[2].sum())
    assert fired > 0
    assert np.max(np.abs(_totals(prob, T, u)[:, 0] - tot0)) < 1e-12 * np.abs(tot0).max()


def test_conservation_with_limiter_active():
    prob = Problem(equation="euler1d", nx=24, p=3, gpc_order=4, nq1d=6, limiter=True,
                   filter="l2", sensor="detector", s0=-3 * math.log10(3), kappa=4.0)
    T, R = build_tables(prob)
    u = inputs.fuzz_euler(1, R.M, prob.E, 4, seed=4, vacuum_frac=0.2)
    u, f0 = __import__("oracle").limit(prob, T, R, u)
    assert f0.sum() > 0
    tot0 = _totals(prob, T, u)[:, 0]
    for _ in range(5):
        u, dt, flags = step(prob, u, dt=1e-4, tables=(T, R))
    assert np.max(np.abs(_totals(prob, T, u)[:, 0] - tot0)) < 1e-12 * np.abs(tot0).max()


def test_sod_uncertain_interface_needs_the_limiter():
    """Sec. 5.3 second case: plain SG fails at the first step; the limiter keeps it realizable."""
    for lim in (False, True):
        cfg = inputs.small(inputs.SOD, 100, limiter=lim)
        prob = Problem.from_config(cfg)
        T, R = build_tables(prob)
        u = project_initial(prob, cfg["ic"], (T, R))
        bad = False
        for _ in range(10):
            U = nodal_at_solution_points(R, u)
            with np.errstate(all="ignore"):
                if not np.all(np.isfinite(u)) or U[0].min() <= 0 or euler_pressure(U, prob.gamma, 1).min() <= 0:
                    bad = True
                    break
                u, _, _ = step(prob, u, tables=(T, R))
        assert bad == (not lim)


def test_burgers_sg_converges_to_collocation():
    """Smooth Burgers (T = 0.2 < 1/(0.7 pi)): SG moments -> brute-force collocation, spectrally in N_c."""
    nx, p, dt, nsteps = 16, 3, 2.5e-3, 80
    r, _ = gl(p + 1)
    xc = (np.arange(nx) + 0.5) * (2.0 / nx)
    x = xc[:, None] + (1.0 / nx) * r[None, :]
    zc, wc, _ = chaos(0, 48)

    def rk3(u, f):
        w1 = u + dt * f(u)
        w2 = 0.75 * u + 0.25 * (w1 + dt * f(w1))
        return u / 3 + 2.0 / 3.0 * (w2 + dt * f(w2))

    det = lambda u: dg_weak_rhs_1d("burgers", u, p, 0, 1, 2.0 / nx)
    col = []
    for zi in zc:
        u = (1 + 0.5 * np.sin(np.pi * x) + 0.2 * zi * np.sin(np.pi * x))[None, None]
        for _ in range(nsteps):
            u = rk3(u, det)
        col.append(u[0, 0])
    col = np.array(col)
    Ec = np.einsum("z,zej->ej", wc, col)
    Vc = np.einsum("z,zej->ej", wc, col * col) - Ec * Ec
    errs = []
    for order in (1, 2, 4):
        prob = Problem(equation="burgers", nx=nx, p=p, gpc_order=order, nq1d=2 * order + 2, xhi=2.0)
        T, R = build_tables(prob)
        u = project_initial(prob, "burgers_sine", (T, R))
        for _ in range(nsteps):
            u, _, _ = step(prob, u, dt=dt, tables=(T, R))
        errs.append(max(np.abs(u[0, 0] - Ec).max(), np.abs(np.sum(u[0, 1:] ** 2, axis=0) - Vc).max()))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6

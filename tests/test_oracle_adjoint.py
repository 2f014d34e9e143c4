"""Pins for the oracle's discrete adjoint (scalar 1D equations).

What fixes the adjoint without reference to itself:
* linear advection: the right-hand side and the step (filter on every element)
  are affine maps of the state, so <lam, L v> = <L^T lam, v> holds to rounding
  with L v = R(v) - R(0) from the forward oracle (exact dot-product identity);
  R is homogeneous of degree one in the advection speed a, so d<lam, R>/da =
  <lam, R(u)>/a exactly;
* Burgers: the right-hand side is piecewise quadratic, so central differences
  of the forward oracle reproduce the directional derivative up to rounding;
  for the step (degree 8 in the state) central differences with h = 1e-5 agree
  to O(h^2);
* the objective: J = integral of E[u^2] by nodal quadrature (independent of
  the modal sum), and its gradient by central differences.
"""

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fr as ofr
from oracle import stepper as ostep
from oracle.initial import project_initial
from oracle.problem import Problem
from oracle.tables import build_tables
from paper_2112_05946_amd import inputs


def _setup(cfg):
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    return prob, T, R


def _dot(a, b):
    return float(np.sum(a * b))


ADV_CASES = [
    ("periodic", dict(inputs.small(inputs.ADVECTION, 9))),
    ("dirichlet_outflow", dict(inputs.small(inputs.ADVECTION, 9), bc=["dirichlet", "outflow", "periodic", "periodic"],
                               bc_state=[[0.7, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]])),
    ("negative_speed", dict(inputs.small(inputs.ADVECTION, 9), adv_speed=-1.3)),
]


@pytest.mark.parametrize("label,cfg", ADV_CASES)
def test_advection_rhs_dot_product_exact(label, cfg):
    prob, T, R = _setup(cfg)
    rng = np.random.default_rng(1)
    shape = (1, R.M, prob.E, T.n)
    zero = np.zeros(shape)
    R0 = ofr.rhs(prob, T, R, zero)
    for _ in range(3):
        v = rng.standard_normal(shape)
        lam = rng.standard_normal(shape)
        Lv = ofr.rhs(prob, T, R, v) - R0
        g, _ = oadj.rhs_vjp(prob, T, R, v, lam)
        lhs, rhs_ = _dot(lam, Lv), _dot(g, v)
        assert abs(lhs - rhs_) <= 1e-13 * max(abs(lhs), np.linalg.norm(lam) * np.linalg.norm(Lv))


@pytest.mark.parametrize("label,cfg", ADV_CASES)
def test_advection_speed_derivative_homogeneity(label, cfg):
    prob, T, R = _setup(cfg)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((1, R.M, prob.E, T.n))
    lam = rng.standard_normal(u.shape)
    _, da = oadj.rhs_vjp(prob, T, R, u, lam)
    ref = _dot(lam, ofr.rhs(prob, T, R, u)) / prob.adv_speed
    assert abs(da - ref) <= 1e-12 * max(1.0, abs(ref))


def test_advection_step_dot_product_exact():
    """Exponential filter on every element: the whole step is linear in the state."""
    cfg = dict(inputs.small(inputs.ADVECTION, 10), filter="exp", alpha=36.0, s=8.0, sensor="always")
    prob, T, R = _setup(cfg)
    rng = np.random.default_rng(3)
    dt = 2e-3
    shape = (1, R.M, prob.E, T.n)
    flags = np.ones((4, prob.E), dtype=np.uint8)
    flags[[0, 1, 3]] = 0
    for _ in range(3):
        v = rng.standard_normal(shape)
        lam = rng.standard_normal(shape)
        Sv, _, fl = ostep.step(prob, v, dt, (T, R))
        assert np.array_equal(fl, flags)
        g, _ = oadj.step_vjp(prob, T, R, v, dt, flags, lam)
        lhs, rhs_ = _dot(lam, Sv), _dot(g, v)
        assert abs(lhs - rhs_) <= 1e-13 * max(abs(lhs), np.linalg.norm(lam) * np.linalg.norm(Sv))


def test_advection_step_speed_derivative_fd():
    cfg = dict(inputs.small(inputs.ADVECTION, 8), adv_speed=0.8)
    prob, T, R = _setup(cfg)
    rng = np.random.default_rng(4)
    u = project_initial(prob, cfg["ic"], (T, R))
    lam = rng.standard_normal(u.shape)
    dt = 1e-3
    _, _, flags = ostep.step(prob, u, dt, (T, R))
    _, da = oadj.step_vjp(prob, T, R, u, dt, flags, lam)
    h = 1e-5
    vals = []
    for a in (0.8 + h, 0.8 - h):
        p2 = Problem.from_config(dict(cfg, adv_speed=a))
        un, _, fl = ostep.step(p2, u, dt, (T, R))
        assert np.array_equal(fl, flags)
        vals.append(_dot(lam, un))
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(fd - da) <= 1e-8 * max(1.0, abs(da))


def _burgers():
    """Smooth projected initial state, rough (random modal) on half of the elements."""
    cfg = inputs.small(inputs.BURGERS, 12)
    prob, T, R = _setup(cfg)
    u = project_initial(prob, cfg["ic"], (T, R))
    u[:, :, ::2] += inputs.fuzz_scalar(R.M, prob.E, T.n, 7)[:, :, ::2]
    return cfg, prob, T, R, u


def test_burgers_rhs_central_differences():
    cfg, prob, T, R, u = _burgers()
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(u.shape)
    g, da = oadj.rhs_vjp(prob, T, R, u, lam)
    assert da == 0.0
    h = 1e-6
    for _ in range(20):
        v = rng.standard_normal(u.shape)
        v /= np.linalg.norm(v)
        fd = (_dot(lam, ofr.rhs(prob, T, R, u + h * v)) - _dot(lam, ofr.rhs(prob, T, R, u - h * v))) / (2 * h)
        assert abs(fd - _dot(g, v)) <= 1e-8 * np.linalg.norm(g)


def test_burgers_step_central_differences_20_directions():
    """Detector-switched exponential filter at frozen flags, fixed dt."""
    cfg, prob, T, R, u = _burgers()
    rng = np.random.default_rng(6)
    lam = rng.standard_normal(u.shape)
    dt = 4e-4
    _, _, flags = ostep.step(prob, u, dt, (T, R))
    assert flags[2].any() and not flags[2].all()   # both filter branches are exercised
    g, _ = oadj.step_vjp(prob, T, R, u, dt, flags, lam)
    h = 1e-5
    for _ in range(20):
        v = rng.standard_normal(u.shape)
        v /= np.linalg.norm(v)
        up, _, fp = ostep.step(prob, u + h * v, dt, (T, R))
        um, _, fm = ostep.step(prob, u - h * v, dt, (T, R))
        assert np.array_equal(fp, flags) and np.array_equal(fm, flags)
        fd = (_dot(lam, up) - _dot(lam, um)) / (2 * h)
        assert abs(fd - _dot(g, v)) <= 1e-7 * np.linalg.norm(g)


def test_filter_transpose_matches_matrix():
    """Filter adjoint == transpose of the filter matrix assembled column by column."""
    cfg = dict(inputs.small(inputs.BURGERS, 2), sensor="always")
    prob, T, R = _setup(cfg)
    from oracle.stabilize import sensor_filter
    n = R.M * prob.E * T.n
    A = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = sensor_filter(prob, T, R, e.reshape(1, R.M, prob.E, T.n), 3e-3)[0].ravel()
    g = np.random.default_rng(8).standard_normal(n)
    got = oadj.filter_vjp(prob, T, R, g.reshape(1, R.M, prob.E, T.n), np.ones(prob.E, bool), 3e-3).ravel()
    assert np.allclose(got, A.T @ g, rtol=0, atol=1e-14)


def test_objective_is_mean_square_by_quadrature():
    cfg, prob, T, R, u = _burgers()
    J = oadj.objective(prob, T, u)
    U = np.einsum("kq,kej->qej", R.Phi, u[0])               # nodal values at (node, element, point)
    Jq = (prob.dx / 2.0) * np.einsum("q,qej,j->", R.wq, U * U, T.w)
    assert abs(J - Jq) <= 1e-13 * J
    g = oadj.objective_grad(prob, T, u)
    rng = np.random.default_rng(9)
    h = 1e-3  # J is quadratic: central differences are exact up to rounding at any h
    for _ in range(5):
        v = rng.standard_normal(u.shape)
        fd = (oadj.objective(prob, T, u + h * v) - oadj.objective(prob, T, u - h * v)) / (2 * h)
        assert abs(fd - _dot(g, v)) <= 1e-11 * max(1.0, abs(fd))


def test_adjoint_rejects_what_it_does_not_cover():
    prob, T, R = _setup(inputs.small(inputs.SOD, 4))
    u = np.zeros((prob.S, R.M, prob.E, T.n))
    with pytest.raises(ValueError):
        oadj.rhs_vjp(prob, T, R, u, u)

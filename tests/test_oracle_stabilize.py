"""Pins for the oracle's sensor, filters and limiter (Sec. 4.1-4.3)."""

import math

import numpy as np
import pytest

from indep import chaos, gl, lagrange_matrix
from oracle.problem import Problem
from oracle.stabilize import (filter_strength, limit, pressure_root, sensor_filter, sensor_flags,
                              to_nodal, to_spatial_modal)
from oracle.tables import build_tables
from paper_2112_05946_amd import inputs


def _p(**kw):
    base = dict(equation="burgers", nx=6, p=3, gpc_order=4, nq1d=6, filter="l2", sensor="detector",
                s0=-3 * math.log10(3), kappa=4.0, eps1=0.6, eps2=0.6)
    base.update(kw)
    return Problem.from_config(base)


def test_l2_filter_strengths():
    """Eq. (filter function)/(l2 strength): lambda_00 = 1; last modes damped to 1/(1 + 1/eps)."""
    prob = _p(eps1=0.6, eps2=0.8)
    T, R = build_tables(prob)
    lam = filter_strength(prob, T, R, dt=0.1)
    assert lam[0, 0] == 1.0
    assert abs(lam[0, prob.p] - 1 / (1 + 1 / 0.6)) < 1e-15
    assert abs(lam[R.M - 1, 0] - 1 / (1 + 1 / 0.8)) < 1e-15
    assert np.all(np.diff(lam[0]) < 0) and np.all(np.diff(lam[:, 0]) < 0)


def test_exponential_filter_strengths():
    prob = _p(filter="exp", alpha=36.0, s=8.0)
    T, R = build_tables(prob)
    dt = 0.01
    lam = filter_strength(prob, T, R, dt)
    assert lam[0, 0] == 1.0
    assert abs(lam[0, prob.p] - math.exp(-36.0 * dt)) < 1e-15          # eta_x = 1
    assert abs(lam[R.M - 1, 0] - math.exp(-36.0 * dt)) < 1e-15         # eta_z = 1
    assert abs(lam[R.M - 1, prob.p] - math.exp(-72.0 * dt)) < 1e-15


def test_exponential_filter_cutoff():
    """Sec. 4.1.1 with N* = 2 (p = 3, N_c = 4): eta* = 2/3 in x, 1/2 in z.  Modes below
    both cutoffs are untouched, the factor is continuous (= 1) at the cutoff, the top
    modes are still damped by exp(-alpha dt), and eta = 3/4 in z gives
    ((3/4 - 1/2) / (1/2))^8 = 1/256 in the exponent (values worked by hand)."""
    prob = _p(filter="exp", alpha=36.0, s=8.0, nstar=2.0)
    T, R = build_tables(prob)
    dt = 0.01
    lam = filter_strength(prob, T, R, dt)
    for k in (0, 1):
        for j in (0, 1, 2):
            assert lam[k, j] == 1.0
    assert lam[2, 0] == 1.0                                              # eta_z = 1/2 = eta*
    assert abs(lam[0, 3] - math.exp(-36.0 * dt)) < 1e-15
    assert abs(lam[4, 0] - math.exp(-36.0 * dt)) < 1e-15
    assert abs(lam[4, 3] - math.exp(-72.0 * dt)) < 1e-15
    assert abs(lam[3, 0] - math.exp(-36.0 * dt / 256.0)) < 1e-15
    assert abs(lam[3, 3] - math.exp(-36.0 * dt * (1.0 + 1.0 / 256.0))) < 1e-15
    assert np.all(np.diff(lam, axis=0) <= 0) and np.all(np.diff(lam, axis=1) <= 0)
    # 2D tensor modes (p = 3, N* = 1): eta* = 1/3 in each direction, per-direction terms add
    p2 = Problem.from_config(dict(equation="euler2d", nx=2, ny=2, p=3, gpc_order=2, nq1d=3, rdim=2,
                                  filter="exp", alpha=36.0, s=2.0, nstar=1.0))
    T2, R2 = build_tables(p2)
    lam2 = filter_strength(p2, T2, R2, dt)
    for j in range(16):
        a, b = j % 4, j // 4
        tx = sum(0.0 if d / 3 < 1 / 3 else ((d / 3 - 1 / 3) / (2 / 3)) ** 2 for d in (a, b))
        assert abs(lam2[0, j] - math.exp(-36.0 * dt * tx)) < 1e-15
    assert lam2[0, 1 + 4] == 1.0 and lam2[1, 0] == 1.0 and lam2[2, 0] == 1.0       # (1,1) x and |k| = 1


def test_filter_nodal_form_equals_modal_form():
    """F* = V Lambda o V^-1 on nodal values (Sec. 4.1.1) equals filtering the modal coefficients."""
    prob = _p(sensor="always")
    T, R = build_tables(prob)
    u = inputs.fuzz_scalar(R.M, prob.E, 4, seed=9)
    out, flags = sensor_filter(prob, T, R, u, dt=0.05)
    assert flags.all()
    lam = filter_strength(prob, T, R, 0.05)
    # independent: modal coefficients by Gauss quadrature against sqrt(2j+1) P_j
    r, w = gl(4)
    Psi = np.array([math.sqrt(2 * j + 1) * np.polynomial.legendre.legval(r, np.eye(4)[j]) for j in range(4)])
    modal = np.einsum("j,mj,skej->skem", w / 2, Psi, u)
    back = np.einsum("mj,skem->skej", Psi, modal * lam[None, :, None, :])
    assert np.max(np.abs(out - back)) < 1e-13
    # the element x random mean (mode (0, 0)) is untouched
    m0 = np.einsum("j,skej->ske", w / 2, out)[:, 0]
    assert np.max(np.abs(m0 - np.einsum("j,skej->ske", w / 2, u)[:, 0])) < 1e-14


def test_two_dim_spatial_modal_roundtrip():
    prob = Problem(equation="euler2d", nx=2, ny=2, p=3, gpc_order=2, nq1d=3, rdim=2)
    T, R = build_tables(prob)
    u = inputs.fuzz_euler(2, R.M, prob.E, 16, seed=1)
    assert np.max(np.abs(to_nodal(prob, T, to_spatial_modal(prob, T, u)) - u)) < 1e-13


def test_sensor_smooth_and_discontinuous_cases():
    """Eq. (detector): no flag without outer-shell energy; a jump inside an element is flagged."""
    prob = _p(nx=3, gpc_order=4, nq1d=6)
    T, R = build_tables(prob)
    u = np.zeros((1, R.M, 3, 4))
    # element 0: quadratic in x (degree < p), chaos modes below N_c
    u[0, 0, 0] = 1.0 + 0.3 * T.r + 0.2 * T.r ** 2
    u[0, 2, 0] = 0.1 * T.r
    # element 1: zero state (zero denominator, not flagged)
    # element 2: a jump between solution points
    u[0, 0, 2] = np.array([1.0, 1.0, 0.0, 0.0])
    flags = sensor_flags(prob, T, R, u)
    assert list(flags) == [False, False, True]
    # energy in the last chaos mode alone is the outer shell too
    u2 = np.zeros_like(u)
    u2[0, 0, 0] = 1.0
    u2[0, R.M - 1, 0] = 0.5
    assert sensor_flags(prob, T, R, u2)[0]


# ----------------------------------------------------------------------------
# limiter
# ----------------------------------------------------------------------------

def _nodal_points_indep(u, p, order, nq, dim=1):
    """Density/pressure at (solution + face points) x nodes with test-side tables."""
    r, _ = gl(p + 1)
    z, wq, Phi = chaos(order, nq)
    U = np.einsum("kq,skej->sqej", Phi, u)
    Lf = lagrange_matrix(r, [-1.0, 1.0])
    F = np.einsum("fj,sqej->sqef", Lf, U)
    return np.concatenate([U, F], axis=-1)


def _press(U, g=1.4):
    return (g - 1) * (U[2] - 0.5 * U[1] ** 2 / U[0])


def test_limiter_restores_positivity_and_keeps_means():
    prob = Problem(equation="euler1d", nx=40, p=3, gpc_order=4, nq1d=6, limiter=True)
    T, R = build_tables(prob)
    u = inputs.fuzz_euler(1, R.M, prob.E, 4, seed=12, vacuum_frac=0.3)
    before = _nodal_points_indep(u, 3, 4, 6)
    assert (before[0].min() < 0) or (_press(before).min() < 0)
    out, flags = limit(prob, T, R, u)
    assert flags.sum() >= 10
    after = _nodal_points_indep(out, 3, 4, 6)
    wts = T.w / 2
    means0 = np.einsum("sej,j->se", u[:, 0], wts)
    means1 = np.einsum("sej,j->se", out[:, 0], wts)
    eps = np.minimum(1e-8, np.minimum(means0[0], _press(means0)))
    assert np.all(after[0].min(axis=(0, 2)) >= eps * (1 - 1e-6) - 1e-14)
    assert np.all(_press(after).min(axis=(0, 2)) >= eps * (1 - 1e-6) - 1e-13)
    assert np.max(np.abs(means1 - means0)) < 1e-14
    # untouched elements are bitwise identical
    assert np.array_equal(out[:, :, ~flags], u[:, :, ~flags])


def test_limiter_closed_form_beta1():
    """One deterministic p=1 element whose face density is negative: beta1 = (rho_bar-eps)/(rho_bar-rho_min)."""
    prob = Problem(equation="euler1d", nx=1, p=1, gpc_order=0, nq1d=1, limiter=True)
    T, R = build_tables(prob)
    rb, d = 0.5, 0.4                       # rho at r = -+1/sqrt(3): rb -+ d; at r = -1: rb - sqrt(3) d < 0
    u = np.zeros((3, 1, 1, 2))
    u[0, 0, 0] = [rb - d, rb + d]
    u[2, 0, 0] = [2.5, 2.5]
    out, flags = limit(prob, T, R, u)
    eps = 1e-8
    beta1 = (rb - eps) / (math.sqrt(3.0) * d)
    assert flags[0]
    assert np.allclose(out[0, 0, 0], [rb - beta1 * d, rb + beta1 * d], atol=1e-15, rtol=0)
    assert np.array_equal(out[2], u[2])


def test_pressure_root_matches_bisection():
    rng = np.random.default_rng(0)
    g, eps = 1.4, 1e-8
    prob = Problem(equation="euler1d", nx=1, p=1, gpc_order=0, nq1d=1, gamma=g)
    press = lambda w: (g - 1) * (w[2] - 0.5 * w[1] ** 2 / w[0])
    count = 0
    while count < 200:
        ubar = np.array([rng.uniform(0.1, 2), rng.uniform(-1, 1), 0.0])
        ubar[2] = rng.uniform(0.05, 2) / (g - 1) + 0.5 * ubar[1] ** 2 / ubar[0]
        star = ubar + rng.normal(0, 1.0, 3) * np.array([0.5 * ubar[0], 1.0, 1.0])
        if star[0] <= eps or press(star) >= eps:
            continue
        beta = pressure_root(prob, ubar[:, None], star[:, None], eps)[0]
        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if press(mid * (star - ubar) + ubar) > eps:
                lo = mid
            else:
                hi = mid
        assert 0.0 < beta < 1.0
        assert abs(beta - lo) < 1e-12
        count += 1


def test_limiter_inactive_is_identity():
    prob = Problem(equation="euler1d", nx=10, p=2, gpc_order=3, nq1d=5, limiter=True)
    T, R = build_tables(prob)
    u = inputs.fuzz_euler(1, R.M, prob.E, 3, seed=2)
    out, flags = limit(prob, T, R, u)
    assert not flags.any() and np.array_equal(out, u)

"""Pins of the oracle's time-step rules by the stability of SSP-RK3 with the
assembled FR operator.

The paper gives CFL numbers (Tables 1, 4-6) but no formula for the time step.
The rules read here are dt = CFL dx / ((p+1) lambda) in 1D,
dt = CFL / ((p+1) max(lambda_x/dx + lambda_y/dy)) on rectangles and
dt = CFL / ((p+1) max(lambda/d_e)) on triangles (d_e the inscribed diameter).
What fixes their constants is the mathematics of the method: the SSP-RK3
amplification factor g(z) = 1 + z + z^2/2 + z^3/6 must stay within the unit
disc for z = dt mu over every eigenvalue mu of the (linearised) semi-discrete
operator.  The operator of a periodic, translation-invariant mesh is
block-circulant, so its eigenvalues are those of the Fourier symbol
sum_d B_d exp(i theta . d), with the blocks B_d read from the oracle's own
right-hand side (linear advection directly; the Euler equations linearised
about a uniform state by a complex step, exact to rounding).

Pinned: every rule is stable at the workloads' CFL 0.3; in 1D the largest
stable CFL for p = 2 equals 3 x 0.209, the known stability limit
lambda dt / dx = 0.209 of P2 discontinuous Galerkin with third-order
Runge-Kutta (Cockburn and Shu, J. Sci. Comput. 16, 2001, Table 2.2); on 2 x 1
rectangles the 2D limit is the 1D limit for flow along x, along y and
diagonally (so the rule weighs the two directions with their own cell sizes);
on triangles the limit stays within [0.4, 1.0] (a margin over 0.3, and not
over-conservative by the factor 2 a radius-for-diameter slip would give).
"""

import numpy as np
import pytest

from oracle.fr import rhs
from oracle.problem import Problem
from oracle.stepper import cfl_dt
from oracle.tables import build_tables
from paper_2112_05946_amd import inputs

GAMMA = 1.4


def _amp(z):
    return np.abs(1.0 + z + z * z / 2.0 + z ** 3 / 6.0)


def _limit(mus, tol):
    """Largest CFL with max |g(cfl mu)| <= 1 + tol (bisection)."""
    lo, hi = 0.01, 4.0
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if _amp(mid * mus).max() > 1.0 + tol:
            hi = mid
        else:
            lo = mid
    return lo


def _symbol_eigs(blocks, thetas):
    out = []
    for tx in thetas:
        for ty in thetas:
            S = sum(B * np.exp(1j * (tx * a + ty * b)) for (a, b), B in blocks.items())
            out.append(np.linalg.eigvals(S))
    return np.concatenate(out)


def _uniform(prob, E, npt, vel):
    base = np.zeros((4, 1, E, npt))
    rho, p = 1.0, 1.0 / GAMMA
    base[0] = rho
    base[1] = rho * vel[0]
    base[2] = rho * vel[1]
    base[3] = p / (GAMMA - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2)
    return base


def _jacobian_columns(prob, T, R, base, elems):
    """d rhs / d u for every coefficient of the listed elements (complex step)."""
    S, M, E, npt = base.shape
    cols = []
    for e in elems:
        for s in range(S):
            for j in range(npt):
                d = np.zeros(base.shape, dtype=complex)
                d[s, 0, e, j] = 1e-30j
                cols.append((rhs(prob, T, R, base + d).imag / 1e-30).reshape(S, E, npt))
    return np.stack(cols, axis=-1)


def _advection_eigs(p):
    prob = Problem.from_config(dict(equation="advection", nx=3, p=p, gpc_order=0, nq1d=1, adv_speed=1.0))
    T, R = build_tables(prob)
    n = p + 1
    L = np.zeros((3 * n, 3 * n))
    for c in range(3 * n):
        u = np.zeros((1, 1, 3, n))
        u.reshape(-1)[c] = 1.0
        L[:, c] = rhs(prob, T, R, u).reshape(-1)
    blocks = {(d, 0): L[n:2 * n, ((1 + d) % 3) * n:((1 + d) % 3 + 1) * n] for d in (-1, 0, 1)}
    dt_per_cfl = cfl_dt(prob, T, R, np.ones((1, 1, 3, n))) / prob.cfl
    return np.concatenate([np.linalg.eigvals(sum(B * np.exp(1j * t * d) for (d, _), B in blocks.items()))
                           for t in np.linspace(0.0, 2.0 * np.pi, 1001)]) * dt_per_cfl


@pytest.mark.parametrize("p", [1, 2, 3])
def test_1d_rule_stable_at_cfl_03_and_p2_limit_is_published(p):
    mus = _advection_eigs(p)
    assert _amp(0.3 * mus).max() <= 1.0 + 1e-13
    lim = _limit(mus, 1e-12)
    assert lim > 0.4
    if p == 2:
        assert abs(lim / 3.0 - 0.209) < 0.002


def _rect_eigs(p, vel):
    prob = Problem.from_config(dict(equation="euler2d", nx=3, ny=3, p=p, gpc_order=0, nq1d=1, rdim=1,
                                    xlo=0.0, xhi=2.0, ylo=0.0, yhi=1.0))
    assert abs(prob.dx - 2.0 * prob.dy) < 1e-15
    T, R = build_tables(prob)
    n2 = (p + 1) ** 2
    base = _uniform(prob, 9, n2, vel)
    Lc = _jacobian_columns(prob, T, R, base, [4])          # the centre element (1, 1)
    blocks = {(1 - e % 3, 1 - e // 3): Lc[:, e].reshape(4 * n2, 4 * n2) for e in range(9)}
    dt_per_cfl = cfl_dt(prob, T, R, base) / prob.cfl
    return _symbol_eigs(blocks, np.linspace(0.0, 2.0 * np.pi, 25)) * dt_per_cfl


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("vel", [(1.5, 0.0), (0.0, 1.5), (0.6, 0.3)])
def test_2d_rule_on_rectangles_matches_1d_limit(p, vel):
    mus = _rect_eigs(p, vel)
    assert _amp(0.3 * mus).max() <= 1.0 + 1e-12
    lim2 = _limit(mus, 1e-12)
    lim1 = _limit(_advection_eigs(p), 1e-12)
    assert abs(lim2 - lim1) < 0.05, (lim2, lim1)


def _tri_eigs(p, vel):
    nx = ny = 3
    mesh = inputs.tri_mesh_rectangle(nx, ny, xhi=2.0, yhi=1.0)
    prob = Problem.from_config(dict(equation="euler2d", element="tri", mesh=mesh, nx=1, ny=1, p=p, gpc_order=0,
                                    nq1d=1, rdim=1, bc=["outflow"] * 4))
    T, R = build_tables(prob)
    E, npt = prob.E, prob.nsp
    base = _uniform(prob, E, npt, vel)
    cell = lambda i, j: 2 * ((j % ny) * nx + (i % nx))
    c0 = cell(1, 1)
    Lc = _jacobian_columns(prob, T, R, base, [c0, c0 + 1])   # the two triangles of the centre cell
    blocks = {}
    for j in range(ny):
        for i in range(nx):
            e0 = cell(i, j)
            blocks[(1 - i, 1 - j)] = np.concatenate([Lc[:, e0 + t].reshape(4 * npt, -1) for t in (0, 1)], axis=0)
    dt_per_cfl = cfl_dt(prob, T, R, base) / prob.cfl
    return _symbol_eigs(blocks, np.linspace(0.0, 2.0 * np.pi, 17)) * dt_per_cfl


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("vel", [(0.0, 0.0), (1.5, 0.0)])
def test_triangle_rule_stable_with_margin(p, vel):
    mus = _tri_eigs(p, vel)
    assert _amp(0.3 * mus).max() <= 1.0 + 1e-12
    lim = _limit(mus, 1e-12)
    assert 0.4 <= lim <= 1.0, lim

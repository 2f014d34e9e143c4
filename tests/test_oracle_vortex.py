"""Pin of the oracle's 2D Euler step on rectangular cells: an isentropic vortex
convected by a uniform flow (Sec. 5.4 vortex form; tensor FR of Sec. 3.5).

The cells are twice as long in x as in y, so every term that scales with the
cell size in one direction is exercised against its own Jacobian.  The exact
solution at each random node is the initial field translated by that node's
free-stream velocity.  The error is the L2 norm over the elements (7-point
Gauss rule per direction applied to the solution polynomial, at every random
node), relative to the norm of the exact state.  For discontinuous Galerkin
schemes (which FR with Radau corrections is) on smooth hyperbolic problems the
L2 error decays at an order between p + 1/2 (the general bound) and p + 1; the
fitted order over three meshes must lie in that range (with 0.1 of slack),
and the finest error must be small.
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.fr import nodal_at_solution_points, rhs
from oracle.initial import project_initial, solution_point_coords
from oracle.problem import Problem
from oracle.stepper import cfl_dt, ssprk3
from oracle.tables import build_tables
from paper_2112_05946_amd import inputs

T_END = 0.1


def _l2_error(prob, T, R, u, t):
    n = prob.p + 1
    g, gw = npleg.leggauss(7)
    # Lagrange basis of the solution points evaluated at the fine rule (numpy's Legendre routines)
    Lg = npleg.legvander(g, n - 1) @ np.linalg.inv(npleg.legvander(T.r, n - 1))
    U = nodal_at_solution_points(R, u).reshape(4, R.Nq, prob.E, n, n)        # [s, q, e, b, a]
    Uf = np.einsum("ia,jb,sqeba->sqeji", Lg, Lg, U)
    ix = np.arange(prob.E) % prob.nx
    iy = np.arange(prob.E) // prob.nx
    Xf = (ix[:, None, None] + 0.5) * prob.dx + 0.5 * prob.dx * g[None, None, :] + 0.0 * g[None, :, None]
    Yf = (iy[:, None, None] + 0.5) * prob.dy + 0.5 * prob.dy * g[None, :, None] + 0.0 * g[None, None, :]
    Ue = np.stack([inputs.vortex_convection_exact(Xf, Yf, zq, t) for zq in R.z[:, 0]], axis=1)
    W = np.outer(gw, gw)[None, None, None]
    return np.sqrt(np.sum(W * (Uf - Ue) ** 2) / np.sum(W * Ue ** 2))


def _convect(p, n):
    prob = Problem.from_config(inputs.vortex_convection(n, p))
    assert abs(prob.dx - 2.0 * prob.dy) < 1e-15
    T, R = build_tables(prob)
    u = project_initial(prob, "vortex_convection", (T, R))
    t = 0.0
    while t < T_END - 1e-14:
        dt = min(cfl_dt(prob, T, R, u), T_END - t)
        u, _ = ssprk3(u, dt, lambda w: rhs(prob, T, R, w))
        t += dt
    return _l2_error(prob, T, R, u, T_END)


def test_vortex_exact_solution_is_steady_in_the_moving_frame():
    """The problem statement itself: radial equilibrium makes the translated vortex an
    Euler solution; check the residual of the exact field by central differences."""
    h = 1e-4
    x, y = np.meshgrid(np.linspace(0.6, 1.4, 9), np.linspace(0.2, 0.8, 9))
    z = 0.3

    def flux(U):
        rho, mx, my, E = U
        u, v = mx / rho, my / rho
        p = 0.4 * (E - 0.5 * rho * (u * u + v * v))
        return (np.stack([mx, mx * u + p, my * u, (E + p) * u]), np.stack([my, mx * v, my * v + p, (E + p) * v]))

    dUdt = (inputs.vortex_convection_exact(x, y, z, h) - inputs.vortex_convection_exact(x, y, z, -h)) / (2 * h)
    dF = (flux(inputs.vortex_convection_exact(x + h, y, z, 0))[0]
          - flux(inputs.vortex_convection_exact(x - h, y, z, 0))[0]) / (2 * h)
    dG = (flux(inputs.vortex_convection_exact(x, y + h, z, 0))[1]
          - flux(inputs.vortex_convection_exact(x, y - h, z, 0))[1]) / (2 * h)
    assert np.max(np.abs(dUdt + dF + dG)) < 1e-6 * np.max(np.abs(dF))


@pytest.mark.parametrize("p,meshes", [(2, (8, 16, 24)), (3, (8, 16, 24))])
def test_vortex_convection_order_on_rectangles(p, meshes):
    errs = np.array([_convect(p, n) for n in meshes])
    h = 1.0 / np.asarray(meshes, dtype=float)
    order = np.polyfit(np.log(h), np.log(errs), 1)[0]
    print("p=%d errors %s fitted order %.2f" % (p, errs, order))
    assert p + 0.4 <= order <= p + 1.1
    assert errs[-1] < (4e-4 if p == 2 else 1e-4)

"""Time step: three-stage SSP Runge-Kutta around the FR-SG right-hand side.

The paper writes the fully discrete scheme for forward Euler (Eq.
schemefullDiscr): limit, update, filter, and notes that other integrators are
possible.  Here each forward-Euler stage of the Shu-Osher SSP-RK3 scheme is
followed by the limiter, and the sensor-gated filter runs once at the end of
the step (the exponential filter strength contains the step size), followed by
the limiter:

  w1 = Lim(u + dt R(u))
  w2 = Lim(3/4 u + 1/4 (w1 + dt R(w1)))
  v  = 1/3 u + 2/3 (w2 + dt R(w2))
  u+ = Lim(Filter(v))

Time-step restriction (parity unpinned as to the constant; the paper gives CFL
numbers but no formula): dt = CFL dx / ((p+1) lambda_max) in 1D and
dt = CFL / ((p+1) max(lambda_x/dx + lambda_y/dy)) in 2D, the maxima taken over
solution points x random nodes of the state at the start of the step.
"""

import numpy as np

from .fr import nodal_at_solution_points, rhs, speed_x, speed_y
from .stabilize import limit, sensor_filter
from .tables import build_tables


def ssprk3(u, dt, R, L=lambda w: (w, None), F=lambda w: (w, None), record=None):
    """Generic SSP-RK3 step with stage post-processing L and end-of-step F.

    R(u) is the right-hand side; L and F return (state, flags).  If `record`
    is a list, the inputs of the four switch passes are appended to it.
    """
    a = u + dt * R(u)
    w1, f1 = L(a)
    b = 0.75 * u + 0.25 * (w1 + dt * R(w1))
    w2, f2 = L(b)
    v = (1.0 / 3.0) * u + (2.0 / 3.0) * (w2 + dt * R(w2))
    vf, ff = F(v)
    un, f3 = L(vf)
    if record is not None:
        record.extend([a, b, v, vf])
    return un, (f1, f2, ff, f3)


def cfl_dt(prob, T, R, u):
    U = nodal_at_solution_points(R, u)
    n = prob.p + 1
    if prob.dim == 1:
        lam = speed_x(prob, U).max()
        return prob.cfl * prob.dx / (n * lam)
    rate = speed_x(prob, U) / prob.dx + speed_y(prob, U) / prob.dy
    return prob.cfl / (n * rate.max())


def step(prob, u, dt=None, tables=None, record=None):
    """One SSP-RK3 step.  Returns (u_new, dt_used, flags[4, E] uint8).

    flags rows: limiter after stage 1, limiter after stage 2, sensor/filter at
    the end of the step, limiter at the end of the step.  `record`: optional
    list that receives the inputs of those four passes.
    """
    T, R = tables if tables is not None else build_tables(prob)
    if dt is None or dt <= 0.0:
        dt = cfl_dt(prob, T, R, u)
    E = u.shape[2]
    none = np.zeros(E, dtype=bool)

    def Lim(w):
        if not prob.limiter:
            return w, none
        return limit(prob, T, R, w)

    def Filt(w):
        return sensor_filter(prob, T, R, w, dt)

    un, (f1, f2, ff, f3) = ssprk3(u, dt, lambda w: rhs(prob, T, R, w), Lim, Filt, record)
    flags = np.stack([f1, f2, ff, f3]).astype(np.uint8)
    return un, dt, flags


def solve(prob, u0, t_end, max_steps=10**9, tables=None):
    """Advance to t_end with CFL steps, the last one clipped to land on t_end."""
    T, R = tables if tables is not None else build_tables(prob)
    u, t, nsteps = u0.copy(), 0.0, 0
    while t < t_end - 1e-14 * max(1.0, t_end) and nsteps < max_steps:
        dt = cfl_dt(prob, T, R, u)
        if t + dt > t_end:
            dt = t_end - t
        u, _, _ = step(prob, u, dt, (T, R))
        t += dt
        nsteps += 1
    return u, t, nsteps

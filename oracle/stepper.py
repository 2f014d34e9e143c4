"""Time step: three-stage SSP Runge-Kutta around the FR-SG right-hand side, or
one of the paper's explicit integrators (RK4, Bogacki-Shampine 3(2),
Tsitouras 5(4)) at the same CFL step.

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

Time-step restriction (the paper gives CFL numbers but no formula):
dt = CFL dx / ((p+1) lambda_max) in 1D and
dt = CFL / ((p+1) max(lambda_x/dx + lambda_y/dy)) in 2D, the maxima taken over
solution points x random nodes of the state at the start of the step.  Its
constants are pinned by the stability of SSP-RK3 with the assembled operator:
stable at CFL 0.3, and for p = 2 the limit is 3 x 0.209, the published
lambda dt / dx limit of P2 discontinuous Galerkin with third-order Runge-Kutta;
in 2D the limit on 2 x 1 cells equals the 1D one for every flow direction.
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


# Explicit Runge-Kutta tableaux (A strictly lower triangular, weights b, nodes c)
# of the paper's integrators: RK4 (Table 1), Tsitouras 5(4) (Table 4),
# Bogacki-Shampine 3(2) (Tables 5, 6).  They are used with the CFL step, so
# only the propagating weights enter; the stages that exist for the embedded
# error estimate (the first-same-as-last stage) are left out.
TABLEAUS = {
    "rk4": (
        [[0.0, 0.0, 0.0, 0.0],
         [0.5, 0.0, 0.0, 0.0],
         [0.0, 0.5, 0.0, 0.0],
         [0.0, 0.0, 1.0, 0.0]],
        [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0],
        [0.0, 0.5, 0.5, 1.0]),
    "bs3": (
        [[0.0, 0.0, 0.0],
         [0.5, 0.0, 0.0],
         [0.0, 0.75, 0.0]],
        [2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0],
        [0.0, 0.5, 0.75]),
    "tsit5": (
        [[0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
         [0.161, 0.0, 0.0, 0.0, 0.0, 0.0],
         [-0.008480655492356989, 0.335480655492357, 0.0, 0.0, 0.0, 0.0],
         [2.897153057105493, -6.359448489975075, 4.3622954328695815, 0.0, 0.0, 0.0],
         [5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525, 0.0, 0.0],
         [5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401, -0.028269050394068383,
          0.0]],
        [0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081,
         2.324710524099774],
        [0.0, 0.161, 0.327, 0.9, 0.9800255409045097, 1.0]),
}


def explicit_rk(u, dt, R, tableau, L=lambda w: (w, None), F=lambda w: (w, None), record=None):
    """One explicit Runge-Kutta step with Butcher tableau (A, b, c): stage states
    Y_1 = u, Y_i = L(u + dt sum_{j<i} A_ij K_j), K_i = R(Y_i); then
    u+ = L(F(u + dt sum_i b_i K_i)).  Returns (u+, (any stage limiter flag, None,
    filter flags, end limiter flags))."""
    A, b, _ = tableau
    K = []
    fany = None
    for i in range(len(b)):
        if i == 0:
            Y = u
        else:
            acc = np.zeros_like(u)
            for j in range(i):
                if A[i][j] != 0.0:
                    acc = acc + A[i][j] * K[j]
            Y, fl = L(u + dt * acc)
            if fl is not None:
                fany = fl if fany is None else (fany | fl)
        K.append(R(Y))
    acc = np.zeros_like(u)
    for i in range(len(b)):
        if b[i] != 0.0:
            acc = acc + b[i] * K[i]
    v = u + dt * acc
    vf, ff = F(v)
    un, f3 = L(vf)
    if record is not None:
        record.extend([None, None, v, vf])
    return un, (fany, None, ff, f3)


def cfl_dt(prob, T, R, u):
    if prob.element == "tri":
        from .tri import cfl_dt_tri
        return cfl_dt_tri(prob, T, R, u)
    U = nodal_at_solution_points(R, u)
    n = prob.p + 1
    if prob.dim == 1:
        lam = speed_x(prob, U).max()
        return prob.cfl * prob.dx / (n * lam)
    rate = speed_x(prob, U) / prob.dx + speed_y(prob, U) / prob.dy
    return prob.cfl / (n * rate.max())


def step(prob, u, dt=None, tables=None, record=None):
    """One step of the configured integrator (SSP-RK3 unless prob.integrator
    names one of TABLEAUS).  Returns (u_new, dt_used, flags[4, E] uint8).

    flags rows: limiter after stage 1, limiter after stage 2, sensor/filter at
    the end of the step, limiter at the end of the step (for the tableau
    integrators: row 0 = limiter acted on any stage state, row 1 = 0).
    `record`: optional list that receives the inputs of those four passes
    (None where a pass has no single input).
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

    Rf = lambda w: rhs(prob, T, R, w)
    if prob.integrator == "ssprk3":
        un, (f1, f2, ff, f3) = ssprk3(u, dt, Rf, Lim, Filt, record)
    else:
        un, (f1, f2, ff, f3) = explicit_rk(u, dt, Rf, TABLEAUS[prob.integrator], Lim, Filt, record)
        f1 = none if f1 is None else f1
        f2 = none
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

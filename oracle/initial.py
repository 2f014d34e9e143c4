"""Initial gPC coefficients (Sec. 2.1, Eq. sg conservation laws, third line).

u_k(0, x) = <u0(x, z) Phi_k>, evaluated with the random quadrature rule
(Eq. discrete expectation value) at every solution point x of every element.
Euler data are converted to conservative variables before projection (the
shared input module returns conservative states).  The projected state is
limited once, so that every right-hand-side input is limited.
"""

import numpy as np

from paper_2112_05946_amd.inputs import initial_condition

from .stabilize import limit
from .tables import build_tables


def solution_point_coords(prob, T):
    """Physical coordinates of every solution point: x[e, j], y[e, j]."""
    if prob.element == "tri":
        from .tri import solution_point_coords_tri
        return solution_point_coords_tri(prob, T)
    xc = prob.xlo + (np.arange(prob.nx) + 0.5) * prob.dx
    if prob.dim == 1:
        x = xc[:, None] + 0.5 * prob.dx * T.r[None, :]
        return x, np.zeros_like(x)
    yc = prob.ylo + (np.arange(prob.ny) + 0.5) * prob.dy
    n = T.n
    # element e = iy*nx + ix, point j = a + n*b
    X = xc[None, :, None, None] + 0.5 * prob.dx * T.r[None, None, None, :]
    Y = yc[:, None, None, None] + 0.5 * prob.dy * T.r[None, None, :, None]
    X = np.broadcast_to(X, (prob.ny, prob.nx, n, n)).reshape(prob.E, n * n)
    Y = np.broadcast_to(Y, (prob.ny, prob.nx, n, n)).reshape(prob.E, n * n)
    return X, Y


def project_initial(prob, ic_name, tables=None, apply_limiter=True):
    T, R = tables if tables is not None else build_tables(prob)
    x, y = solution_point_coords(prob, T)
    # evaluate u0 at (x, z_q): shape [S, Nq, E, Nsp]
    Xq = np.broadcast_to(x[None], (R.Nq,) + x.shape)
    Yq = np.broadcast_to(y[None], (R.Nq,) + y.shape)
    Zq = np.broadcast_to(R.z[:, None, None, :], (R.Nq,) + x.shape + (R.rdim,))
    U0 = initial_condition(ic_name, Xq, Yq, Zq, prob.gamma)
    u = np.einsum("kq,sqej->skej", R.PW, U0)
    if apply_limiter and prob.limiter:
        u, _ = limit(prob, T, R, u)
    return u

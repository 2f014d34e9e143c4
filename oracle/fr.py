"""Semi-discrete FR-SG right-hand side, FP64, in the paper's order of operations.

For each element and each gPC mode k (Sec. 2.1 Eq. sg conservation laws,
Sec. 3.2-3.5):

1. evaluate the gPC expansion at the random quadrature nodes,
   U_q = sum_k u_k Phi_k(z_q), at every solution point (Eq. polynomial chaos);
2. evaluate the physical flux f(U_q) and Galerkin-project it,
   f_k = sum_q w_q Phi_k(z_q) f(U_q)  (Eq. discrete expectation value), which
   gives the discontinuous flux at the solution points (Eq. local direct flux);
3. interpolate the solution to the element faces per node (Lagrange
   interpolation, Sec. 3.2) and form the interactive flux there with the
   Lax-Friedrichs (Rusanov) solver, per node, with the dissipation speed the
   larger spectral radius of the two traces (Sec. 3.3), or with the HLL
   solver (Euler equations), then project it;
4. interpolate the projected discontinuous flux polynomial to the faces
   (Eq. discontinuous flux polynomial);
5. total-flux derivative at the solution points: sum_l f_l l_l'(r_j) plus the
   Radau corrections (f^I_L - f^D_L) h_L'(r_j) + (f^I_R - f^D_R) h_R'(r_j)
   (Sec. 3.4), divided by the Jacobian J = dx/2 (Eq. local direct flux);
6. du/dt = -(that derivative) (Eq. fr update).  In 2D, the tensor-product
   extension of Sec. 3.5 applies the same along each coordinate line and sums
   the x and y parts.

State layout: u[s, k, e, j] (state, gPC mode, element, solution point); in 2D
e = iy * nx + ix and j = a + (p+1) * b with a along x.

Boundary operator (Sec. 2.1, <B(u) Phi_k> = 0): ghost traces per node.
periodic wraps; dirichlet uses a fixed conservative state; outflow copies the
interior trace; reflect copies it with the normal momentum negated.
"""

import numpy as np


# ----------------------------------------------------------------------------
# physical fluxes and spectral radii (Sec. 5.1-5.4)
# ----------------------------------------------------------------------------

def euler_pressure(U, gamma, dim):
    rho = U[0]
    if dim == 1:
        kin = 0.5 * U[1] * U[1] / rho
        return (gamma - 1.0) * (U[2] - kin)
    kin = 0.5 * (U[1] * U[1] + U[2] * U[2]) / rho
    return (gamma - 1.0) * (U[3] - kin)


def flux_x(prob, U):
    eq = prob.equation
    if eq == "advection":
        return prob.adv_speed * U
    if eq == "burgers":
        return 0.5 * U * U
    if eq == "euler1d":
        rho, m, E = U[0], U[1], U[2]
        v = m / rho
        p = euler_pressure(U, prob.gamma, 1)
        return np.stack([m, m * v + p, (E + p) * v])
    rho, mx, my, E = U[0], U[1], U[2], U[3]
    vx = mx / rho
    p = euler_pressure(U, prob.gamma, 2)
    return np.stack([mx, mx * vx + p, my * vx, (E + p) * vx])


def flux_y(prob, U):
    rho, mx, my, E = U[0], U[1], U[2], U[3]
    vy = my / rho
    p = euler_pressure(U, prob.gamma, 2)
    return np.stack([my, mx * vy, my * vy + p, (E + p) * vy])


def speed_x(prob, U):
    """Spectral radius of df/du along x at each node."""
    eq = prob.equation
    if eq == "advection":
        return np.full(U.shape[1:], abs(prob.adv_speed))
    if eq == "burgers":
        return np.abs(U[0])
    dim = 1 if eq == "euler1d" else 2
    p = euler_pressure(U, prob.gamma, dim)
    c = np.sqrt(prob.gamma * p / U[0])
    return np.abs(U[1] / U[0]) + c


def speed_y(prob, U):
    p = euler_pressure(U, prob.gamma, 2)
    c = np.sqrt(prob.gamma * p / U[0])
    return np.abs(U[2] / U[0]) + c


def rusanov(prob, UL, UR, direction):
    """Lax-Friedrichs interactive flux per node (Sec. 3.3)."""
    if direction == 0:
        fL, fR = flux_x(prob, UL), flux_x(prob, UR)
        lam = np.maximum(speed_x(prob, UL), speed_x(prob, UR))
    else:
        fL, fR = flux_y(prob, UL), flux_y(prob, UR)
        lam = np.maximum(speed_y(prob, UL), speed_y(prob, UR))
    return 0.5 * (fL + fR) - 0.5 * lam[None] * (UR - UL)


def hll(prob, UL, UR, direction):
    """HLL interactive flux per node for the Euler equations (named in Tables 5 and 6;
    the paper gives no formula).  Two waves bound the Riemann fan, with Davis's
    estimates S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R)
    (u the velocity normal to the face, c the sound speed); between them one
    constant state conserves the fan, which gives
      F = f_L                                   if S_L >= 0,
      F = f_R                                   if S_R <= 0,
      F = (S_R f_L - S_L f_R + S_L S_R (U_R - U_L)) / (S_R - S_L) otherwise."""
    if not prob.equation.startswith("euler"):
        raise ValueError("the HLL flux is provided for the Euler equations")
    dim = 1 if prob.equation == "euler1d" else 2
    flux = flux_x if direction == 0 else flux_y
    fL, fR = flux(prob, UL), flux(prob, UR)
    uL = UL[1 + direction] / UL[0]
    uR = UR[1 + direction] / UR[0]
    cL = np.sqrt(prob.gamma * euler_pressure(UL, prob.gamma, dim) / UL[0])
    cR = np.sqrt(prob.gamma * euler_pressure(UR, prob.gamma, dim) / UR[0])
    SL = np.minimum(uL - cL, uR - cR)
    SR = np.maximum(uL + cL, uR + cR)
    with np.errstate(divide="ignore", invalid="ignore"):
        mid = (SR[None] * fL - SL[None] * fR + (SL * SR)[None] * (UR - UL)) / (SR - SL)[None]
    return np.where((SL >= 0.0)[None], fL, np.where((SR <= 0.0)[None], fR, mid))


def interactive_flux(prob, UL, UR, direction):
    """The configured interactive flux (Sec. 3.3): Lax-Friedrichs, or HLL for Euler."""
    if prob.flux == "hll":
        return hll(prob, UL, UR, direction)
    return rusanov(prob, UL, UR, direction)


# ----------------------------------------------------------------------------
# boundary ghosts and face pairing
# ----------------------------------------------------------------------------

def ghost(prob, side, trace):
    """Ghost trace outside boundary `side` (0: x-lo, 1: x-hi, 2: y-lo, 3: y-hi)."""
    kind = prob.bc[side]
    if kind == "outflow":
        return trace.copy()
    if kind == "dirichlet":
        st = np.asarray(prob.bc_state[side][: prob.S], dtype=np.float64)
        return np.broadcast_to(st.reshape((prob.S,) + (1,) * (trace.ndim - 1)), trace.shape).copy()
    if kind == "reflect":
        g = trace.copy()
        normal = 1 if side < 2 else 2
        g[normal] = -g[normal]
        return g
    raise ValueError("unknown boundary kind " + kind)


def face_pairs(prob, Tminus, Tplus, axis, sides):
    """Left/right states at the n+1 faces along element axis `axis`.

    Tminus/Tplus: each element's trace at its r=-1 / r=+1 face.
    Face i sits between element i-1 (its + trace) and element i (its - trace).
    """
    n = Tminus.shape[axis]
    take = lambda a, i: np.take(a, [i], axis=axis)
    if prob.bc[sides[0]] == "periodic":
        left = np.concatenate([take(Tplus, n - 1), Tplus], axis=axis)
        right = np.concatenate([Tminus, take(Tminus, 0)], axis=axis)
    else:
        left = np.concatenate([ghost(prob, sides[0], take(Tminus, 0)), Tplus], axis=axis)
        right = np.concatenate([Tminus, ghost(prob, sides[1], take(Tplus, n - 1))], axis=axis)
    return left, right


# ----------------------------------------------------------------------------
# right-hand side
# ----------------------------------------------------------------------------

def rhs(prob, T, R, u):
    if prob.element == "tri":
        from .tri import rhs_tri
        return rhs_tri(prob, T, R, u)
    if prob.dim == 1:
        return _rhs_1d(prob, T, R, u)
    return _rhs_2d(prob, T, R, u)


def _rhs_1d(prob, T, R, u):
    S, M, E, N = u.shape
    J = prob.dx / 2.0
    # 1. gPC expansion at the random nodes, every solution point
    U = np.einsum("kq,skej->sqej", R.Phi, u)
    # 2. physical flux at (solution point, node), projected onto the chaos
    fh = np.einsum("kq,sqej->skej", R.PW, flux_x(prob, U))
    # 3. solution traces at the faces, interactive flux per node, projected
    Um = np.einsum("j,sqej->sqe", T.lL, U)
    Up = np.einsum("j,sqej->sqe", T.lR, U)
    left, right = face_pairs(prob, Um, Up, axis=2, sides=(0, 1))
    Fstar = np.einsum("kq,sqf->skf", R.PW, interactive_flux(prob, left, right, 0))
    # 4. discontinuous flux polynomial at the faces
    fDL = np.einsum("j,skej->ske", T.lL, fh)
    fDR = np.einsum("j,skej->ske", T.lR, fh)
    # 5. total-flux derivative at the solution points
    dfdr = np.einsum("jl,skel->skej", T.D, fh)
    dfdr = dfdr + (Fstar[:, :, :E] - fDL)[..., None] * T.dhL + (Fstar[:, :, 1:] - fDR)[..., None] * T.dhR
    # 6. du/dt = -(1/J) df/dr
    return -dfdr / J


def _rhs_2d(prob, T, R, u):
    S, M, E, Nsp = u.shape
    n = T.n
    nx, ny = prob.nx, prob.ny
    Jx, Jy = prob.dx / 2.0, prob.dy / 2.0
    u6 = u.reshape(S, M, ny, nx, n, n)  # [s, k, iy, ix, b, a]
    U = np.einsum("kq,skyxba->sqyxba", R.Phi, u6)
    fh = np.einsum("kq,sqyxba->skyxba", R.PW, flux_x(prob, U))
    gh = np.einsum("kq,sqyxba->skyxba", R.PW, flux_y(prob, U))

    # x-direction: lines along a, faces between ix-1 and ix at flux points b
    Um = np.einsum("a,sqyxba->sqyxb", T.lL, U)
    Up = np.einsum("a,sqyxba->sqyxb", T.lR, U)
    left, right = face_pairs(prob, Um, Up, axis=3, sides=(0, 1))
    Fx = np.einsum("kq,sqyfb->skyfb", R.PW, interactive_flux(prob, left, right, 0))
    fDL = np.einsum("a,skyxba->skyxb", T.lL, fh)
    fDR = np.einsum("a,skyxba->skyxb", T.lR, fh)
    dx_part = np.einsum("ac,skyxbc->skyxba", T.D, fh)
    dx_part = (dx_part
               + (Fx[:, :, :, :nx, :] - fDL)[..., None] * T.dhL
               + (Fx[:, :, :, 1:, :] - fDR)[..., None] * T.dhR)

    # y-direction: lines along b, faces between iy-1 and iy at flux points a
    Vm = np.einsum("b,sqyxba->sqyxa", T.lL, U)
    Vp = np.einsum("b,sqyxba->sqyxa", T.lR, U)
    left, right = face_pairs(prob, Vm, Vp, axis=2, sides=(2, 3))
    Gy = np.einsum("kq,sqfxa->skfxa", R.PW, interactive_flux(prob, left, right, 1))
    gDL = np.einsum("b,skyxba->skyxa", T.lL, gh)
    gDR = np.einsum("b,skyxba->skyxa", T.lR, gh)
    dy_part = np.einsum("bc,skyxca->skyxba", T.D, gh)
    dy_part = (dy_part
               + (Gy[:, :, :ny] - gDL)[:, :, :, :, None, :] * T.dhL[:, None]
               + (Gy[:, :, 1:] - gDR)[:, :, :, :, None, :] * T.dhR[:, None])

    out = -dx_part / Jx - dy_part / Jy
    return out.reshape(S, M, E, Nsp)


# ----------------------------------------------------------------------------
# nodal values used by the limiter and the time-step restriction
# ----------------------------------------------------------------------------

def nodal_at_solution_points(R, u):
    """U[s, q, e, j] = sum_k u[s, k, e, j] Phi_k(z_q)."""
    return np.einsum("kq,skej->sqej", R.Phi, u)


def nodal_at_face_points(prob, T, U):
    """Per element, solution traces at the face (flux) points, U[s, q, e, f].

    1D: the two faces r = -1, +1.  2D: for each of the 4 faces the (p+1) flux
    points on it, ordered x-lo (b), x-hi (b), y-lo (a), y-hi (a).
    """
    if prob.element == "tri":
        # the 3 (p+1) flux points, face-major
        return np.einsum("fki,sqei->sqefk", T.Lf, U).reshape(U.shape[:3] + (-1,))
    if prob.dim == 1:
        return np.stack([np.einsum("j,sqej->sqe", T.lL, U), np.einsum("j,sqej->sqe", T.lR, U)], axis=-1)
    S, Nq, E, _ = U.shape
    n = T.n
    U5 = U.reshape(S, Nq, E, n, n)  # [.., b, a]
    xlo = np.einsum("a,sqeba->sqeb", T.lL, U5)
    xhi = np.einsum("a,sqeba->sqeb", T.lR, U5)
    ylo = np.einsum("b,sqeba->sqea", T.lL, U5)
    yhi = np.einsum("b,sqeba->sqea", T.lR, U5)
    return np.concatenate([xlo, xhi, ylo, yhi], axis=-1)

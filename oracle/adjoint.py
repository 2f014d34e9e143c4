"""Discrete adjoint of the FR-SG step for the scalar 1D equations, and the
mean-square objective.  Test infrastructure: plain FP64 NumPy, slow, written
for checking by eye; nothing here is used by the library.

The paper has no adjoint.  The object here is the exact transpose of the
discrete map the forward oracle computes, at frozen switch decisions (the
detector flags of the step) and frozen dt:

    lam_n = (d u_{n+1} / d u_n)^T lam_{n+1}.

Every function below runs the operations of its forward counterpart
(oracle.fr._rhs_1d, oracle.stabilize.sensor_filter, oracle.stepper.ssprk3) in
reverse order, each replaced by its transpose (reverse-mode differentiation
written out by hand).  The Lax-Friedrichs dissipation speed max(|f'(L)|,
|f'(R)|) is differentiated through the side that attains the maximum (the
left one on a tie); it is exact wherever the two speeds differ.

Objective (mean square over space and random space; with orthonormal bases it
is the sum of the integrals of E[u]^2 and Var[u]):

    J(u) = sum_e J_e sum_j w_j sum_k u[0, k, e, j]^2,   J_e = dx / 2,

whose gradient is 2 J_e w_j u.

Parameters: the derivative with respect to the advection speed a is returned
alongside (zero for Burgers).  dt is frozen, so the CFL dependence of dt on a
is not part of it.
"""

import numpy as np

from .fr import face_pairs, rhs
from .stabilize import filter_strength


def _check(prob):
    if prob.dim != 1 or prob.equation not in ("advection", "burgers"):
        raise ValueError("the adjoint covers the scalar 1D equations (advection, Burgers)")
    if prob.limiter:
        raise ValueError("the adjoint has no limiter (the scalar equations do not use it)")
    if prob.flux != "rusanov":
        raise ValueError("the adjoint covers the Lax-Friedrichs flux")
    if prob.filter == "lasso":
        raise ValueError("the adjoint covers the linear filters (exponential, L2), not the Lasso filter")


# ----------------------------------------------------------------------------
# transposes of the pointwise pieces
# ----------------------------------------------------------------------------

def flux_vjp(prob, U, g):
    """g * f'(U) for the scalar flux; and d/da of <g, f(U)>."""
    if prob.equation == "advection":
        return prob.adv_speed * g, float(np.sum(g * U))
    return U * g, 0.0


def rusanov_vjp(prob, L, R, g):
    """Transpose of F = (f(L) + f(R))/2 - lam (R - L)/2, lam = max(|f'(L)|, |f'(R)|).

    Returns (gL, gR, d/da of <g, F>)."""
    if prob.equation == "advection":
        a = prob.adv_speed
        gL = 0.5 * a * g + 0.5 * abs(a) * g
        gR = 0.5 * a * g - 0.5 * abs(a) * g
        da = float(np.sum(g * (0.5 * (L + R) - 0.5 * np.sign(a) * (R - L))))
        return gL, gR, da
    sL, sR = np.abs(L), np.abs(R)
    lam = np.maximum(sL, sR)
    left_wins = sL >= sR
    jump = R - L
    gL = 0.5 * L * g + 0.5 * lam * g
    gR = 0.5 * R * g - 0.5 * lam * g
    dlam = -0.5 * jump * g  # adjoint of lam
    gL = gL + np.where(left_wins, np.sign(L) * dlam, 0.0)
    gR = gR + np.where(left_wins, 0.0, np.sign(R) * dlam)
    return gL, gR, 0.0


def ghost_vjp(prob, side, g):
    """Transpose of the ghost trace of a boundary side, applied to its adjoint."""
    kind = prob.bc[side]
    if kind == "outflow":
        return g.copy()
    if kind == "dirichlet":
        return np.zeros_like(g)
    raise ValueError("boundary kind without a scalar adjoint: " + kind)


def face_pairs_vjp(prob, g_left, g_right, E):
    """Transpose of oracle.fr.face_pairs along the element axis (last axis here)."""
    g_m = np.zeros(g_left.shape[:-1] + (E,))
    g_p = np.zeros_like(g_m)
    g_p += g_left[..., 1:]
    g_m += g_right[..., :E]
    if prob.bc[0] == "periodic":
        g_p[..., E - 1] += g_left[..., 0]
        g_m[..., 0] += g_right[..., E]
    else:
        g_m[..., 0] += ghost_vjp(prob, 0, g_left[..., 0])
        g_p[..., E - 1] += ghost_vjp(prob, 1, g_right[..., E])
    return g_m, g_p


# ----------------------------------------------------------------------------
# right-hand side
# ----------------------------------------------------------------------------

def rhs_vjp(prob, T, R, u, g):
    """(dR/du)^T g and d<g, R(u)>/da, by reversing the steps of the 1D right-hand side."""
    _check(prob)
    S, M, E, N = u.shape
    J = prob.dx / 2.0
    # forward quantities the transposes need
    U = np.einsum("kq,skej->sqej", R.Phi, u)
    Um = np.einsum("j,sqej->sqe", T.lL, U)
    Up = np.einsum("j,sqej->sqe", T.lR, U)
    left, right = face_pairs(prob, Um, Up, axis=2, sides=(0, 1))

    # 6. out = -dfdr / J
    g_dfdr = -g / J
    # 5. dfdr = D fh + (Fstar_L - fDL) h_L' + (Fstar_R - fDR) h_R'
    g_fh = np.einsum("jl,skej->skel", T.D, g_dfdr)
    gcL = np.einsum("skej,j->ske", g_dfdr, T.dhL)
    gcR = np.einsum("skej,j->ske", g_dfdr, T.dhR)
    g_Fstar = np.zeros((S, M, E + 1))
    g_Fstar[:, :, :E] += gcL
    g_Fstar[:, :, 1:] += gcR
    # 4. fDL = l(-1) . fh, fDR = l(+1) . fh (entering with a minus sign)
    g_fh -= gcL[..., None] * T.lL
    g_fh -= gcR[..., None] * T.lR
    # 3. Fstar = PW Fq, Fq = rusanov(left, right), left/right from the traces
    g_Fq = np.einsum("kq,skf->sqf", R.PW, g_Fstar)
    g_left, g_right, da_face = rusanov_vjp(prob, left, right, g_Fq)
    g_Um, g_Up = face_pairs_vjp(prob, g_left, g_right, E)
    # 2. fh = PW f(U)
    g_fU = np.einsum("kq,skej->sqej", R.PW, g_fh)
    g_U, da_flux = flux_vjp(prob, U, g_fU)
    # traces Um = l(-1) . U, Up = l(+1) . U
    g_U = g_U + np.einsum("j,sqe->sqej", T.lL, g_Um) + np.einsum("j,sqe->sqej", T.lR, g_Up)
    # 1. U = Phi^T u
    g_u = np.einsum("kq,sqej->skej", R.Phi, g_U)
    return g_u, da_flux + da_face


# ----------------------------------------------------------------------------
# filter and step
# ----------------------------------------------------------------------------

def filter_vjp(prob, T, R, g, flags, dt):
    """Transpose of the filter V diag(Lambda) V^-1 on the flagged elements (identity elsewhere)."""
    if prob.filter == "none":
        return g.copy()
    lam = filter_strength(prob, T, R, dt)
    gt = np.einsum("jl,skej->skel", T.V, g)          # V^T g
    gt = gt * lam[None, :, None, :]
    gf = np.einsum("ml,skem->skel", T.Vinv, gt)       # V^-T (Lambda V^T g)
    out = g.copy()
    fl = np.asarray(flags, dtype=bool)
    out[:, :, fl, :] = gf[:, :, fl, :]
    return out


def step_vjp(prob, T, R, u, dt, flags, lam):
    """Adjoint of one SSP-RK3 step at the step's filter flags (flags[2]) and dt.

    Returns (lam_n, d<lam, u_{n+1}>/da)."""
    _check(prob)
    Rf = lambda w: rhs(prob, T, R, w)
    # stage states of the forward step (no limiter for the scalar equations)
    w1 = u + dt * Rf(u)
    w2 = 0.75 * u + 0.25 * (w1 + dt * Rf(w1))
    # u+ = Filter(v)
    vb = filter_vjp(prob, T, R, lam, flags[2], dt)
    # v = u/3 + 2/3 (w2 + dt R(w2))
    g, da = rhs_vjp(prob, T, R, w2, vb)
    b2 = (2.0 / 3.0) * (vb + dt * g)
    ga = (2.0 / 3.0) * dt * da
    # w2 = 3/4 u + 1/4 (w1 + dt R(w1))
    g, da = rhs_vjp(prob, T, R, w1, b2)
    b1 = 0.25 * (b2 + dt * g)
    ga += 0.25 * dt * da
    # w1 = u + dt R(u)
    g, da = rhs_vjp(prob, T, R, u, b1)
    out = (1.0 / 3.0) * vb + 0.75 * b2 + b1 + dt * g
    ga += dt * da
    return out, ga


# ----------------------------------------------------------------------------
# objective
# ----------------------------------------------------------------------------

def objective(prob, T, u):
    """J = sum_e J_e sum_j w_j sum_k u_k^2 (first state)."""
    Je = prob.dx / 2.0
    return float(Je * np.einsum("kej,j->", u[0] ** 2, T.w))


def objective_grad(prob, T, u):
    """dJ/du = 2 J_e w_j u (zero on the other states)."""
    g = np.zeros_like(u)
    g[0] = 2.0 * (prob.dx / 2.0) * u[0] * T.w
    return g

"""Discontinuity sensor, modal filters and positivity-preserving limiter (Sec. 4).

Modal form (Sec. 4, Eq. modal solution): inside an element the solution is
sum_j sum_k u~_{j,k} Psi_j Phi_k with Psi orthonormal under dr/2 and Phi the
gPC basis; the spatial modal coefficients follow from the nodal ones with the
inverse Vandermonde matrix (tensor product in 2D).  With both bases
orthonormal, the inner product over element x random space is the sum of
squared coefficients.

Sensor (Sec. 4.2, Eq. detector): S_e = <u^N - u^{N-1}, same> / <u^N, u^N> on
the first state, where u^N - u^{N-1} is the outermost shell of the expansion:
spatial degree p in some direction, or total chaos degree N_c.  An element is
flagged when theta < 0.99, i.e. S_e > S* = 10^(s0 - (2 kappa/pi) asin 0.98);
a zero denominator is not flagged.

Filters (Sec. 4.1): u~* = Lambda o u~ and back to nodal with V.
* exponential (Sec. 4.1.1): lambda = exp(-alpha dt sum_i t_i) with
  eta = j/p per spatial direction (the total degree over p on triangles) and
  |k|/N_c in random space; per dimension t = 0 below the cutoff
  eta* = N*/p (N*/N_c in random space), t = ((eta - eta*)/(1 - eta*))^s from it
  on, so the product of the per-dimension factors is 1 where every eta is below
  its cutoff; N* = 0 (App. A) gives t = eta^s;
* L2 (Sec. 4.1.2, Eq. filter function, Eq. l2 strength):
  lambda = 1 / (1 + alpha1 sum_d j_d^2 (j_d+1)^2 + alpha2 |k|^2 (|k|+1)^2),
  alpha1 = 1/(eps1 N_p^2 (N_p-1)^2), alpha2 = 1/(eps2 N_c^2 (N_c+1)^2);
* Lasso (Sec. 4.1.3, Eq. LassoFilterFunction, Eq. fStrength), one physical and
  one random dimension: per element and conserved variable,
    u~*_{j,k} = ReLU(1 - (a1 j(j+1) + a2 k(k+1)) ||Psi_j Phi_k||_1 / |u~_{j,k}|) u~_{j,k},
    a1 = |u~_{N_p-1,0}| / (N_p (N_p-1) ||Psi_{N_p-1} Phi_0||_1),
    a2 = |u~_{0,N_c}| / (N_c (N_c+1) ||Psi_0 Phi_{N_c}||_1),
  with ||Psi_j Phi_k||_1 = ||Psi_j||_1 ||Phi_k||_1 (both under their
  probability measures); a zero coefficient stays zero.

Limiter (Sec. 4.3): per element, mean state u_bar over element x random space,
eps = min(1e-8, rho_bar, p_bar); if the minimum of density or pressure over
(solution and flux points) x (random nodes) is below eps, density slopes are
scaled by beta1 = min((rho_bar - eps)/(rho_bar - rho_min), 1), then every
point whose pressure is still below eps gets the root beta_l of
p(beta (u* - u_bar) + u_bar) = eps, and all states are scaled by
beta2 = min_l beta_l.  Because the map u -> beta (u - u_bar) + u_bar is
affine, it is applied to the gPC coefficients directly (only the k = 0 mode
carries the mean).
"""

import numpy as np

from .fr import euler_pressure, nodal_at_face_points, nodal_at_solution_points
from .tables import legendre_l1_norms, sensor_threshold


class NotRealizable(ArithmeticError):
    pass


# ----------------------------------------------------------------------------
# spatial modal transforms
# ----------------------------------------------------------------------------

def to_spatial_modal(prob, T, u):
    if prob.element == "tri":
        return np.einsum("ml,skel->skem", T.Vinv, u)
    if prob.dim == 1:
        return np.einsum("jl,skel->skej", T.Vinv, u)
    S, M, E, _ = u.shape
    n = T.n
    u5 = u.reshape(S, M, E, n, n)  # [.., b, a]
    m = np.einsum("ac,bd,skedc->skeba", T.Vinv, T.Vinv, u5)
    return m.reshape(S, M, E, n * n)


def to_nodal(prob, T, ut):
    if prob.element == "tri":
        return np.einsum("jm,skem->skej", T.V, ut)
    if prob.dim == 1:
        return np.einsum("jl,skel->skej", T.V, ut)
    S, M, E, _ = ut.shape
    n = T.n
    u5 = ut.reshape(S, M, E, n, n)
    m = np.einsum("ac,bd,skedc->skeba", T.V, T.V, u5)
    return m.reshape(S, M, E, n * n)


def spatial_degrees(prob, T):
    """Per solution-point mode index: tuple of per-direction degrees (on triangles
    the total degree of the orthonormal mode, a one-element tuple)."""
    if prob.element == "tri":
        return [(int(d),) for d in T.deg]
    n = T.n
    if prob.dim == 1:
        return [(j,) for j in range(n)]
    return [(j % n, j // n) for j in range(n * n)]


# ----------------------------------------------------------------------------
# sensor and filter
# ----------------------------------------------------------------------------

def sensor_flags(prob, T, R, u):
    """Boolean flag per element (Eq. detector)."""
    E = u.shape[2]
    if prob.sensor == "always":
        return np.ones(E, dtype=bool)
    ut = to_spatial_modal(prob, T, u)[0]  # first state: [k, e, j]
    degs = spatial_degrees(prob, T)
    shell = np.zeros((R.M, len(degs)), dtype=bool)
    for k in range(R.M):
        for j, d in enumerate(degs):
            shell[k, j] = (max(d) == prob.p) or (R.kdeg[k] == prob.gpc_order)
    e2 = ut * ut
    num = np.einsum("kej,kj->e", e2, shell.astype(np.float64))
    den = np.einsum("kej->e", e2)
    thr = sensor_threshold(prob.s0, prob.kappa)
    flags = np.zeros(E, dtype=bool)
    nz = den > 0.0
    flags[nz] = (num[nz] / den[nz]) > thr
    return flags


def filter_strength(prob, T, R, dt):
    """Lambda[k, j]: filter factor per (gPC mode, spatial mode)."""
    degs = spatial_degrees(prob, T)
    lam = np.ones((R.M, len(degs)))
    Nc = prob.gpc_order
    if prob.filter == "exp":
        def term(eta, eta_star):
            # modes below the cutoff are left untouched (Sec. 4.1.1)
            return 0.0 if eta < eta_star else ((eta - eta_star) / (1.0 - eta_star)) ** prob.s

        for k in range(R.M):
            ez = term(R.kdeg[k] / Nc, prob.nstar / Nc) if Nc > 0 else 0.0
            for j, d in enumerate(degs):
                ex = sum(term(dj / prob.p, prob.nstar / prob.p) for dj in d)
                lam[k, j] = np.exp(-prob.alpha * dt * (ex + ez))
    elif prob.filter == "l2":
        # N_p solution points per direction: the damping of the top degree p is 1/(1 + 1/eps1)
        Np = prob.p + 1
        a1 = 1.0 / (prob.eps1 * Np * Np * (Np - 1) * (Np - 1))
        a2 = 1.0 / (prob.eps2 * Nc * Nc * (Nc + 1) * (Nc + 1)) if Nc > 0 else 0.0
        for k in range(R.M):
            kk = R.kdeg[k]
            for j, d in enumerate(degs):
                pen = a1 * sum(dj * dj * (dj + 1) * (dj + 1) for dj in d) + a2 * kk * kk * (kk + 1) * (kk + 1)
                lam[k, j] = 1.0 / (1.0 + pen)
    return lam


def lasso_norms(prob, T, R):
    """||Psi_j Phi_k||_1, indexed [k, j] (one physical, one random dimension)."""
    check_lasso(prob)
    lx = legendre_l1_norms(T.n)
    lz = legendre_l1_norms(R.M)
    return np.outer(lz, lx)


def check_lasso(prob):
    if prob.dim != 1 or prob.rdim != 1:
        raise ValueError("the Lasso filter is defined here for one physical and one random dimension")


def lasso_modal(prob, T, R, ut):
    """Eq. LassoFilterFunction with the strengths of Eq. fStrength, on spatial-
    modal coefficients ut[s, k, e, j] (k = chaos degree); returns the filtered ones."""
    nrm = lasso_norms(prob, T, R)
    Np, Nc = T.n, R.M - 1
    j = np.arange(Np, dtype=np.float64)
    k = np.arange(R.M, dtype=np.float64)
    au = np.abs(ut)
    a1 = au[:, 0, :, Np - 1] / (float(Np * (Np - 1)) * nrm[0, Np - 1])   # [s, e]
    a2 = au[:, Nc, :, 0] / (float(Nc * (Nc + 1)) * nrm[Nc, 0]) if Nc > 0 else np.zeros_like(a1)
    pen = (a1[:, None, :, None] * (j * (j + 1.0))[None, None, None, :]
           + a2[:, None, :, None] * (k * (k + 1.0))[None, :, None, None]) * nrm[None, :, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(au > 0.0, 1.0 - pen / au, 0.0)
    return np.maximum(f, 0.0) * ut


def sensor_filter(prob, T, R, u, dt):
    """Sensor-gated filter; returns (u_filtered, flags)."""
    if prob.filter == "none":
        return u.copy(), np.zeros(u.shape[2], dtype=bool)
    flags = sensor_flags(prob, T, R, u)
    ut = to_spatial_modal(prob, T, u)
    if prob.filter == "lasso":
        uf = to_nodal(prob, T, lasso_modal(prob, T, R, ut))
    else:
        lam = filter_strength(prob, T, R, dt)
        uf = to_nodal(prob, T, ut * lam[None, :, None, :])
    out = u.copy()
    out[:, :, flags, :] = uf[:, :, flags, :]
    return out, flags


# ----------------------------------------------------------------------------
# positivity-preserving limiter
# ----------------------------------------------------------------------------

def element_mean(prob, T, u):
    """Mean over element x random space: sum_j (w_j/2) u[s, 0, e, j] (tensor in 2D; on
    triangles the coefficient of the constant orthonormal mode)."""
    if prob.element == "tri":
        return np.einsum("sej,j->se", u[:, 0], T.mean_w)
    if prob.dim == 1:
        wts = T.w / 2.0
    else:
        wts = np.outer(T.w / 2.0, T.w / 2.0).ravel()  # index b*n + a
    return np.einsum("sej,j->se", u[:, 0], wts)


def pressure_root(prob, ubar, ustar, eps):
    """Root in (0, 1) of p(beta (u* - u_bar) + u_bar) = eps.

    With d = u* - u_bar and e' = eps/(gamma-1), rho (E - e') - |m|^2/2 = 0 is
    the quadratic a beta^2 + b beta + c with
      a = dE drho - |dm|^2/2,  b = dE rho_bar + (E_bar - e') drho - m_bar.dm,
      c = (E_bar - e') rho_bar - |m_bar|^2/2 > 0;
    its root in (0, 1) is taken in the cancellation-free form.
    """
    g = prob.gamma
    ep = eps / (g - 1.0)
    d = ustar - ubar
    rb, Eb = ubar[0], ubar[-1]
    mb = ubar[1:-1]
    dr, dE = d[0], d[-1]
    dm = d[1:-1]
    a = dE * dr - 0.5 * np.sum(dm * dm, axis=0)
    b = dE * rb + (Eb - ep) * dr - np.sum(mb * dm, axis=0)
    c = (Eb - ep) * rb - 0.5 * np.sum(mb * mb, axis=0)
    disc = np.maximum(b * b - 4.0 * a * c, 0.0)
    sq = np.sqrt(disc)
    with np.errstate(divide="ignore", invalid="ignore"):
        beta = np.where(b < 0.0, 2.0 * c / (-b + sq), (-b - sq) / (2.0 * a))
    return beta


def limiter_margin(prob, T, R, u):
    """Per element: min(rho_min, p_min) - eps and the magnitude of the state.

    Diagnostic for comparing switch decisions made in different arithmetic
    orders: a decision whose margin is at the rounding level of the state
    (about 1e-16 times its magnitude) is a tie.
    """
    E = u.shape[2]
    dim = prob.dim
    ubar = element_mean(prob, T, u)
    pbar = euler_pressure(ubar, prob.gamma, dim)
    Usp = nodal_at_solution_points(R, u)
    Ufp = nodal_at_face_points(prob, T, Usp)
    pts = np.concatenate([Usp.transpose(0, 2, 1, 3).reshape(prob.S, E, -1),
                          Ufp.transpose(0, 2, 1, 3).reshape(prob.S, E, -1)], axis=2)
    eps = np.minimum(1e-8, np.minimum(ubar[0], pbar))
    m = np.minimum(pts[0].min(axis=1), euler_pressure(pts, prob.gamma, dim).min(axis=1)) - eps
    scale = np.abs(pts).max(axis=(0, 2))
    return m, scale


def sensor_margin(prob, T, R, u):
    """Per element: (S_e, S*) of the detector (diagnostic, see limiter_margin)."""
    ut = to_spatial_modal(prob, T, u)[0]
    degs = spatial_degrees(prob, T)
    shell = np.array([[(max(d) == prob.p) or (R.kdeg[k] == prob.gpc_order) for d in degs] for k in range(R.M)])
    e2 = ut * ut
    num = np.einsum("kej,kj->e", e2, shell.astype(np.float64))
    den = np.einsum("kej->e", e2)
    with np.errstate(divide="ignore", invalid="ignore"):
        se = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return se, sensor_threshold(prob.s0, prob.kappa)


def limit(prob, T, R, u):
    """Positivity-preserving limiter; returns (u_limited, flags)."""
    E = u.shape[2]
    flags = np.zeros(E, dtype=bool)
    if not prob.limiter:
        return u.copy(), flags
    dim = prob.dim
    out = u.copy()
    ubar = element_mean(prob, T, u)  # [s, e]
    pbar = euler_pressure(ubar, prob.gamma, dim)
    if np.any(ubar[0] <= 0.0) or np.any(pbar <= 0.0) or not np.all(np.isfinite(ubar)):
        raise NotRealizable("element mean density or pressure not positive")
    Usp = nodal_at_solution_points(R, u)                  # [s, q, e, j]
    Ufp = nodal_at_face_points(prob, T, Usp)              # [s, q, e, f]
    # density and pressure at (solution + flux points) x nodes, per element
    pts_all = np.concatenate([Usp.transpose(0, 2, 1, 3).reshape(prob.S, E, -1),
                              Ufp.transpose(0, 2, 1, 3).reshape(prob.S, E, -1)], axis=2)
    rho_min = pts_all[0].min(axis=1)
    p_min = euler_pressure(pts_all, prob.gamma, dim).min(axis=1)
    eps_all = np.minimum(1e-8, np.minimum(ubar[0], pbar))
    mode0 = (np.arange(R.M) == 0)[:, None]
    for e in np.nonzero(np.minimum(rho_min, p_min) < eps_all)[0]:
        flags[e] = True
        pts = pts_all[:, e, :]
        rb = ubar[0, e]
        eps = eps_all[e]
        beta1 = 1.0 if rho_min[e] >= eps else (rb - eps) / (rb - rho_min[e])
        star = pts.copy()
        star[0] = beta1 * (pts[0] - rb) + rb
        out[0, :, e, :] = beta1 * (out[0, :, e, :] - rb * mode0) + rb * mode0
        pstar = euler_pressure(star, prob.gamma, dim)
        low = pstar < eps
        beta2 = 1.0
        if np.any(low):
            roots = pressure_root(prob, ubar[:, e][:, None], star[:, low], eps)
            beta2 = float(np.min(roots))
        for s in range(prob.S):
            out[s, :, e, :] = beta2 * (out[s, :, e, :] - ubar[s, e] * mode0) + ubar[s, e] * mode0
    return out, flags

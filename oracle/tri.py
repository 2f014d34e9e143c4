"""Triangular elements for the 2D Euler equations: the FR-SG right-hand side on
straight-sided triangles (Sec. 3.1 reference map of the isosceles right
triangle, Sec. 3.5 multi-dimensional extension).  Test infrastructure: the
plain reference that the HIP path is checked against; nothing here is used by
the library.

Reference triangle T with vertices (-1, -1), (1, -1), (-1, 1), mapped to an
element by x = lam1 x1 + lam2 x2 + lam3 x3, lam1 = -(r+s)/2, lam2 = (r+1)/2,
lam3 = (s+1)/2 (Sec. 3.1).  Face f joins vertices f and f+1 (mod 3); its p+1
flux points are Gauss-Legendre points in the edge parameter t in [-1, 1] from
the first vertex to the second.

Readings (the paper gives the constraint on the correction fields of Sec. 3.5
but no choice of fields or points for triangles):

* solution points: the warp-and-blend nodes (Warburton's construction, without
  the optimisation parameter); for p <= 2 they are the equispaced lattice;
* correction fields: the choice that makes FR equal to nodal DG, the analogue
  of the Radau choice in one dimension.  Its divergence at the solution points
  is the DG lifting of the face's Lagrange function: the polynomial phi of
  degree p with int_T phi v = int_face l_k v ds for every v of degree p;
* the discontinuous flux at a flux point is the interpolant of the projected
  flux, as on quadrilaterals; the interactive flux is evaluated per random node
  along the unit outward normal;
* time step: dt = CFL d_min / ((p+1) lambda_max) with d_e the diameter of the
  element's inscribed circle (4 area / perimeter) and lambda = |v| + c, taken
  as the maximum of lambda / d_e over solution points, nodes and elements.

For affine elements the reference-space form of Sec. 3.5 and the physical one
coincide: the contravariant flux is det * (metric) * F, the reference normal
flux is (F . n) times the ratio of physical to reference face length, and both
sides are divided by det = area / 2.

State layout as on quadrilaterals: u[s, k, e, j] with j the solution point.
"""

import math
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

from .fr import euler_pressure
from .tables import gauss_legendre, lagrange_values, legendre_values

REF_FACE_LEN = (2.0, 2.0 * math.sqrt(2.0), 2.0)


# ----------------------------------------------------------------------------
# quadrature, basis, points
# ----------------------------------------------------------------------------

def duffy_rule(n):
    """Quadrature on T from n x n Gauss points through the collapsed coordinates
    r = (1 + a)(1 - b)/2 - 1, s = b (Jacobian (1 - b)/2).  Weights sum to 2."""
    x, w = gauss_legendre(n)
    a, b = np.meshgrid(x, x, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    r = (1.0 + a) * (1.0 - b) / 2.0 - 1.0
    return r.ravel(), b.ravel(), (wa * wb * (1.0 - b) / 2.0).ravel()


def monomial_exponents(p):
    """(i, j) for r^i s^j of total degree <= p, graded: degree d, then j = 0..d."""
    return [(d - j, j) for d in range(p + 1) for j in range(d + 1)]


@lru_cache(maxsize=None)
def orthonormal_basis(p):
    """Coefficients C[m, n] of psi_m = sum_n C[m, n] r^i_n s^j_n, orthonormal under
    (1/2) int_T: Gram-Schmidt of the graded monomials (so the first modes of
    degree <= d span the polynomials of degree <= d).  Returns (C, exps, degree)."""
    exps = monomial_exponents(p)
    r, s, w = duffy_rule(p + 2)
    Vm = np.stack([r ** i * s ** j for i, j in exps], axis=1)
    G = 0.5 * (Vm * w[:, None]).T @ Vm
    N = len(exps)
    C = np.zeros((N, N))
    for m in range(N):
        c = np.zeros(N)
        c[m] = 1.0
        for _ in range(2):  # Gram-Schmidt twice for full orthogonality
            for l in range(m):
                c = c - (C[l] @ G @ c) * C[l]
        C[m] = c / math.sqrt(c @ G @ c)
    deg = np.array([i + j for i, j in exps])
    return C, exps, deg


def basis_eval(p, r, s):
    """psi_m(r, s), shape (len(r), N)."""
    C, exps, _ = orthonormal_basis(p)
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    Vm = np.stack([r ** i * s ** j for i, j in exps], axis=1)
    return Vm @ C.T


def basis_grad(p, r, s):
    """(d psi_m / dr, d psi_m / ds), each of shape (len(r), N)."""
    C, exps, _ = orthonormal_basis(p)
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    dr = np.stack([i * r ** max(i - 1, 0) * s ** j if i > 0 else np.zeros_like(r) for i, j in exps], axis=1)
    ds = np.stack([j * r ** i * s ** max(j - 1, 0) if j > 0 else np.zeros_like(r) for i, j in exps], axis=1)
    return dr @ C.T, ds @ C.T


def lgl_nodes(n):
    """n+1 Legendre-Gauss-Lobatto nodes: -1, 1 and the roots of P_n'."""
    if n == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(n).deriv().roots()
    return np.concatenate(([-1.0], np.sort(inner.real), [1.0]))


def _warp(n, x):
    """Warp of the equispaced points towards the LGL points, evaluated at x and
    divided by the edge blend factor 1 - x^2 (0 at the end points)."""
    req = np.linspace(-1.0, 1.0, n + 1)
    disp = lgl_nodes(n) - req
    L = lagrange_values(req, x)
    w = L @ disp
    inside = np.abs(x) < 1.0 - 1e-10
    out = np.zeros_like(w)
    out[inside] = w[inside] / (1.0 - x[inside] ** 2)
    return out


@lru_cache(maxsize=None)
def solution_points(p):
    """Warp-and-blend nodes on T (no optimisation parameter), ordered by the
    equispaced lattice: row b = 0..p (bottom to top), in each row a = 0..p-b."""
    n = p
    if n == 0:
        return np.array([-1.0 / 3.0]), np.array([-1.0 / 3.0])
    L1, L3 = [], []
    for b in range(n + 1):
        for a in range(n + 1 - b):
            L1.append(a / n)
            L3.append(b / n)
    # barycentric coordinates of (r, s): lam2 weights vertex (1,-1), lam3 vertex (-1,1)
    lam2 = np.array(L1)
    lam3 = np.array(L3)
    lam1 = 1.0 - lam2 - lam3
    # equilateral triangle with vertices v1 = (-1, -1/sqrt3), v2 = (1, -1/sqrt3), v3 = (0, 2/sqrt3)
    X = -lam1 + lam2
    Y = (-lam1 - lam2 + 2.0 * lam3) / math.sqrt(3.0)
    # warp along each edge direction, blended towards the interior
    for (la, lb, lc), ang in (((lam1, lam2, lam3), 0.0),
                              ((lam2, lam3, lam1), 2.0 * math.pi / 3.0),
                              ((lam3, lam1, lam2), 4.0 * math.pi / 3.0)):
        # edge from vertex a to vertex b, opposite vertex c
        blend = 4.0 * la * lb
        warp = blend * _warp(n, lb - la)
        X = X + math.cos(ang) * warp
        Y = Y + math.sin(ang) * warp
    # back to barycentric, then to (r, s)
    l3 = (math.sqrt(3.0) * Y + 1.0) / 3.0
    l2 = (X + 1.0 - l3) / 2.0
    l1 = 1.0 - l2 - l3
    r = -l1 + l2 - l3
    s = -l1 - l2 + l3
    return r, s


def face_param(f, t):
    """(r, s) of edge parameter t on reference face f (vertex f to vertex f+1)."""
    t = np.asarray(t, dtype=np.float64)
    if f == 0:
        return t, -np.ones_like(t)
    if f == 1:
        return -t, t
    return -np.ones_like(t), -t


@dataclass
class TriTables:
    p: int
    r: np.ndarray        # solution points
    s: np.ndarray
    V: np.ndarray        # V[j, m] = psi_m(r_j)
    Vinv: np.ndarray
    Dr: np.ndarray       # Dr[j, i] = d l_i / dr (r_j)
    Ds: np.ndarray
    tq: np.ndarray       # face Gauss points (p+1) and weights (sum 2)
    wq: np.ndarray
    Lf: np.ndarray       # Lf[f, k, i] = l_i at flux point k of face f
    divh: np.ndarray     # divh[j, f, k]: divergence of the correction field of (f, k) at r_j
    deg: np.ndarray      # total degree of each modal function
    mean_w: np.ndarray   # element mean = sum_j mean_w[j] u_j

    @property
    def n(self):
        return len(self.r)


def _lagrange_eval(p, V_inv, r, s):
    """l_i(r, s) for the nodal basis on the solution points: psi(r,s) V^{-1}."""
    return basis_eval(p, r, s) @ V_inv


def correction_divergence(p, r, s):
    """divh[j, f, k]: the polynomial phi of degree p with int_T phi v = int_face l_k v ds
    for all v of degree p (the lifting that makes FR on triangles nodal DG),
    evaluated at the points (r_j, s_j).  Face integrals by a (p+3)-point Gauss rule."""
    tq, _ = gauss_legendre(p + 1)
    tg, wg = gauss_legendre(p + 3)
    rq, sq, wq = duffy_rule(p + 2)
    Pq = basis_eval(p, rq, sq)
    Mass = (Pq * wq[:, None]).T @ Pq            # int_T psi_m psi_n
    out = np.zeros((len(r), 3, p + 1))
    Pj = basis_eval(p, r, s)
    for f in range(3):
        fr, fs = face_param(f, tg)
        Pf = basis_eval(p, fr, fs)                  # psi_m at the face Gauss points
        lk = lagrange_values(tq, tg)                # l_k(t_g), 1D Lagrange on the flux points
        for k in range(p + 1):
            rhs = (REF_FACE_LEN[f] / 2.0) * (Pf * (wg * lk[:, k])[:, None]).sum(axis=0)
            c = np.linalg.solve(Mass, rhs)
            out[:, f, k] = Pj @ c
    return out


@lru_cache(maxsize=None)
def build_tri_tables(p):
    r, s = solution_points(p)
    V = basis_eval(p, r, s)
    Vinv = np.linalg.inv(V)
    gr, gs = basis_grad(p, r, s)
    Dr, Ds = gr @ Vinv, gs @ Vinv
    tq, wq = gauss_legendre(p + 1)
    Lf = np.zeros((3, p + 1, len(r)))
    for f in range(3):
        fr, fs = face_param(f, tq)
        Lf[f] = _lagrange_eval(p, Vinv, fr, fs)
    divh = correction_divergence(p, r, s)
    _, _, deg = orthonormal_basis(p)
    # mean over the element = (1/2) int_T u = coefficient of psi_0 (psi_0 = 1)
    mean_w = Vinv[0]
    return TriTables(p, r, s, V, Vinv, Dr, Ds, tq, wq, Lf, divh, deg, mean_w)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

@dataclass
class TriGeometry:
    det: np.ndarray      # [E] = area / 2
    rx: np.ndarray       # [E] metric terms dr/dx, dr/dy, ds/dx, ds/dy
    ry: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    flen: np.ndarray     # [E, 3] face lengths
    nx: np.ndarray       # [E, 3] unit outward normals
    ny: np.ndarray
    dins: np.ndarray     # [E] inscribed-circle diameter


def geometry(xy):
    x1, x2, x3 = xy[:, 0], xy[:, 1], xy[:, 2]
    xr, yr = (x2[:, 0] - x1[:, 0]) / 2.0, (x2[:, 1] - x1[:, 1]) / 2.0
    xs, ys = (x3[:, 0] - x1[:, 0]) / 2.0, (x3[:, 1] - x1[:, 1]) / 2.0
    det = xr * ys - xs * yr
    if np.any(det <= 0.0):
        raise ValueError("triangles must be counter-clockwise and non-degenerate")
    d = np.stack([xy[:, (f + 1) % 3] - xy[:, f] for f in range(3)], axis=1)  # [E, 3, 2]
    flen = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    nx, ny = d[..., 1] / flen, -d[..., 0] / flen
    area = 2.0 * det
    return TriGeometry(det, ys / det, -xs / det, -yr / det, xr / det, flen, nx, ny, 4.0 * area / flen.sum(axis=1))


def solution_point_coords_tri(prob, T):
    xy = prob.mesh["xy"]
    l1 = -(T.r + T.s) / 2.0
    l2 = (T.r + 1.0) / 2.0
    l3 = (T.s + 1.0) / 2.0
    X = l1[None] * xy[:, 0, 0:1] + l2[None] * xy[:, 1, 0:1] + l3[None] * xy[:, 2, 0:1]
    Y = l1[None] * xy[:, 0, 1:2] + l2[None] * xy[:, 1, 1:2] + l3[None] * xy[:, 2, 1:2]
    return X, Y


# ----------------------------------------------------------------------------
# fluxes along a unit normal (Euler 2D)
# ----------------------------------------------------------------------------

def normal_flux(prob, U, nx, ny):
    rho, mx, my, E = U[0], U[1], U[2], U[3]
    p = euler_pressure(U, prob.gamma, 2)
    vn = (mx * nx + my * ny) / rho
    return np.stack([rho * vn, mx * vn + p * nx, my * vn + p * ny, (E + p) * vn])


def _sound(prob, U):
    return np.sqrt(prob.gamma * euler_pressure(U, prob.gamma, 2) / U[0])


def interactive_flux_n(prob, UL, UR, nx, ny):
    """Lax-Friedrichs or HLL flux along the unit normal (nx, ny), per random node."""
    FL, FR = normal_flux(prob, UL, nx, ny), normal_flux(prob, UR, nx, ny)
    uL = (UL[1] * nx + UL[2] * ny) / UL[0]
    uR = (UR[1] * nx + UR[2] * ny) / UR[0]
    cL, cR = _sound(prob, UL), _sound(prob, UR)
    if prob.flux == "hll":
        SL = np.minimum(uL - cL, uR - cR)
        SR = np.maximum(uL + cL, uR + cR)
        mid = (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)
        return np.where(SL >= 0.0, FL, np.where(SR <= 0.0, FR, mid))
    lam = np.maximum(np.abs(uL) + cL, np.abs(uR) + cR)
    return 0.5 * (FL + FR) - 0.5 * lam * (UR - UL)


def ghost_n(prob, side, trace, nx, ny):
    """Ghost state outside a boundary face of kind bc[side]: Dirichlet, outflow, or
    reflection of the velocity about the face (v - 2 (v . n) n)."""
    kind = prob.bc[side]
    if kind == "outflow":
        return trace.copy()
    if kind == "dirichlet":
        st = np.asarray(prob.bc_state[side][:4], dtype=np.float64)
        return np.broadcast_to(st.reshape((4,) + (1,) * (trace.ndim - 1)), trace.shape).copy()
    if kind == "reflect":
        g = trace.copy()
        mn = trace[1] * nx + trace[2] * ny
        g[1] = trace[1] - 2.0 * mn * nx
        g[2] = trace[2] - 2.0 * mn * ny
        return g
    raise ValueError("boundary kind %s on a boundary face" % kind)


# ----------------------------------------------------------------------------
# right-hand side
# ----------------------------------------------------------------------------

def rhs_tri(prob, T, R, u):
    """du/dt at the solution points of every triangle, in the order of the
    quadrilateral path: expand at the nodes, project the fluxes, traces and
    interactive flux per node (projected), interpolated discontinuous flux at
    the flux points, divergence plus corrections, negated."""
    if prob.equation != "euler2d":
        raise ValueError("triangles carry the 2D Euler equations")
    G = geometry(prob.mesh["xy"])
    nbr, nbf = prob.mesh["nbr"], prob.mesh["nbr_face"]
    S, M, E, N = u.shape
    p = T.p
    # 1. chaos expansion at the nodes
    U = np.einsum("kq,skej->sqej", R.Phi, u)
    # 2. projected physical fluxes at the solution points
    from .fr import flux_x, flux_y
    fh = np.einsum("kq,sqej->skej", R.PW, flux_x(prob, U))
    gh = np.einsum("kq,sqej->skej", R.PW, flux_y(prob, U))
    # 3. traces at the flux points, per node: UF[s, q, e, f, k]
    UF = np.einsum("fki,sqei->sqefk", T.Lf, U)
    # the neighbour's trace at the same physical point: its face runs the other way
    interior = nbr >= 0
    outer = UF[:, :, np.where(interior, nbr, 0), np.where(interior, nbf, 0), ::-1].copy()
    for side in range(4):
        bnd = nbr == -1 - side
        if bnd.any():
            outer[:, :, bnd] = ghost_n(prob, side, UF[:, :, bnd], G.nx[bnd][:, None], G.ny[bnd][:, None])
    Fst = interactive_flux_n(prob, UF, outer, G.nx[:, :, None], G.ny[:, :, None])
    Fsth = np.einsum("kq,sqefl->skefl", R.PW, Fst)
    # 4. discontinuous normal flux at the flux points (interpolated projected flux)
    FD = (np.einsum("fki,smei->smefk", T.Lf, fh) * G.nx[None, None, :, :, None]
          + np.einsum("fki,smei->smefk", T.Lf, gh) * G.ny[None, None, :, :, None])
    # 5. divergence of the interpolated flux, plus the corrections
    div = (np.einsum("ji,smei->smej", T.Dr, fh) * G.rx[None, None, :, None]
           + np.einsum("ji,smei->smej", T.Ds, fh) * G.sx[None, None, :, None]
           + np.einsum("ji,smei->smej", T.Dr, gh) * G.ry[None, None, :, None]
           + np.einsum("ji,smei->smej", T.Ds, gh) * G.sy[None, None, :, None])
    scale = G.flen / np.array(REF_FACE_LEN)[None, :] / G.det[:, None]     # [E, 3]
    jump = (Fsth - FD) * scale[None, None, :, :, None]
    corr = np.einsum("jfk,smefk->smej", T.divh, jump)
    # 6. du/dt = -(divergence + corrections)
    return -(div + corr)


def cfl_dt_tri(prob, T, R, u):
    """dt = CFL / ((p+1) max(lambda / d_e)), lambda = |v| + c at the solution points and
    nodes, d_e the inscribed-circle diameter (the paper gives CFL numbers only; the rule
    is pinned by the SSP-RK3 stability of the linearised triangle operator: stable at
    CFL 0.3 with a limit between 0.4 and 1.0)."""
    G = geometry(prob.mesh["xy"])
    U = np.einsum("kq,skej->sqej", R.Phi, u)
    lam = np.sqrt(U[1] ** 2 + U[2] ** 2) / U[0] + _sound(prob, U)
    rate = (lam / G.dins[None, :, None]).max()
    return prob.cfl / ((prob.p + 1) * rate)

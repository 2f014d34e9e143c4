"""Independent test-side formulations used to pin the oracle.

Nothing here is imported by the oracle or by the library.  Tables come from
numpy.polynomial.legendre (a library routine distinct from the oracle's own
Golub-Welsch/recurrence code), and the spatial operator is the nodal
discontinuous Galerkin weak form, which flux reconstruction with Radau
correction functions reproduces exactly (Huynh's g_DG correction, cited in
Sec. 1 and Sec. 3.3 of the paper):

  J w_i du_i/dt = sum_q w_q l_i'(r_q) f_q - l_i(1) F*_R + l_i(-1) F*_L

with the Gauss rule on the solution points (exact for these integrands).
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def gl(n):
    return npleg.leggauss(n)


def lagrange_matrix(nodes, x):
    """L[i, j] = l_j(x_i) via a Vandermonde solve (independent of product formulas)."""
    n = len(nodes)
    Vn = npleg.legvander(nodes, n - 1)
    Vx = npleg.legvander(np.atleast_1d(x), n - 1)
    return Vx @ np.linalg.inv(Vn)


def lagrange_deriv_matrix(nodes, x):
    n = len(nodes)
    Vn = npleg.legvander(nodes, n - 1)
    dV = np.zeros((len(np.atleast_1d(x)), n))
    for m in range(n):
        c = np.zeros(n)
        c[m] = 1.0
        dV[:, m] = npleg.legval(np.atleast_1d(x), npleg.legder(c))
    return dV @ np.linalg.inv(Vn)


def chaos(order, nq):
    """Phi[k, q] = sqrt(2k+1) P_k(z_q) and weights summing to 1 (1D)."""
    z, w = gl(nq)
    Phi = np.array([np.sqrt(2 * k + 1) * npleg.legval(z, np.eye(order + 1)[k]) for k in range(order + 1)])
    return z, w / 2.0, Phi


def euler1d_flux(U, gamma):
    rho, m, E = U
    v = m / rho
    p = (gamma - 1) * (E - 0.5 * rho * v * v)
    return np.array([m, m * v + p, (E + p) * v]), np.abs(v) + np.sqrt(gamma * p / rho)


def scalar_flux(eq, U, a):
    if eq == "advection":
        return a * U, np.full(U.shape[1:], abs(a))
    return 0.5 * U * U, np.abs(U[0])


def dg_weak_rhs_1d(eq, u, p, order, nq, dx, a=1.0, gamma=1.4, bc="periodic", bc_states=None):
    """SG-DG weak-form RHS for 1D problems; u[s, k, e, j] modal in z, nodal in x."""
    r, w = gl(p + 1)
    z, wq, Phi = chaos(order, nq)
    PW = Phi * wq[None]
    Dd = lagrange_deriv_matrix(r, r)        # Dd[q, i] = l_i'(r_q)
    lm = lagrange_matrix(r, [-1.0])[0]
    lp = lagrange_matrix(r, [1.0])[0]
    S, M, E, N = u.shape
    J = dx / 2.0
    U = np.tensordot(Phi, u, axes=([0], [1])).transpose(1, 0, 2, 3)   # [s, q, e, j]

    def flux(X):
        if eq == "euler1d":
            return euler1d_flux(X, gamma)
        return scalar_flux(eq, X, a)

    f, _ = flux(U)
    # volume term: sum_q w_q l_i'(r_q) f(r_q), per node in z
    vol = np.einsum("q,qi,szeq->szei", w, Dd, f)
    Um = np.einsum("j,szej->sze", lm, U)
    Up = np.einsum("j,szej->sze", lp, U)
    if bc == "periodic":
        Lf = np.concatenate([Up[:, :, -1:], Up], axis=2)
        Rf = np.concatenate([Um, Um[:, :, :1]], axis=2)
    else:
        gl_ = np.broadcast_to(np.asarray(bc_states[0][:S])[:, None, None], (S, U.shape[1], 1))
        gr_ = np.broadcast_to(np.asarray(bc_states[1][:S])[:, None, None], (S, U.shape[1], 1))
        Lf = np.concatenate([gl_, Up], axis=2)
        Rf = np.concatenate([Um, gr_], axis=2)
    fL, sL = flux(Lf)
    fR, sR = flux(Rf)
    lam = np.maximum(sL, sR)
    Fs = 0.5 * (fL + fR) - 0.5 * lam[None] * (Rf - Lf)        # [s, q, face]
    surf = np.einsum("i,sze->szei", lp, Fs[:, :, 1:]) - np.einsum("i,sze->szei", lm, Fs[:, :, :-1])
    dudt_nodal = (vol - surf) / (J * w[None, None, None, :])
    return np.einsum("kz,szei->skei", PW, dudt_nodal)


def euler2d_flux(U, gamma, normal):
    """Euler flux along axis `normal` (0: x, 1: y) and the spectral radius |u_n| + c."""
    rho, mx, my, E = U
    ux, uy = mx / rho, my / rho
    p = (gamma - 1) * (E - 0.5 * rho * (ux * ux + uy * uy))
    un = ux if normal == 0 else uy
    m_n = mx if normal == 0 else my
    f = np.array([m_n, mx * un + (p if normal == 0 else 0.0), my * un + (p if normal == 1 else 0.0),
                  (E + p) * un])
    return f, np.abs(un) + np.sqrt(gamma * p / rho)


def _lf(UL, UR, gamma, normal):
    fL, sL = euler2d_flux(UL, gamma, normal)
    fR, sR = euler2d_flux(UR, gamma, normal)
    return 0.5 * (fL + fR) - 0.5 * np.maximum(sL, sR)[None] * (UR - UL)


def _ghost2d(kind, interior, state, normal):
    """Ghost trace beyond a boundary face: fixed state, copy, or mirrored normal momentum."""
    if kind == "dirichlet":
        return np.broadcast_to(np.asarray(state[:4], dtype=float).reshape((4,) + (1,) * (interior.ndim - 1)),
                               interior.shape).copy()
    g = interior.copy()
    if kind == "reflect":
        g[1 + normal] = -g[1 + normal]
    return g


def dg_weak_rhs_2d_euler(u, p, order_nodes, Phi, wq, nx, ny, dx, dy, bc, bc_states, gamma=1.4):
    """SG-DG weak-form RHS for 2D Euler on an nx x ny mesh of dx x dy rectangles.

    u[s, k, e, j]: modal in z (chaos Phi[k, q], weights wq summing to 1), nodal
    in x at the tensor Gauss points, e = iy nx + ix, j = a + (p+1) b.  For the
    test function l_a(r) l_b(s) on the reference square, with Jx = dx/2,
    Jy = dy/2 and the Gauss rule collocated on the solution points:

      Jx Jy w_a w_b dU_ab/dt = Jy sum_c w_c w_b l_a'(r_c) F_cb + Jx sum_c w_a w_c l_b'(s_c) G_ac
                               - Jy w_b [l_a(1) F*_{x+}(b) - l_a(-1) F*_{x-}(b)]
                               - Jx w_a [l_b(1) G*_{y+}(a) - l_b(-1) G*_{y-}(a)]

    per random node, then the nodal residual is projected on the chaos.
    `order_nodes` is unused except as a size check (Phi carries the basis).
    bc: kinds of the x-lo, x-hi, y-lo, y-hi sides."""
    n = p + 1
    r, w = gl(n)
    Dd = lagrange_deriv_matrix(r, r)        # Dd[c, a] = l_a'(r_c)
    lm = lagrange_matrix(r, [-1.0])[0]
    lp = lagrange_matrix(r, [1.0])[0]
    S, M, E, _ = u.shape
    assert S == 4 and E == nx * ny and Phi.shape[1] == order_nodes
    Jx, Jy = dx / 2.0, dy / 2.0
    # nodal values per random node: U[s, q, iy, ix, b, a]
    U = np.einsum("kq,skyxba->sqyxba", Phi, u.reshape(4, M, ny, nx, n, n))
    F, _ = euler2d_flux(U, gamma, 0)
    G, _ = euler2d_flux(U, gamma, 1)
    # volume terms: sum_c w_c l_a'(r_c) F(c, b) and the y analogue
    vol_x = np.einsum("c,ca,sqyxbc->sqyxba", w, Dd, F)
    vol_y = np.einsum("c,cb,sqyxca->sqyxba", w, Dd, G)
    # traces on the x faces (rows b) and y faces (columns a)
    Xm = np.einsum("a,sqyxba->sqyxb", lm, U)
    Xp = np.einsum("a,sqyxba->sqyxb", lp, U)
    Ym = np.einsum("b,sqyxba->sqyxa", lm, U)
    Yp = np.einsum("b,sqyxba->sqyxa", lp, U)
    # the states on both sides of every x face: face ix sits left of element ix
    Lx = np.empty(Xm.shape[:3] + (nx + 1,) + Xm.shape[4:])
    Rx = np.empty_like(Lx)
    Lx[:, :, :, 1:] = Xp
    Rx[:, :, :, :nx] = Xm
    if bc[0] == "periodic":
        Lx[:, :, :, 0] = Xp[:, :, :, nx - 1]
        Rx[:, :, :, nx] = Xm[:, :, :, 0]
    else:
        Lx[:, :, :, 0] = _ghost2d(bc[0], Xm[:, :, :, 0], bc_states[0], 0)
        Rx[:, :, :, nx] = _ghost2d(bc[1], Xp[:, :, :, nx - 1], bc_states[1], 0)
    Fs = _lf(Lx, Rx, gamma, 0)                      # [s, q, iy, face, b]
    Ly = np.empty(Ym.shape[:2] + (ny + 1,) + Ym.shape[3:])
    Ry = np.empty_like(Ly)
    Ly[:, :, 1:] = Yp
    Ry[:, :, :ny] = Ym
    if bc[2] == "periodic":
        Ly[:, :, 0] = Yp[:, :, ny - 1]
        Ry[:, :, ny] = Ym[:, :, 0]
    else:
        Ly[:, :, 0] = _ghost2d(bc[2], Ym[:, :, 0], bc_states[2], 1)
        Ry[:, :, ny] = _ghost2d(bc[3], Yp[:, :, ny - 1], bc_states[3], 1)
    Gs = _lf(Ly, Ry, gamma, 1)                      # [s, q, face, ix, a]
    surf_x = (np.einsum("a,sqyxb->sqyxba", lp, Fs[:, :, :, 1:]) - np.einsum("a,sqyxb->sqyxba", lm, Fs[:, :, :, :nx]))
    surf_y = (np.einsum("b,sqyxa->sqyxba", lp, Gs[:, :, 1:]) - np.einsum("b,sqyxa->sqyxba", lm, Gs[:, :, :ny]))
    wa = w[None, None, None, None, None, :]
    wb = w[None, None, None, None, :, None]
    nodal = (Jy * wb * (vol_x - surf_x) + Jx * wa * (vol_y - surf_y)) / (Jx * Jy * wa * wb)
    out = np.einsum("kq,sqyxba->skyxba", Phi * wq[None], nodal)
    return out.reshape(4, M, E, n * n)

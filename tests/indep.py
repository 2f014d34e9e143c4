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

"""Polynomial, quadrature and operator tables (FP64).

Physical space (Sec. 3.2, 3.3): N_p = p+1 Legendre-Gauss solution points r_j on
[-1, 1]; Lagrange basis l_j; derivative matrix D[i, j] = l_j'(r_i); boundary
values l_j(-1), l_j(+1); Radau correction functions h_L, h_R with
h_L(r) = h_R(-r), h_L(-1) = 1, h_L(1) = 0 (Sec. 3.3 constraints).  The right
Radau polynomial of degree p+1 is used for h_L ("Correction: Radau" in the
setup tables of Sec. 5).

Nodal/modal transform (Sec. 4, Eq. vandermonde matrix): modal basis
Psi_j = sqrt(2j+1) P_j, orthonormal under dr/2; V[j, k] = Psi_k(r_j), so that
nodal = V @ modal.

Random space (Sec. 2.1): Legendre chaos Phi_k = sqrt(2k+1) P_k, orthonormal
under the uniform density on [-1, 1] (E[Phi_j Phi_k] = delta_jk); the
expectation is evaluated with an N_q-point Gauss-Legendre rule whose weights
sum to one (Eq. discrete expectation value).  With two random dimensions the
basis is the total-degree product set |k| <= N_c in graded order
(0,0), (1,0), (0,1), (2,0), (1,1), (0,2), ... with a tensor Gauss rule.
"""

import math
from dataclasses import dataclass

import numpy as np


def legendre_values(n, x):
    """P_0..P_n at x by Bonnet's three-term recurrence; shape (n+1,) + x.shape."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((n + 1,) + x.shape)
    P[0] = 1.0
    if n >= 1:
        P[1] = x
    for m in range(1, n):
        P[m + 1] = ((2 * m + 1) * x * P[m] - m * P[m - 1]) / (m + 1)
    return P


def legendre_derivs(n, x):
    """P_0'..P_n' at x from P'_{m+1} = P'_{m-1} + (2m+1) P_m."""
    x = np.asarray(x, dtype=np.float64)
    P = legendre_values(n, x)
    dP = np.zeros_like(P)
    if n >= 1:
        dP[1] = 1.0
    for m in range(1, n):
        dP[m + 1] = dP[m - 1] + (2 * m + 1) * P[m]
    return dP


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes and weights on [-1, 1] (weights sum to 2).

    Golub-Welsch: the nodes are the eigenvalues of the symmetric Jacobi matrix
    of the Legendre recurrence, the weights 2 * (first eigenvector component)^2.
    """
    if n == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, n, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    Jm = np.diag(beta, 1) + np.diag(beta, -1)
    vals, vecs = np.linalg.eigh(Jm)
    order = np.argsort(vals)
    x = vals[order]
    w = 2.0 * vecs[0, order] ** 2
    # one Newton polish of each node on P_n for full double accuracy
    P = legendre_values(n, x)
    dP = legendre_derivs(n, x)
    x = x - P[n] / dP[n]
    dP = legendre_derivs(n, x)
    w = 2.0 / ((1.0 - x * x) * dP[n] ** 2)
    return x, w


def legendre_l1_norms(n):
    """||sqrt(2j+1) P_j||_1 under dr/2 on [-1, 1], j = 0..n-1 (the L1 norms of the
    orthonormal Legendre functions that enter the Lasso filter, Sec. 4.1.3).

    |P_j| is integrated piece by piece between consecutive roots of P_j, where
    it has one sign, by a Gauss-Legendre rule of j+1 points on each piece
    (exact for a polynomial of degree j)."""
    out = np.zeros(n)
    for j in range(n):
        roots = gauss_legendre(j)[0] if j > 0 else np.zeros(0)
        cuts = np.concatenate(([-1.0], roots, [1.0]))
        xg, wg = gauss_legendre(j + 1)
        total = 0.0
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            x = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
            total += abs(0.5 * (hi - lo) * np.dot(wg, legendre_values(j, x)[j]))
        out[j] = math.sqrt(2 * j + 1) * 0.5 * total
    return out


def lagrange_values(r_nodes, x):
    """l_j(x) for the Lagrange basis on r_nodes (Sec. 3.2); shape (len(x), N)."""
    r_nodes = np.asarray(r_nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    N = len(r_nodes)
    L = np.ones((len(x), N))
    for j in range(N):
        for m in range(N):
            if m != j:
                L[:, j] *= (x - r_nodes[m]) / (r_nodes[j] - r_nodes[m])
    return L


def lagrange_derivs(r_nodes, x):
    """l_j'(x) by the product rule; shape (len(x), N)."""
    r_nodes = np.asarray(r_nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    N = len(r_nodes)
    dL = np.zeros((len(x), N))
    for j in range(N):
        for m in range(N):
            if m == j:
                continue
            term = np.full(len(x), 1.0 / (r_nodes[j] - r_nodes[m]))
            for n in range(N):
                if n != j and n != m:
                    term *= (x - r_nodes[n]) / (r_nodes[j] - r_nodes[n])
            dL[:, j] += term
    return dL


def radau_right(p, x):
    """Right Radau polynomial of degree p+1: ((-1)^(p+1)/2) (P_{p+1} - P_p); and its derivative."""
    P = legendre_values(p + 1, x)
    dP = legendre_derivs(p + 1, x)
    s = (-1.0) ** (p + 1) / 2.0
    return s * (P[p + 1] - P[p]), s * (dP[p + 1] - dP[p])


@dataclass
class Tables1D:
    """One-direction FR tables for degree p (N_p = p+1 points)."""
    p: int
    r: np.ndarray        # solution points
    w: np.ndarray        # Gauss weights (sum 2)
    D: np.ndarray        # D[i, j] = l_j'(r_i)
    lL: np.ndarray       # l_j(-1)
    lR: np.ndarray       # l_j(+1)
    dhL: np.ndarray      # h_L'(r_j)
    dhR: np.ndarray      # h_R'(r_j)
    V: np.ndarray        # V[j, k] = Psi_k(r_j)
    Vinv: np.ndarray

    @property
    def n(self):
        return self.p + 1


def build_fr_tables(p):
    r, w = gauss_legendre(p + 1)
    D = lagrange_derivs(r, r)
    lL = lagrange_values(r, [-1.0])[0]
    lR = lagrange_values(r, [1.0])[0]
    _, dhL = radau_right(p, r)
    # h_R(r) = h_L(-r)  =>  h_R'(r) = -h_L'(-r)
    _, dhL_neg = radau_right(p, -r)
    dhR = -dhL_neg
    P = legendre_values(p, r)  # (p+1, N)
    V = (np.sqrt(2.0 * np.arange(p + 1) + 1.0)[:, None] * P).T
    Vinv = np.linalg.inv(V)
    return Tables1D(p, r, w, D, lL, lR, dhL, dhR, V, Vinv)


def total_degree_indices(order, rdim):
    """Multi-indices with |k| <= order in graded order; rdim in {1, 2}."""
    if rdim == 1:
        return [(k,) for k in range(order + 1)]
    out = []
    for d in range(order + 1):
        for k2 in range(d + 1):
            out.append((d - k2, k2))
    return out


@dataclass
class RandomTables:
    order: int
    rdim: int
    kidx: list           # multi-indices, length M
    kdeg: np.ndarray     # |k| per mode
    z: np.ndarray        # (Nq, rdim) nodes
    wq: np.ndarray       # (Nq,) weights, sum 1
    Phi: np.ndarray      # (M, Nq): Phi_k(z_q)
    PW: np.ndarray       # (M, Nq): w_q Phi_k(z_q)

    @property
    def M(self):
        return len(self.kidx)

    @property
    def Nq(self):
        return len(self.wq)


def build_random_tables(order, rdim, nq1d):
    z1, w1 = gauss_legendre(nq1d)
    w1 = w1 / 2.0
    kidx = total_degree_indices(order, rdim)
    P1 = legendre_values(order, z1) * np.sqrt(2.0 * np.arange(order + 1) + 1.0)[:, None]
    if rdim == 1:
        z = z1[:, None]
        wq = w1.copy()
        Phi = np.array([P1[k[0]] for k in kidx])
    else:
        # node q = a + nq1d * b  (first random coordinate fastest)
        za, zb = np.meshgrid(z1, z1, indexing="xy")
        z = np.stack([za.ravel(), zb.ravel()], axis=1)
        wq = (w1[None, :] * w1[:, None]).ravel()
        Phi = np.array([np.outer(P1[k2], P1[k1]).ravel() for (k1, k2) in kidx])
    kdeg = np.array([sum(k) for k in kidx])
    return RandomTables(order, rdim, kidx, kdeg, z, wq, Phi, Phi * wq[None, :])


def build_tables(problem):
    if problem.element == "tri":
        from .tri import build_tri_tables
        return build_tri_tables(problem.p), build_random_tables(problem.gpc_order, problem.rdim, problem.nq1d)
    return build_fr_tables(problem.p), build_random_tables(problem.gpc_order, problem.rdim, problem.nq1d)


def sensor_threshold(s0, kappa):
    """Eq. (detector): theta < 0.99 with s_e = log10(S_e) rewritten as S_e > S*.

    In the middle branch theta = (1 - sin(pi (s_e - s0) / (2 kappa))) / 2 < 0.99
    iff s_e > s0 - (2 kappa / pi) asin(0.98); the outer branches agree with it.
    """
    return 10.0 ** (s0 - (2.0 * kappa / math.pi) * math.asin(0.98))

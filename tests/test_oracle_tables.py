"""Pins for the oracle's tables (Sec. 2.1, Sec. 3.2-3.3, Sec. 4, Eq. detector)."""

import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import tables as ot


@pytest.mark.parametrize("n", list(range(1, 26)))
def test_gauss_legendre_matches_library_and_is_exact(n):
    x, w = ot.gauss_legendre(n)
    xr, wr = npleg.leggauss(n)
    assert np.allclose(x, xr, atol=2e-15, rtol=0)
    assert np.allclose(w, wr, atol=6e-15, rtol=0)
    # exact on monomials up to degree 2n-1: int_{-1}^{1} x^m dx
    for m in range(2 * n):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(w * x ** m) - exact) < 5e-14


def test_legendre_recurrence_matches_library():
    x = np.linspace(-1, 1, 37)
    P = ot.legendre_values(12, x)
    dP = ot.legendre_derivs(12, x)
    for n in range(13):
        c = np.eye(13)[n]
        assert np.allclose(P[n], npleg.legval(x, c), atol=1e-14)
        assert np.allclose(dP[n], npleg.legval(x, npleg.legder(c)), atol=1e-12)


@pytest.mark.parametrize("order,rdim,nq", [(4, 1, 8), (8, 1, 16), (10, 1, 24), (4, 2, 5), (3, 2, 4)])
def test_chaos_orthonormal_under_discrete_expectation(order, rdim, nq):
    """E[Phi_j Phi_k] = delta_jk (Sec. 2.1) with the Gauss rule, weights summing to 1."""
    R = ot.build_random_tables(order, rdim, nq)
    assert abs(R.wq.sum() - 1.0) < 1e-14
    G = (R.Phi * R.wq[None]) @ R.Phi.T
    assert np.allclose(G, np.eye(R.M), atol=1e-13)
    expect_M = order + 1 if rdim == 1 else (order + 1) * (order + 2) // 2
    assert R.M == expect_M


def test_two_dim_chaos_is_a_product_and_graded():
    R = ot.build_random_tables(4, 2, 5)
    assert R.kidx[:6] == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    assert list(R.kdeg) == sorted(R.kdeg)
    z1, _ = npleg.leggauss(5)
    # node q = a + 5 b : z = (z1[a], z1[b])
    q = 2 + 5 * 3
    assert np.allclose(R.z[q], [z1[2], z1[3]])
    k = R.kidx.index((2, 1))
    v = math.sqrt(5) * npleg.legval(z1[2], [0, 0, 1]) * math.sqrt(3) * z1[3]
    assert abs(R.Phi[k, q] - v) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_derivative_matrix_exact_on_polynomials(p):
    T = ot.build_fr_tables(p)
    for m in range(p + 1):
        f = T.r ** m
        df = m * T.r ** (m - 1) if m > 0 else np.zeros_like(T.r)
        assert np.allclose(T.D @ f, df, atol=1e-12)
    # Lagrange boundary values reproduce polynomials at the faces
    for m in range(p + 1):
        assert abs(T.lL @ (T.r ** m) - (-1.0) ** m) < 1e-13
        assert abs(T.lR @ (T.r ** m) - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_radau_correction_constraints_and_dg_identity(p):
    """h_L(-1)=1, h_L(1)=0, h_L(r)=h_R(-r) (Sec. 3.3); Radau == DG lifting."""
    hL = lambda r: ot.radau_right(p, np.asarray(r, float))[0]
    assert abs(hL(-1.0) - 1.0) < 1e-14 and abs(hL(1.0)) < 1e-14
    T = ot.build_fr_tables(p)
    # h_R(r) = h_L(-r): derivative relation checked numerically by finite differences
    h = 1e-6
    for rj, dR in zip(T.r, T.dhR):
        fd = (hL(-(rj + h)) - hL(-(rj - h))) / (2 * h)
        assert abs(fd - dR) < 1e-7
    # closed-form DG identity: h_R'(r_j) = l_j(1)/w_j, h_L'(r_j) = -l_j(-1)/w_j
    assert np.allclose(T.dhR, T.lR / T.w, atol=1e-12)
    assert np.allclose(T.dhL, -T.lL / T.w, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_vandermonde_orthonormal_modal_basis(p):
    T = ot.build_fr_tables(p)
    G = T.V.T @ np.diag(T.w / 2.0) @ T.V
    assert np.allclose(G, np.eye(p + 1), atol=1e-13)
    assert np.allclose(T.V @ T.Vinv, np.eye(p + 1), atol=1e-13)


def test_sensor_threshold_is_detector_boundary():
    """theta(log10 S*) = 0.99 with theta from Eq. (detector); c2 value."""
    for s0, kappa in [(-2 * math.log10(3), 4.0), (-3 * math.log10(3), 4.0), (-1.0, 2.0)]:
        thr = ot.sensor_threshold(s0, kappa)
        se = math.log10(thr)
        assert s0 - kappa <= se <= s0 + kappa
        theta = 0.5 * (1 - math.sin(math.pi * (se - s0) / (2 * kappa)))
        assert abs(theta - 0.99) < 1e-12
    assert abs(ot.sensor_threshold(-2 * math.log10(3), 4.0) - 3.597e-5) < 1e-8

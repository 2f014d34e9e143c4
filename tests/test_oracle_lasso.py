"""Pins for the oracle's Lasso filter (Sec. 4.1.3, Eq. LassoFilterFunction, Eq. fStrength).

Fixed independently of the oracle's own formulas:
* ||sqrt(2j+1) P_j||_1 under dr/2 in closed form for j = 0..3;
* the filtered coefficients are the minimiser of the Lasso cost (squared L2
  distance, halved as in the paper's optimality condition, plus the L1 penalty
  of the Legendre operator applied to each term), found by brute-force search,
  with the L1 norms of the basis functions taken by dense quadrature of the
  functions themselves;
* the strengths are the smallest ones for which that minimiser sets the
  highest pure spatial and pure chaos coefficients to zero (the stated purpose
  of Eq. fStrength), found by bisection on the brute-force minimiser;
* invariants: the mean is untouched, no coefficient grows or changes sign,
  and a second pass changes nothing.
"""

import functools
import math

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import stabilize as ost
from oracle.problem import Problem
from oracle.tables import build_tables, legendre_l1_norms
from paper_2112_05946_amd import inputs


def test_l1_norms_closed_form():
    got = legendre_l1_norms(4)
    ref = [1.0, math.sqrt(3) / 2, 2 * math.sqrt(5) / (3 * math.sqrt(3)), 13 * math.sqrt(7) / 40]
    assert np.allclose(got, ref, rtol=1e-14, atol=0)


@functools.lru_cache(maxsize=None)
def _l1_dense(j):
    """||sqrt(2j+1) P_j||_1 under dr/2 by the midpoint rule on 400k cells."""
    x = (np.arange(400000) + 0.5) / 400000 * 2.0 - 1.0
    P = np.polynomial.legendre.Legendre.basis(j)(x)
    return math.sqrt(2 * j + 1) * 0.5 * np.mean(np.abs(P)) * 2.0


def _brute_min(u, t):
    """argmin_v 0.5 (v - u)^2 + t |v| by grid search around u (resolution 1e-7 |u|)."""
    if u == 0.0:
        return 0.0
    cost = lambda v: 0.5 * (v - u) ** 2 + t * np.abs(v)
    lo, hi = min(0.0, u), max(0.0, u)
    for _ in range(4):
        v = np.linspace(lo, hi, 2001)
        c = cost(v)
        i = int(np.argmin(c))
        span = (hi - lo) / 200
        lo, hi = v[max(i - 1, 0)] - span, v[min(i + 1, 2000)] + span
    # v = 0 (the kink of the penalty) is a candidate of its own
    return 0.0 if cost(0.0) <= c[i] else v[i]


def _penalties(Np, M, a1, a2):
    lx = np.array([_l1_dense(j) for j in range(Np)])
    lz = np.array([_l1_dense(k) for k in range(M)])
    # (a Legendre term is an eigenfunction of L_i: L_i multiplies it by -j(j+1))
    return np.array([[(a1 * j * (j + 1) + a2 * k * (k + 1)) * lx[j] * lz[k] for j in range(Np)] for k in range(M)])


def _setup(p=3, order=4):
    cfg = dict(inputs.small(inputs.BURGERS, 2), p=p, gpc_order=order, nq1d=order + 3, filter="lasso",
               sensor="always")
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    return prob, T, R


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_filter_is_brute_force_minimiser_with_purpose_strengths(seed):
    prob, T, R = _setup()
    Np, M = T.n, R.M
    rng = np.random.default_rng(seed)
    ut = rng.standard_normal((1, M, 1, Np)) * np.exp(-0.4 * (np.arange(M)[None, :, None, None]
                                                             + np.arange(Np)[None, None, None, :]))
    got = ost.lasso_modal(prob, T, R, ut)[0, :, 0, :]
    u = ut[0, :, 0, :]

    # smallest a1 (a2) that zeroes the (Np-1, 0) ((0, Nc)) coefficient of the brute-force minimiser
    def zeroed(a1, a2, kk, jj):
        t = _penalties(Np, M, a1, a2)
        return _brute_min(u[kk, jj], t[kk, jj]) == 0.0
    def bisect(pred):
        lo, hi = 0.0, 1.0
        while not pred(hi):
            hi *= 2
            assert hi < 1e12
        for _ in range(40):
            mid = 0.5 * (lo + hi)
            lo, hi = (lo, mid) if pred(mid) else (mid, hi)
        return hi
    a1 = bisect(lambda a: zeroed(a, 0.0, 0, Np - 1))
    a2 = bisect(lambda a: zeroed(0.0, a, M - 1, 0))
    t = _penalties(Np, M, a1, a2)
    ref = np.array([[_brute_min(u[k, j], t[k, j]) for j in range(Np)] for k in range(M)])
    scale = np.abs(u).max()
    assert np.allclose(got, ref, rtol=0, atol=2e-6 * scale)
    assert got[0, Np - 1] == 0.0 or abs(got[0, Np - 1]) < 1e-15 * scale
    assert got[M - 1, 0] == 0.0 or abs(got[M - 1, 0]) < 1e-15 * scale


def test_invariants():
    prob, T, R = _setup(p=4, order=6)
    rng = np.random.default_rng(5)
    ut = rng.standard_normal((1, R.M, 40, T.n))
    once = ost.lasso_modal(prob, T, R, ut)
    assert np.array_equal(once[:, 0, :, 0], ut[:, 0, :, 0])          # the mean
    assert np.all(np.abs(once) <= np.abs(ut))                          # no growth
    assert np.all(once * ut >= 0.0)                                    # no sign change
    twice = ost.lasso_modal(prob, T, R, once)
    assert np.allclose(twice, once, rtol=0, atol=1e-15 * np.abs(ut).max())


def test_zero_coefficients_and_zero_state():
    prob, T, R = _setup()
    ut = np.zeros((1, R.M, 3, T.n))
    assert np.array_equal(ost.lasso_modal(prob, T, R, ut), ut)
    ut[0, 0, :, 0] = 2.0        # only the mean: untouched
    ut[0, 2, 1, 1] = 0.5        # top coefficients zero: no penalty, untouched
    assert np.array_equal(ost.lasso_modal(prob, T, R, ut), ut)


def test_step_with_lasso_filter_conserves_the_mean():
    cfg = dict(inputs.small(inputs.BURGERS, 16), filter="lasso", sensor="always")
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    from oracle.initial import project_initial
    u = project_initial(prob, cfg["ic"], (T, R))
    u = u + inputs.fuzz_scalar(R.M, prob.E, T.n, 3)
    uf, flags = ost.sensor_filter(prob, T, R, u, 1e-3)
    assert flags.all()
    mean = lambda v: np.einsum("ej,j->e", v[0, 0], T.w / 2.0)
    assert np.allclose(mean(uf), mean(u), rtol=0, atol=1e-15)


def test_lasso_scope():
    cfg = dict(inputs.small(inputs.SHOCK_VORTEX, 4, 2), filter="lasso")
    prob = Problem.from_config(cfg)
    T, R = build_tables(prob)
    with pytest.raises(ValueError):
        ost.lasso_norms(prob, T, R)
    bcfg = dict(inputs.small(inputs.BURGERS, 4), filter="lasso")
    bprob = Problem.from_config(bcfg)
    bT, bR = build_tables(bprob)
    u = np.zeros((1, bR.M, bprob.E, bT.n))
    with pytest.raises(ValueError):
        oadj.rhs_vjp(bprob, bT, bR, u, u)

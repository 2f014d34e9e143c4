"""Pins of the oracle's triangle path (Sec. 3.1 reference triangle, Sec. 3.5
correction fields) against closed forms, an independent construction of the
correction fields, the DG weak form, exactness and convergence."""

import math

import numpy as np
import pytest

from oracle import tri
from oracle.problem import Problem
from oracle.stepper import cfl_dt, step
from oracle.tables import build_random_tables, gauss_legendre, lagrange_values
from paper_2112_05946_amd import inputs

GAMMA = 1.4


def _monomials(p, r, s):
    return [(i, j, r ** i * s ** j) for i, j in tri.monomial_exponents(p)]


def test_duffy_rule_exact_on_monomials():
    """int_T (1+r)^a (1+s)^b = 2^(a+b+2) a! b! / (a+b+2)! (the simplex integral)."""
    n = 6
    r, s, w = tri.duffy_rule(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = 2.0 ** (a + b + 2) * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.dot(w, (1 + r) ** a * (1 + s) ** b) / exact - 1.0) < 1e-13, (a, b)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_basis_orthonormal_and_graded(p):
    r, s, w = tri.duffy_rule(p + 4)
    P = tri.basis_eval(p, r, s)
    G = 0.5 * (P * w[:, None]).T @ P
    assert np.max(np.abs(G - np.eye(len(G)))) < 1e-12
    _, _, deg = tri.orthonormal_basis(p)
    # a mode of degree d is orthogonal to every monomial of lower degree
    for m in range(P.shape[1]):
        for i, j, mono in _monomials(p, r, s):
            if i + j < deg[m]:
                assert abs(np.dot(w, P[:, m] * mono)) < 1e-12
    # psi_0 = 1
    assert np.max(np.abs(P[:, 0] - 1.0)) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_solution_points(p):
    r, s = tri.solution_points(p)
    n = (p + 1) * (p + 2) // 2
    assert len(r) == n
    assert np.all(r >= -1 - 1e-14) and np.all(s >= -1 - 1e-14) and np.all(r + s <= 1e-14)
    # on the bottom edge (s = -1) the nodes are the 1D LGL nodes
    lgl = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real) if p > 1 else np.zeros(0)
    edge = np.sort(r[np.abs(s + 1) < 1e-13])
    assert np.allclose(edge, np.concatenate(([-1.0], lgl, [1.0])), atol=1e-14)
    # the set is invariant under the symmetries of the triangle (permutations of
    # the barycentric coordinates)
    lam = np.stack([-(r + s) / 2, (r + 1) / 2, (s + 1) / 2], axis=1)
    key = lambda L: sorted(tuple(np.round(x, 12)) for x in L)
    for perm in ((1, 0, 2), (0, 2, 1), (2, 1, 0), (1, 2, 0), (2, 0, 1)):
        assert key(lam[:, perm]) == key(lam)
    if p <= 2:
        # equispaced lattice
        lat = [(-1 + 2 * a / p, -1 + 2 * b / p) for b in range(p + 1) for a in range(p + 1 - b)]
        assert np.allclose(np.stack([r, s], 1), np.array(lat), atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_derivative_and_face_interpolation_exact(p):
    T = tri.build_tri_tables(p)
    for i, j, _ in _monomials(p, T.r, T.s):
        f = T.r ** i * T.s ** j
        fr = i * T.r ** max(i - 1, 0) * T.s ** j if i else 0 * T.r
        fs = j * T.r ** i * T.s ** max(j - 1, 0) if j else 0 * T.r
        assert np.max(np.abs(T.Dr @ f - fr)) < 1e-11
        assert np.max(np.abs(T.Ds @ f - fs)) < 1e-11
        for face in range(3):
            rr, ss = tri.face_param(face, T.tq)
            assert np.max(np.abs(T.Lf[face] @ f - rr ** i * ss ** j)) < 1e-12
    # element mean = (1/2) int_T
    rq, sq, wq = tri.duffy_rule(p + 2)
    for i, j, _ in _monomials(p, T.r, T.s):
        assert abs(T.mean_w @ (T.r ** i * T.s ** j) - 0.5 * np.dot(wq, rq ** i * sq ** j)) < 1e-13


def _raviart_thomas_correction_divergence(p, r_eval, s_eval):
    """Independent construction of the correction fields: h_{f,k} in the
    Raviart-Thomas space RT_p = (P_p)^2 + (r, s) P~_p (P~_p homogeneous of degree p)
    with normal component (reference unit normal) equal to the face's Lagrange
    function l_k on face f and 0 on the other faces, and vanishing moments
    against (P_{p-1})^2 (what makes the correction DG).  Returns div h at the
    given points and the normal components at every flux point."""
    exps = tri.monomial_exponents(p)
    hom = [(p - j, j) for j in range(p + 1)]
    nP = len(exps)
    nU = 2 * nP + len(hom)

    def field(rr, ss):
        """Basis fields of RT_p at points: (hx, hy) of shape (len, nU) and div (len, nU)."""
        rr, ss = np.atleast_1d(rr), np.atleast_1d(ss)
        hx = np.zeros((len(rr), nU))
        hy = np.zeros((len(rr), nU))
        dv = np.zeros((len(rr), nU))
        for m, (i, j) in enumerate(exps):
            mono = rr ** i * ss ** j
            hx[:, m] = mono
            hy[:, nP + m] = mono
            dv[:, m] = i * rr ** max(i - 1, 0) * ss ** j if i else 0.0
            dv[:, nP + m] = j * rr ** i * ss ** max(j - 1, 0) if j else 0.0
        for m, (i, j) in enumerate(hom):
            mono = rr ** i * ss ** j
            hx[:, 2 * nP + m] = rr * mono
            hy[:, 2 * nP + m] = ss * mono
            dv[:, 2 * nP + m] = (i + j + 2) * mono    # div((r, s) m) = 2 m + (r d_r + s d_s) m
        return hx, hy, dv

    normals = ((0.0, -1.0), (1 / math.sqrt(2), 1 / math.sqrt(2)), (-1.0, 0.0))
    tq, _ = gauss_legendre(p + 1)
    rows = []
    for f in range(3):
        rr, ss = tri.face_param(f, tq)
        hx, hy, _ = field(rr, ss)
        rows.append(normals[f][0] * hx + normals[f][1] * hy)
    Nrm = np.concatenate(rows)                                  # (3 (p+1), nU)
    rq, sq, wq = tri.duffy_rule(p + 3)
    hx, hy, _ = field(rq, sq)
    mom = []
    for i, j in tri.monomial_exponents(p - 1) if p >= 1 else []:
        v = rq ** i * sq ** j
        mom.append((hx * (wq * v)[:, None]).sum(0))
        mom.append((hy * (wq * v)[:, None]).sum(0))
    A = np.concatenate([Nrm, np.array(mom).reshape(-1, nU)])
    assert A.shape == (nU, nU)
    rhs = np.zeros((nU, 3 * (p + 1)))
    rhs[: 3 * (p + 1)] = np.eye(3 * (p + 1))
    coef = np.linalg.solve(A, rhs)                               # one column per (f, k)
    _, _, dv = field(r_eval, s_eval)
    return (dv @ coef).reshape(len(r_eval), 3, p + 1), Nrm @ coef


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_correction_divergence_equals_raviart_thomas_fields(p):
    """The lifting used by the oracle equals the divergence of the vector
    correction fields built from the constraint of Sec. 3.5 (h_{f,k} . n = 1 at
    its own flux point, 0 at the others) in RT_p with the DG moment conditions."""
    T = tri.build_tri_tables(p)
    divh, normal_traces = _raviart_thomas_correction_divergence(p, T.r, T.s)
    assert np.max(np.abs(normal_traces - np.eye(3 * (p + 1)))) < 1e-12
    assert np.max(np.abs(divh - T.divh)) < 1e-10 * np.max(np.abs(T.divh))


def _tri_problem(mesh, p=2, gpc_order=2, nq1d=3, rdim=1, **kw):
    return Problem(equation="euler2d", nx=1, ny=1, p=p, gpc_order=gpc_order, nq1d=nq1d, rdim=rdim,
                   element="tri", mesh=mesh, gamma=GAMMA, **kw)


def _cons(rho, u, v, pr):
    return np.stack([rho, rho * u, rho * v, pr / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


def _state_from_nodal(prob, R, Unodal):
    """Project nodal values U[s, q, e, j] onto the chaos."""
    return np.einsum("kq,sqej->skej", R.PW, Unodal)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_free_stream_preserved_on_perturbed_mesh(p):
    mesh = inputs.tri_mesh_rectangle(4, 3, perturb=0.25, seed=3)
    prob = _tri_problem(mesh, p=p)
    T = tri.build_tri_tables(p)
    R = build_random_tables(prob.gpc_order, 1, prob.nq1d)
    z = R.z[:, 0]
    E, N = prob.E, T.n
    U = _cons(np.ones((R.Nq, E, N)) * (1 + 0.1 * z)[:, None, None], 0.7 + 0.05 * z[:, None, None],
              -0.3 + 0 * z[:, None, None], 1.0 + 0 * z[:, None, None])
    u = _state_from_nodal(prob, R, U)
    res = tri.rhs_tri(prob, T, R, u)
    assert np.max(np.abs(res)) < 1e-12


@pytest.mark.parametrize("flux", ["rusanov", "hll"])
def test_conservation_periodic(flux):
    mesh = inputs.tri_mesh_rectangle(5, 4, perturb=0.2, seed=5)
    prob = _tri_problem(mesh, p=3, flux=flux)
    T = tri.build_tri_tables(3)
    R = build_random_tables(prob.gpc_order, 1, prob.nq1d)
    u = inputs.fuzz_euler(2, R.M, prob.E, T.n, seed=11)
    res = tri.rhs_tri(prob, T, R, u)
    G = tri.geometry(mesh["xy"])
    tot = np.einsum("skej,j,e->sk", res, T.mean_w, 2 * G.det)
    scale = np.einsum("skej,j,e->sk", np.abs(res), np.abs(T.mean_w), 2 * G.det)
    assert np.max(np.abs(tot) / scale) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_density_wave_exact_on_interior_elements(p):
    """Constant velocity and pressure, density a global polynomial of degree p:
    the flux is polynomial of degree p and continuous, so the interactive flux
    equals it and the right-hand side is -(u rho_x + v rho_y) (1, u, v, |v|^2/2)
    exactly, on every element whose neighbours are not periodic images."""
    mesh = inputs.tri_mesh_rectangle(5, 5, perturb=0.2, seed=2)
    prob = _tri_problem(mesh, p=p)
    T = tri.build_tri_tables(p)
    R = build_random_tables(prob.gpc_order, 1, prob.nq1d)
    X, Y = tri.solution_point_coords_tri(prob, T)
    z = R.z[:, 0][:, None, None]
    rho = 1.0 + 0.3 * X ** p - 0.2 * X * Y ** (p - 1) + 0.1 * Y
    drx = 0.3 * p * X ** (p - 1) - 0.2 * Y ** (p - 1)
    dry = -0.2 * (p - 1) * X * Y ** max(p - 2, 0) + 0.1
    uu, vv = 0.8 + 0.1 * z, -0.4 + 0 * z
    U = _cons(np.broadcast_to(rho, (R.Nq,) + rho.shape), uu + 0 * rho, vv + 0 * rho, 1.0 + 0 * rho)
    u = _state_from_nodal(prob, R, U)
    res = tri.rhs_tri(prob, T, R, u)
    adv = -(uu * drx + vv * dry)
    exact = np.stack([adv, adv * uu, adv * vv, adv * 0.5 * (uu * uu + vv * vv)])
    exact = np.einsum("kq,sqej->skej", R.PW, exact)
    xy = mesh["xy"]
    inside = np.all((xy[:, :, 0] > 1e-9) & (xy[:, :, 0] < 1 - 1e-9) & (xy[:, :, 1] > 1e-9) & (xy[:, :, 1] < 1 - 1e-9),
                    axis=1)
    nb = mesh["nbr"]
    keep = inside & np.all(inside[nb], axis=1)
    assert keep.sum() >= 4
    assert np.max(np.abs(res[:, :, keep] - exact[:, :, keep])) < 1e-11


def _weak_form_rhs(prob, T, R, u):
    """Nodal DG in weak form, assembled per element with the collapsed-coordinate
    quadrature: M du/dt = int grad(l_i) . F^D - sum_faces int l_i F* . n ds, F^D the
    interpolant of the projected flux, F* (Lax-Friedrichs per node, projected) at
    the flux points and integrated with their Gauss weights."""
    p = T.p
    G = tri.geometry(prob.mesh["xy"])
    nbr, nbf = prob.mesh["nbr"], prob.mesh["nbr_face"]
    rq, sq, wq = tri.duffy_rule(p + 2)
    Pq = tri.basis_eval(p, rq, sq)
    gr, gs = tri.basis_grad(p, rq, sq)
    Lq = Pq @ T.Vinv                          # l_i at the quadrature points
    Lr, Ls = gr @ T.Vinv, gs @ T.Vinv
    Mref = (Lq * wq[:, None]).T @ Lq
    U = np.einsum("kq,skej->sqej", R.Phi, u)
    rho, mx, my, En = U
    pr = (GAMMA - 1) * (En - 0.5 * (mx * mx + my * my) / rho)
    F = np.stack([mx, mx * mx / rho + pr, mx * my / rho, (En + pr) * mx / rho])
    Gf = np.stack([my, mx * my / rho, my * my / rho + pr, (En + pr) * my / rho])
    fh = np.einsum("kq,sqej->skej", R.PW, F)
    gh = np.einsum("kq,sqej->skej", R.PW, Gf)
    out = np.zeros_like(u)
    Lface = [lagrange_values(T.tq, T.tq)]      # identity: F* known at the flux points
    del Lface
    for e in range(prob.E):
        fq = np.einsum("qi,ski->skq", Lq, fh[:, :, e])
        gq = np.einsum("qi,ski->skq", Lq, gh[:, :, e])
        gx = Lr * G.rx[e] + Ls * G.sx[e]      # d l_i / dx at the quadrature points
        gy = Lr * G.ry[e] + Ls * G.sy[e]
        vol = np.einsum("q,qi,skq->ski", wq, gx, fq) + np.einsum("q,qi,skq->ski", wq, gy, gq)
        vol = vol * G.det[e]
        surf = np.zeros_like(vol)
        for f in range(3):
            nx, ny = G.nx[e, f], G.ny[e, f]
            UL = np.einsum("ki,sqi->sqk", T.Lf[f], U[:, :, e])
            if nbr[e, f] >= 0:
                UR = np.einsum("ki,sqi->sqk", T.Lf[nbf[e, f]], U[:, :, nbr[e, f]])[:, :, ::-1]
            else:
                raise AssertionError("periodic mesh expected")
            def nf(W):
                r_, m1, m2, e_ = W
                p_ = (GAMMA - 1) * (e_ - 0.5 * (m1 * m1 + m2 * m2) / r_)
                vn = (m1 * nx + m2 * ny) / r_
                return np.stack([r_ * vn, m1 * vn + p_ * nx, m2 * vn + p_ * ny, (e_ + p_) * vn]), \
                    np.abs(vn) + np.sqrt(GAMMA * p_ / r_)
            FL, aL = nf(UL)
            FR, aR = nf(UR)
            Fs = 0.5 * (FL + FR) - 0.5 * np.maximum(aL, aR) * (UR - UL)
            Fsh = np.einsum("kq,sql->skl", R.PW, Fs)
            surf += np.einsum("l,li,skl->ski", 0.5 * G.flen[e, f] * T.wq, T.Lf[f], Fsh)
        out[:, :, e] = np.linalg.solve(Mref * G.det[e], (vol - surf).transpose(2, 0, 1).reshape(T.n, -1)) \
            .reshape(T.n, u.shape[0], u.shape[1]).transpose(1, 2, 0)
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rhs_equals_dg_weak_form(p):
    mesh = inputs.tri_mesh_rectangle(3, 3, perturb=0.25, seed=9)
    prob = _tri_problem(mesh, p=p)
    T = tri.build_tri_tables(p)
    R = build_random_tables(prob.gpc_order, 1, prob.nq1d)
    u = inputs.fuzz_euler(2, R.M, prob.E, T.n, seed=4)
    a = tri.rhs_tri(prob, T, R, u)
    b = _weak_form_rhs(prob, T, R, u)
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(b))


def _density_wave_mean_error(p, n, t_end=0.05):
    mesh = inputs.tri_mesh_rectangle(n, n, perturb=0.15, seed=7)
    prob = _tri_problem(mesh, p=p, gpc_order=3, nq1d=4, cfl=0.1)
    T = tri.build_tri_tables(p)
    R = build_random_tables(prob.gpc_order, 1, prob.nq1d)
    X, Y = tri.solution_point_coords_tri(prob, T)
    z = R.z[:, 0][:, None, None]
    uu = 1.0 + 0.1 * z
    rho0 = lambda x, y: 1.0 + 0.2 * np.sin(2 * np.pi * (x + y))
    U = _cons(rho0(X, Y)[None] + 0 * z, uu + 0 * X, 0.5 + 0 * X, 1.0 + 0 * X)
    u = _state_from_nodal(prob, R, U)
    tables = (T, R)
    dt = cfl_dt(prob, T, R, u)
    nsteps = int(math.ceil(t_end / dt))
    dt = t_end / nsteps
    for _ in range(nsteps):
        u, _, _ = step(prob, u, dt, tables)
    # L2 over the domain: the solution interpolated to a collapsed-coordinate rule
    # in every element, against the exact mean of rho over z ~ U(-1, 1) (24-point rule)
    rq, sq, wq = tri.duffy_rule(p + 4)
    Lq = tri.basis_eval(p, rq, sq) @ T.Vinv
    xy = mesh["xy"]
    l1, l2, l3 = -(rq + sq) / 2, (rq + 1) / 2, (sq + 1) / 2
    Xq = l1[None] * xy[:, 0, 0:1] + l2[None] * xy[:, 1, 0:1] + l3[None] * xy[:, 2, 0:1]
    Yq = l1[None] * xy[:, 0, 1:2] + l2[None] * xy[:, 1, 1:2] + l3[None] * xy[:, 2, 1:2]
    zg, wg = gauss_legendre(24)
    mean = sum(0.5 * w * rho0(Xq - (1 + 0.1 * zz) * t_end, Yq - 0.5 * t_end) for zz, w in zip(zg, wg))
    G = tri.geometry(xy)
    e = u[0, 0] @ Lq.T - mean
    return math.sqrt(np.einsum("eq,q,e->", e * e, wq, G.det))


@pytest.mark.parametrize("p", [1, 2])
def test_density_wave_convergence_order(p):
    errs = [_density_wave_mean_error(p, n) for n in (6, 12)]
    order = math.log2(errs[0] / errs[1])
    assert abs(order - (p + 1)) < 0.4, (errs, order)


# ----------------------------------------------------------------------------
# discontinuity sensor, modal filters and positivity limiter on triangles
# ----------------------------------------------------------------------------

def _mono_poly(p, seed):
    """A random polynomial of total degree <= p as (coefficients, exponents)."""
    rng = np.random.default_rng(seed)
    ex = tri.monomial_exponents(p)
    return rng.normal(size=len(ex)), ex


def test_tri_modal_coefficients_are_orthonormal_projections():
    """Nodal -> modal on triangles equals (1/2) int_T u psi_m of the polynomial itself,
    integrated by the collapsed rule (no Vandermonde inverse on this side)."""
    from oracle.stabilize import to_spatial_modal
    for p in (1, 2, 3, 4):
        mesh = inputs.tri_mesh_rectangle(1, 1)
        prob = _tri_problem(mesh, p=p)
        T = tri.build_tri_tables(p)
        c, ex = _mono_poly(p, p)
        f = lambda r, s: sum(ci * r ** i * s ** j for ci, (i, j) in zip(c, ex))
        u = np.zeros((4, 1, 2, T.n))
        u[0, 0, 0] = f(T.r, T.s)
        ut = to_spatial_modal(prob, T, u)[0, 0, 0]
        rq, sq, wq = tri.duffy_rule(p + 3)
        ref = 0.5 * (tri.basis_eval(p, rq, sq) * (wq * f(rq, sq))[:, None]).sum(axis=0)
        assert np.max(np.abs(ut - ref)) < 1e-12


@pytest.mark.parametrize("filt", ["exp", "l2"])
def test_tri_filter_acts_mode_by_mode(filt):
    """A state made of one orthonormal mode psi_m Phi_k (any state variable) comes back
    times the filter factor of its total degree d and chaos degree |k|:
    exp(-alpha dt ((d/p)^s + (|k|/N_c)^s)) or 1 / (1 + d^2 (d+1)^2 / (eps1 p^2 (p+1)^2)
    + |k|^2 (|k|+1)^2 / (eps2 N_c^2 (N_c+1)^2)); the mean mode is untouched."""
    from oracle.stabilize import sensor_filter
    p, Nc = 3, 3
    mesh = inputs.tri_mesh_rectangle(1, 1)
    prob = _tri_problem(mesh, p=p, gpc_order=Nc, nq1d=5, filter=filt, sensor="always", alpha=36.0, s=3.0,
                        eps1=0.6, eps2=0.8)
    T = tri.build_tri_tables(p)
    R = build_random_tables(Nc, 1, 5)
    dt = 2e-3
    _, _, deg = tri.orthonormal_basis(p)
    for m in range(T.n):
        for k in range(R.M):
            u = np.zeros((4, R.M, 2, T.n))
            u[2, k, 1] = T.V[:, m]          # psi_m at the solution points
            out, flags = sensor_filter(prob, T, R, u, dt)
            d = deg[m]
            if filt == "exp":
                lam = math.exp(-36.0 * dt * ((d / p) ** 3 + (k / Nc) ** 3))
            else:
                lam = 1.0 / (1.0 + d * d * (d + 1) ** 2 / (0.6 * p * p * (p + 1) ** 2)
                             + k * k * (k + 1) ** 2 / (0.8 * Nc * Nc * (Nc + 1) ** 2))
            assert np.max(np.abs(out - lam * u)) < 1e-13, (m, k)
            if d == 0 and k == 0:
                assert abs(lam - 1.0) < 1e-15


def test_tri_sensor_flags_top_degree_content():
    """S_e = energy of the modes of total degree p or chaos degree N_c (state 0) over the total."""
    from oracle.stabilize import sensor_flags
    p = 3
    mesh = inputs.tri_mesh_rectangle(1, 1)
    prob = _tri_problem(mesh, p=p, gpc_order=2, nq1d=3, filter="exp", sensor="detector", s0=-3.0, kappa=1.0)
    T = tri.build_tri_tables(p)
    R = build_random_tables(2, 1, 3)
    _, _, deg = tri.orthonormal_basis(p)
    low = [m for m in range(T.n) if deg[m] < p]
    top = [m for m in range(T.n) if deg[m] == p]
    u = np.zeros((4, R.M, 2, T.n))
    u[0, 0, 0] = T.V[:, low] @ np.linspace(1.0, 0.2, len(low))   # smooth: no top-degree content
    u[0, 1, 0] = 0.3 * T.V[:, low[1]]
    u[0, 0, 1] = T.V[:, low] @ np.linspace(1.0, 0.2, len(low)) + 0.5 * T.V[:, top[0]]
    flags = sensor_flags(prob, T, R, u)
    assert not flags[0] and flags[1]


def test_tri_limiter_restores_positivity_and_keeps_means():
    from oracle.stabilize import element_mean, limit
    mesh = inputs.tri_mesh_rectangle(5, 4, perturb=0.2, seed=8)
    prob = _tri_problem(mesh, p=3, gpc_order=3, nq1d=4, limiter=True)
    T = tri.build_tri_tables(3)
    R = build_random_tables(3, 1, 4)
    u = inputs.fuzz_euler(2, R.M, prob.E, T.n, seed=21, vacuum_frac=0.3)
    out, flags = limit(prob, T, R, u)
    assert flags.sum() >= 6
    m0, m1 = element_mean(prob, T, u), element_mean(prob, T, out)
    assert np.max(np.abs(m1 - m0)) < 1e-14
    assert np.array_equal(out[:, :, ~flags], u[:, :, ~flags])
    # density and pressure at solution and flux points, every node: independent
    # evaluation through the polynomials (orthonormal basis at the points)
    def pts(v):
        U = np.einsum("kq,skej->sqej", R.Phi, v)
        fr, fs = zip(*[tri.face_param(f, T.tq) for f in range(3)])
        rr = np.concatenate([T.r] + list(fr))
        ss = np.concatenate([T.s] + list(fs))
        L = tri.basis_eval(3, rr, ss) @ T.Vinv
        return np.einsum("pj,sqej->sqep", L, U)
    P = pts(out)
    rho = P[0]
    pr = (GAMMA - 1) * (P[3] - 0.5 * (P[1] ** 2 + P[2] ** 2) / P[0])
    pbar = (GAMMA - 1) * (m0[3] - 0.5 * (m0[1] ** 2 + m0[2] ** 2) / m0[0])
    eps = np.minimum(1e-8, np.minimum(m0[0], pbar))
    lo = np.minimum(rho.min(axis=(0, 2)), pr.min(axis=(0, 2)))
    assert np.all(lo[flags] >= eps[flags] * (1 - 1e-6) - 1e-13)
    # tight: each limited element touches eps at some point and node
    assert np.all(np.abs(lo[flags] - eps[flags]) < 1e-9)

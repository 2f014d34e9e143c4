"""Workload definitions and seeded synthetic inputs.

This module is shared by the HIP path and by the CPU oracle.  It holds only
problem statements (sizes, parameters, analytic initial data) and seeded
random states; it contains no part of the FR-SG method (no quadrature, no
basis, no projection, no flux).  Each side evaluates initial data at its own
solution points and random nodes and projects with its own tables.

Workloads are shaped like the paper's experiments (Sec. 5):

* ``advection_sine``      stochastic linear advection u_t + u_x = 0 (Sec. 5.1)
                          with u0 = sin(2 pi (x + 0.1 z)) on periodic [0, 1];
* ``burgers_sine``        inviscid Burgers f = u^2/2 (Sec. 5.2) with
                          u0 = 1 + 0.5 sin(pi x) + 0.2 z sin(pi x) on periodic [0, 2];
* ``sod_interface``       1D Euler Sod tube with uncertain interface
                          x0 = 0.5 + 0.05 z (Sec. 5.3, second case);
* ``wave_propagation``    the convergence study of Sec. 5.1 (Tables 1-3):
                          u_t + u_x = 0 on periodic [-1, 1] with
                          u0 = xi(z) sin(pi x), xi = 1 + 0.1 z ~ U(0.9, 1.1);
                          exact solution xi(z) sin(pi (x - t));
* ``shock_vortex``        2D Euler stationary Mach 1.1 normal shock at x = 0.5
                          and an isentropic vortex of strength 0.3 + 0.05 z1
                          centred at (0.25 + 0.02 z2, 0.5) (Sec. 5.4 setup with
                          two random dimensions).
"""

import math

import numpy as np

GAMMA = 1.4


def _cons1d(rho, u, p, gamma=GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _cons2d(rho, u, v, p, gamma=GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ----------------------------------------------------------------------------
# shock-vortex problem data (Sec. 5.4, Rankine-Hugoniot + isentropic vortex)
# ----------------------------------------------------------------------------

SV_MACH = 1.1
SV_XSHOCK = 0.5
SV_MU = 0.204
SV_RC = 0.05


def shock_states(mach=SV_MACH, gamma=GAMMA):
    """Upstream (x < shock) and downstream primitive states (rho, u, v, p)."""
    rho1, p1 = 1.0, 1.0
    u1 = mach * math.sqrt(gamma * p1 / rho1)
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u2 = u1 * rho1 / rho2
    return (rho1, u1, 0.0, p1), (rho2, u2, 0.0, p2)


def shock_vortex_ic(x, y, z1, z2, gamma=GAMMA):
    up, down = shock_states(gamma=gamma)
    zeta = 0.3 + 0.05 * z1
    xc = 0.25 + 0.02 * z2
    yc = 0.5
    upstream = x < SV_XSHOCK
    rho0 = np.where(upstream, up[0], down[0])
    u0 = np.where(upstream, up[1], down[1])
    p0 = np.where(upstream, up[3], down[3])
    dx, dy = x - xc, y - yc
    r = np.sqrt(dx * dx + dy * dy)
    eta = r / SV_RC
    # (du, dv) = zeta eta exp(mu (1 - eta^2)) (sin theta, -cos theta)
    amp = zeta * eta * np.exp(SV_MU * (1.0 - eta * eta))
    with np.errstate(invalid="ignore", divide="ignore"):
        st = np.where(r > 0, dy / np.where(r > 0, r, 1.0), 0.0)
        ct = np.where(r > 0, dx / np.where(r > 0, r, 1.0), 0.0)
    du, dv = amp * st, -amp * ct
    dT = -(gamma - 1.0) * zeta * zeta / (4.0 * SV_MU * gamma) * np.exp(2.0 * SV_MU * (1.0 - eta * eta))
    T0 = p0 / rho0
    T = T0 + dT
    # isentropic: p / rho^gamma unchanged  =>  rho = rho0 (T/T0)^(1/(gamma-1))
    rho = rho0 * (T / T0) ** (1.0 / (gamma - 1.0))
    p = rho * T
    return _cons2d(rho, u0 + du, dv, p, gamma)


def vortex_ic(x, y, z1, z2, gamma=GAMMA):
    """The isentropic vortex of Sec. 5.4 (strength 0.3 + 0.05 z1, mu = 0.204,
    r_c = 0.05) centred at (0.5 + 0.02 z2, 0.5) in the uniform Mach 1.1 upstream
    state of the shock-vortex problem, without the shock (periodic [0, 1]^2)."""
    up, _ = shock_states(gamma=gamma)
    zeta = 0.3 + 0.05 * z1
    dx, dy = x - (0.5 + 0.02 * z2), y - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    eta = r / SV_RC
    amp = zeta * eta * np.exp(SV_MU * (1.0 - eta * eta))
    with np.errstate(invalid="ignore", divide="ignore"):
        st = np.where(r > 0, dy / np.where(r > 0, r, 1.0), 0.0)
        ct = np.where(r > 0, dx / np.where(r > 0, r, 1.0), 0.0)
    dT = -(gamma - 1.0) * zeta * zeta / (4.0 * SV_MU * gamma) * np.exp(2.0 * SV_MU * (1.0 - eta * eta))
    T0 = up[3] / up[0]
    T = T0 + dT
    rho = up[0] * (T / T0) ** (1.0 / (gamma - 1.0))
    return _cons2d(rho, up[1] + amp * st, -amp * ct, rho * T, gamma)


# isentropic vortex carried by a uniform flow through the periodic rectangle
# [0, 2] x [0, 1] (the vortex form of Sec. 5.4 with a wider, faster-decaying
# core, so the rectangle is periodic to ~1e-6): core radius 0.13, mu = 1,
# strength 0.3, free stream rho = p = 1, velocity (1 + 0.001 z1, 0.5).  The
# exact solution at time t is the initial field translated by the free-stream
# velocity of each random node.
VC_RC = 0.13
VC_MU = 1.0
VC_ZETA = 0.3
VC_U = (1.0, 0.5)
VC_DELTA = 0.001


def vortex_convection_exact(x, y, z1, t, gamma=GAMMA):
    """Conservative state of the convected vortex at time t (points x, y; random z1)."""
    ui = VC_U[0] + VC_DELTA * z1
    vi = VC_U[1] + 0.0 * z1
    dx = (x - (1.0 + ui * t) + 1.0) % 2.0 - 1.0
    dy = (y - (0.5 + vi * t) + 0.5) % 1.0 - 0.5
    eta2 = (dx * dx + dy * dy) / (VC_RC * VC_RC)
    amp = VC_ZETA * np.exp(VC_MU * (1.0 - eta2)) / VC_RC
    T = 1.0 - (gamma - 1.0) * VC_ZETA ** 2 / (4.0 * VC_MU * gamma) * np.exp(2.0 * VC_MU * (1.0 - eta2))
    rho = T ** (1.0 / (gamma - 1.0))
    return _cons2d(rho, ui + amp * dy, vi - amp * dx, rho * T, gamma)


def initial_condition(name, x, y, z, gamma=GAMMA):
    """Conservative initial data at points x, y (same shape) and random z[..., rdim]."""
    z1 = z[..., 0]
    if name == "advection_sine":
        return np.sin(2.0 * np.pi * (x + 0.1 * z1))[None]
    if name == "wave_propagation":
        return ((1.0 + 0.1 * z1) * np.sin(np.pi * x))[None]
    if name == "burgers_sine":
        return (1.0 + 0.5 * np.sin(np.pi * x) + 0.2 * z1 * np.sin(np.pi * x))[None]
    if name == "sod_interface":
        left = x < 0.5 + 0.05 * z1
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        return _cons1d(rho, np.zeros_like(rho), p, gamma)
    if name == "tri_density_wave":
        # rho = 1 + 0.2 sin(2 pi (x + y)), velocity (1 + 0.1 z1, 0.5), p = 1
        rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x + y))
        return _cons2d(rho, 1.0 + 0.1 * z1, 0.5 + 0.0 * x, 1.0 + 0.0 * x, gamma)
    if name == "vortex_convection":
        return vortex_convection_exact(x, y, z1, 0.0, gamma)
    if name == "tri_vortex":
        z2 = z[..., 1] if z.shape[-1] > 1 else np.zeros_like(z1)
        return vortex_ic(x, y, z1, z2, gamma)
    if name == "shock_vortex":
        # one random dimension: only the vortex strength is uncertain
        z2 = z[..., 1] if z.shape[-1] > 1 else np.zeros_like(z1)
        return shock_vortex_ic(x, y, z1, z2, gamma)
    raise ValueError(name)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def _sod_bc():
    L = list(_cons1d(np.array(1.0), np.array(0.0), np.array(1.0))) + [0.0]
    R = list(_cons1d(np.array(0.125), np.array(0.0), np.array(0.1))) + [0.0]
    return [[float(v) for v in L], [float(v) for v in R], [0.0] * 4, [0.0] * 4]


def _sv_bc():
    up, _ = shock_states()
    st = [float(v) for v in _cons2d(*[np.array(c) for c in up])]
    return [st, [0.0] * 4, [0.0] * 4, [0.0] * 4]


ADVECTION = dict(
    name="advection_sine", equation="advection", ic="advection_sine",
    nx=64, xlo=0.0, xhi=1.0, p=2, gpc_order=4, nq1d=8, rdim=1,
    bc=["periodic"] * 4, adv_speed=1.0, filter="none", limiter=False,
    cfl=0.3, t_end=0.5)

BURGERS = dict(
    name="burgers_sine", equation="burgers", ic="burgers_sine",
    nx=1024, xlo=0.0, xhi=2.0, p=3, gpc_order=8, nq1d=16, rdim=1,
    bc=["periodic"] * 4, filter="exp", alpha=36.0, s=8.0,
    sensor="detector", s0=-2.0 * math.log10(3.0), kappa=4.0,
    limiter=False, cfl=0.3, t_end=1.0)

SOD = dict(
    name="sod_interface", equation="euler1d", ic="sod_interface",
    nx=2048, xlo=0.0, xhi=1.0, p=3, gpc_order=10, nq1d=24, rdim=1,
    bc=["dirichlet", "dirichlet", "periodic", "periodic"], bc_state=_sod_bc(),
    gamma=GAMMA, filter="l2", eps1=0.6, eps2=0.6,
    sensor="detector", s0=-3.0 * math.log10(3.0), kappa=4.0,
    limiter=True, cfl=0.3, t_end=0.2)

SHOCK_VORTEX = dict(
    name="shock_vortex", equation="euler2d", ic="shock_vortex",
    nx=256, ny=128, xlo=0.0, xhi=2.0, ylo=0.0, yhi=1.0,
    p=3, gpc_order=4, nq1d=5, rdim=2,
    bc=["dirichlet", "outflow", "reflect", "reflect"], bc_state=_sv_bc(),
    gamma=GAMMA, filter="l2", eps1=0.6, eps2=1.0,
    sensor="detector", s0=-3.0 * math.log10(3.0), kappa=4.0,
    limiter=True, cfl=0.3, t_end=0.3)

BURGERS_ADJOINT = dict(BURGERS, name="burgers_adjoint", nx=4096, n_steps=500, checkpoint_every=25)

# the Burgers and Sod workloads with the Lasso filter (Sec. 4.1.3) on every
# element in place of the detector-gated exponential and L2 filters
BURGERS_LASSO = dict(BURGERS, name="burgers_lasso", filter="lasso", sensor="always")
SOD_LASSO = dict(SOD, name="sod_lasso", filter="lasso", sensor="always")

# the Sod and shock-vortex workloads with the HLL interactive flux the paper
# uses for them (Tables 5, 6) in place of Lax-Friedrichs
SOD_HLL = dict(SOD, name="sod_hll", flux="hll")
SHOCK_VORTEX_HLL = dict(SHOCK_VORTEX, name="shock_vortex_hll", flux="hll")
# ... and with the Bogacki-Shampine integrator as well (the paper's settings in
# Tables 5 and 6), at the CFL step
SOD_HLL_BS3 = dict(SOD, name="sod_hll_bs3", flux="hll", integrator="bs3")
SHOCK_VORTEX_HLL_BS3 = dict(SHOCK_VORTEX, name="shock_vortex_hll_bs3", flux="hll", integrator="bs3")

# the convergence study of Sec. 5.1: Table 1's setup (N_c = 5, N_q = 9,
# Lax-Friedrichs, RK4, periodic, no filter) on 4..64 elements, measured at
# t = 2.  Its CFL number 0.1 is read as dt = 0.1 dx / |a|; with the CFL rule
# dt = cfl dx / ((p + 1) lambda_max) used here that is cfl = 0.1 (p + 1).
WAVE_DX = (0.5, 0.25, 0.125, 0.0625, 0.03125)
WAVE_T = 2.0


def wave_propagation(n_points, nx):
    """Table 1 setup with N_p = n_points solution points on nx elements."""
    return dict(
        name="wave_propagation", equation="advection", ic="wave_propagation",
        nx=nx, xlo=-1.0, xhi=1.0, p=n_points - 1, gpc_order=5, nq1d=9, rdim=1,
        bc=["periodic"] * 4, adv_speed=1.0, flux="rusanov", integrator="rk4",
        filter="none", limiter=False, cfl=0.1 * n_points, t_end=WAVE_T)


def wave_exact(x, t, z):
    """Exact solution of the wave-propagation problem at points x, time t, random z."""
    return (1.0 + 0.1 * z) * np.sin(np.pi * (x - t))


WAVE = wave_propagation(3, 64)


def tri_vortex(n, p=3, perturb=0.1, seed=1):
    """The vortex of Sec. 5.4 without the shock, advected through the periodic unit
    square on 2 n^2 perturbed triangles: FR degree p, two random dimensions with
    total-degree-4 chaos (15 modes) on 5 x 5 nodes, Lax-Friedrichs, SSP-RK3, CFL 0.3."""
    return dict(
        name="tri_vortex", equation="euler2d", ic="tri_vortex", element="tri",
        mesh=tri_mesh_rectangle(n, n, perturb=perturb, seed=seed), nx=1, ny=1,
        p=p, gpc_order=4, nq1d=5, rdim=2, bc=["outflow"] * 4, gamma=GAMMA,
        filter="none", limiter=False, cfl=0.3, t_end=0.1)


def tri_shock_vortex(n, p=3, perturb=0.1, seed=2):
    """The shock-vortex problem of Sec. 5.4 as set up on quadrilaterals (Mach 1.1 shock at
    x = 0.5, vortex, left Dirichlet, right outflow, top and bottom reflect, L2 filter
    switched by the detector, positivity limiter) on 2 (2n) n triangles of [0, 2] x [0, 1]
    (a seeded perturbation of a split 2n x n grid), FR degree p."""
    return dict(SHOCK_VORTEX, name="tri_shock_vortex", element="tri", nx=1, ny=1, p=p,
                mesh=tri_mesh_rectangle(2 * n, n, 0.0, 2.0, 0.0, 1.0, periodic=(False, False), perturb=perturb,
                                        seed=seed))


def tri_density_wave(n, p=2, perturb=0.15, seed=7, gpc_order=3, nq1d=4):
    """Density wave rho = 1 + 0.2 sin(2 pi (x + y)) carried by the velocity
    (1 + 0.1 z, 0.5) at unit pressure, periodic unit square, 2 n^2 perturbed
    triangles; exact solution rho(x - (1 + 0.1 z) t, y - t/2)."""
    return dict(
        name="tri_density_wave", equation="euler2d", ic="tri_density_wave", element="tri",
        mesh=tri_mesh_rectangle(n, n, perturb=perturb, seed=seed), nx=1, ny=1,
        p=p, gpc_order=gpc_order, nq1d=nq1d, rdim=1, bc=["outflow"] * 4, gamma=GAMMA,
        filter="none", limiter=False, cfl=0.1, t_end=0.05)

CONFIGS = {c["name"]: c for c in (ADVECTION, WAVE, BURGERS, SOD, SHOCK_VORTEX, BURGERS_ADJOINT, BURGERS_LASSO, SOD_LASSO,
                                  SOD_HLL, SHOCK_VORTEX_HLL, SOD_HLL_BS3, SHOCK_VORTEX_HLL_BS3)}


def vortex_convection(n, p, gpc_order=1, nq1d=2, cfl=0.15):
    """The convected vortex on n x n cells of 2 x 1 aspect ratio (dx = 2 dy), no filter or limiter."""
    return dict(name="vortex_convection", equation="euler2d", ic="vortex_convection", nx=n, ny=n, p=p,
                xlo=0.0, xhi=2.0, ylo=0.0, yhi=1.0, rdim=1, gpc_order=gpc_order, nq1d=nq1d, cfl=cfl,
                bc=["periodic"] * 4, filter="none", limiter=False)


def small(cfg, nx, ny=None, **kw):
    """Same problem on a smaller mesh (parity-test sizes)."""
    out = dict(cfg, nx=nx, **kw)
    if ny is not None:
        out["ny"] = ny
    return out


# ----------------------------------------------------------------------------
# triangle meshes (Sec. 3.1: straight-sided triangles, each the image of the
# isosceles right reference triangle)
# ----------------------------------------------------------------------------

def tri_mesh_rectangle(nx, ny, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, periodic=(True, True), perturb=0.0, seed=0):
    """Triangulation of [xlo, xhi] x [ylo, yhi]: nx x ny cells, each cut along its
    lower-right to upper-left diagonal into two counter-clockwise triangles.

    Cell (i, j) with corners A (lower left), B (lower right), C (upper right),
    D (upper left) gives element 2 (j nx + i) = (A, B, D) and element
    2 (j nx + i) + 1 = (C, D, B).  Face f of an element joins its vertices f and
    (f + 1) mod 3.  With perturb > 0 every vertex not on a non-periodic
    boundary moves by a seeded uniform offset of at most perturb times the cell
    size in each coordinate (the same offset for all periodic copies of a vertex).

    Returns dict(xy [E, 3, 2] vertex coordinates, nbr [E, 3] neighbour element
    across each face or -1 - side for a boundary face (side 0 x-lo, 1 x-hi,
    2 y-lo, 3 y-hi), nbr_face [E, 3] the neighbour's face index or -1).
    """
    dx, dy = (xhi - xlo) / nx, (yhi - ylo) / ny
    rng = np.random.default_rng(seed)
    off = rng.uniform(-perturb, perturb, (ny + 1, nx + 1, 2)) * np.array([dx, dy])
    px, py = periodic
    if px:
        off[:, nx] = off[:, 0]
    else:
        off[:, 0] = 0.0
        off[:, nx] = 0.0
    if py:
        off[ny, :] = off[0, :]
    else:
        off[0, :] = 0.0
        off[ny, :] = 0.0

    def vert(i, j):
        return np.array([xlo + i * dx, ylo + j * dy]) + off[j, i]

    E = 2 * nx * ny
    xy = np.zeros((E, 3, 2))
    nbr = np.zeros((E, 3), dtype=np.int32)
    nbf = np.zeros((E, 3), dtype=np.int32)
    cell = lambda i, j: 2 * (j * nx + i)
    for j in range(ny):
        for i in range(nx):
            e0, e1 = cell(i, j), cell(i, j) + 1
            A, B, C, D = vert(i, j), vert(i + 1, j), vert(i + 1, j + 1), vert(i, j + 1)
            xy[e0] = (A, B, D)
            xy[e1] = (C, D, B)
            # e0: face 0 A-B (bottom), face 1 B-D (diagonal), face 2 D-A (left)
            if j > 0 or py:
                nbr[e0, 0], nbf[e0, 0] = cell(i, (j - 1) % ny) + 1, 0
            else:
                nbr[e0, 0], nbf[e0, 0] = -1 - 2, -1
            nbr[e0, 1], nbf[e0, 1] = e1, 1
            if i > 0 or px:
                nbr[e0, 2], nbf[e0, 2] = cell((i - 1) % nx, j) + 1, 2
            else:
                nbr[e0, 2], nbf[e0, 2] = -1 - 0, -1
            # e1: face 0 C-D (top), face 1 D-B (diagonal), face 2 B-C (right)
            if j < ny - 1 or py:
                nbr[e1, 0], nbf[e1, 0] = cell(i, (j + 1) % ny), 0
            else:
                nbr[e1, 0], nbf[e1, 0] = -1 - 3, -1
            nbr[e1, 1], nbf[e1, 1] = e0, 1
            if i < nx - 1 or px:
                nbr[e1, 2], nbf[e1, 2] = cell((i + 1) % nx, j), 2
            else:
                nbr[e1, 2], nbf[e1, 2] = -1 - 1, -1
    return dict(xy=xy, nbr=nbr, nbr_face=nbf)


# ----------------------------------------------------------------------------
# seeded random modal states (fuzz inputs)
# ----------------------------------------------------------------------------

def fuzz_scalar(M, E, nsp, seed, scale=0.5, decay=0.6, offset=0.0):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((1, M, E, nsp)) * scale
    u *= (decay ** np.arange(M))[None, :, None, None]
    u[:, 0] += offset
    return u


def fuzz_euler(dim, M, E, nsp, seed, pert=0.02, vacuum_frac=0.0, gamma=GAMMA):
    """Realizable Euler states with small gPC perturbations.

    A fraction `vacuum_frac` of the elements gets a low mean density and
    pressure with strong spatial and random variation so that density or
    pressure dips below zero at some nodes (elements the limiter must act on).
    """
    rng = np.random.default_rng(seed)
    S = dim + 2
    rho = rng.uniform(0.5, 2.0, (E, 1)) * (1.0 + 0.1 * rng.uniform(-1, 1, (E, nsp)))
    vel = rng.uniform(-0.5, 0.5, (dim, E, 1)) + 0.05 * rng.uniform(-1, 1, (dim, E, nsp))
    p = rng.uniform(0.5, 2.0, (E, 1)) * (1.0 + 0.1 * rng.uniform(-1, 1, (E, nsp)))
    if dim == 1:
        base = _cons1d(rho, vel[0], p, gamma)
    else:
        base = _cons2d(rho, vel[0], vel[1], p, gamma)
    u = np.zeros((S, M, E, nsp))
    u[:, 0] = base
    k = np.arange(1, M)
    u[:, 1:] = rng.standard_normal((S, M - 1, E, nsp)) * pert * (0.5 ** k)[None, :, None, None]
    u[:, 1:] *= np.abs(u[:, :1])  # relative to the local mean
    nvac = int(round(vacuum_frac * E))
    if nvac > 0:
        idx = rng.choice(E, nvac, replace=False)
        pattern = np.where(np.arange(nsp) % 2 == 0, 1.0, -1.0)
        for e in idx:
            r0 = 10.0 ** rng.uniform(-3, -1)
            u[:, :, e, :] = 0.0
            u[0, 0, e, :] = r0 * (1.0 + 0.9 * pattern)
            u[0, 1, e, :] = 0.8 * r0
            u[1, 0, e, :] = r0 * 0.3 * pattern
            u[-1, 0, e, :] = r0 * (1.0 + 0.5 * pattern) / (gamma - 1.0)
            u[-1, 1, e, :] = -0.7 * r0 / (gamma - 1.0)
    return u

"""Helpers for the GPU parity tests (HIP path vs the CPU oracle)."""

import sys

import numpy as np

from oracle.problem import Problem
from oracle.tables import build_tables

# parity bar for FP64 results (relative L2 over the flat modal state)
RTOL_FP64 = 1e-12


def announce(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_for(cfg):
    prob = Problem.from_config(cfg)
    return prob, build_tables(prob)


def solver_for(cfg, precision="fp64"):
    from paper_2112_05946_amd.binding import Solver
    return Solver(cfg, precision=precision)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


# switch decisions taken in a different arithmetic order may differ only when
# the oracle's own decision margin is at the rounding level of the state
LIMITER_TIE = 1e-12     # |min(rho_min, p_min) - eps| / max|state|
SENSOR_TIE = 1e-9       # |S_e - S*| / S*


def check_flags(prob, T, R, gflags, rflags, record):
    """Assert that every flag mismatch is a tie; return the list of ties."""
    from oracle import stabilize as ost
    ties = []
    for pas in range(4):
        bad = np.nonzero(gflags[pas] != rflags[pas])[0]
        if len(bad) == 0:
            continue
        state = record[pas]
        if pas == 2:
            se, thr = ost.sensor_margin(prob, T, R, state)
            rel = np.abs(se[bad] - thr) / thr
            assert np.all(rel <= SENSOR_TIE), ("sensor mismatch", pas, bad[:5], rel[:5])
            ties += [(pas, int(e), float(r)) for e, r in zip(bad, rel)]
        else:
            m, scale = ost.limiter_margin(prob, T, R, state)
            rel = np.abs(m[bad]) / scale[bad]
            assert np.all(rel <= LIMITER_TIE), ("limiter mismatch", pas, bad[:5], rel[:5])
            ties += [(pas, int(e), float(r)) for e, r in zip(bad, rel)]
    if ties:
        print("[ties]", len(ties), "switch decisions at rounding-level margins, e.g.", ties[:3], flush=True)
    return ties


# largest per-element relative error of a state: max over elements e of
# max|a_e - b_e| / max|b_e| (every variable, mode and point of e); catches a bad
# element that the global relative L2 norm would dilute over the whole mesh
ELEM_RTOL = 1e-12


def elem_max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b).max(axis=(0, 1, 3))
    s = np.abs(b).max(axis=(0, 1, 3))
    return float((d / np.where(s > 0, s, 1.0)).max())


def quad_patch(cfg, cx, cy, radius=3):
    """The (2 radius + 1)^2 elements around element (cx, cy) of a quadrilateral mesh as
    a problem of their own: sides that are cut open get outflow ghosts, sides on the
    domain boundary keep theirs, periodic directions wrap.  One SSP-RK3 step reaches
    three elements across faces, so with radius 3 the oracle's step of the patch equals
    the whole mesh's step on the centre element.  Returns (patch config, element ids of
    the patch in the whole mesh, index of the centre in the patch)."""
    nx, ny = cfg["nx"], cfg["ny"]
    bc = list(cfg.get("bc", ["periodic"] * 4))
    dx = (cfg["xhi"] - cfg["xlo"]) / nx
    dy = (cfg["yhi"] - cfg["ylo"]) / ny

    def span(c, n, lo_side):
        if bc[lo_side] == "periodic":
            return [(c + d) % n for d in range(-radius, radius + 1)], "outflow", "outflow", c - radius
        lo, hi = max(0, c - radius), min(n - 1, c + radius)
        return (list(range(lo, hi + 1)), bc[lo_side] if lo == 0 else "outflow",
                bc[lo_side + 1] if hi == n - 1 else "outflow", lo)

    ixs, bx0, bx1, ix0 = span(cx, nx, 0)
    iys, by0, by1, iy0 = span(cy, ny, 2)
    pcfg = dict(cfg, nx=len(ixs), ny=len(iys), xlo=cfg["xlo"] + ix0 * dx, xhi=cfg["xlo"] + (ix0 + len(ixs)) * dx,
                ylo=cfg["ylo"] + iy0 * dy, yhi=cfg["ylo"] + (iy0 + len(iys)) * dy, bc=[bx0, bx1, by0, by1])
    ids = [iy * nx + ix for iy in iys for ix in ixs]
    centre = iys.index(cy) * len(ixs) + ixs.index(cx)
    return pcfg, np.array(ids), centre


def tri_patch(cfg, e, rings=3):
    """Triangle e and every triangle within `rings` faces of it as a mesh of its own
    (cut faces open with outflow ghosts, boundary faces kept); the oracle's step of
    it equals the whole mesh's step on e.  Returns (patch config, ids, 0)."""
    mesh = cfg["mesh"]
    nbr, nbf = mesh["nbr"], mesh["nbr_face"]
    ids = [int(e)]
    depth = {int(e): 0}
    i = 0
    while i < len(ids):
        a = ids[i]
        i += 1
        if depth[a] == rings:
            continue
        for f in range(3):
            b = int(nbr[a, f])
            if b >= 0 and b not in depth:
                depth[b] = depth[a] + 1
                ids.append(b)
    local = {g: l for l, g in enumerate(ids)}
    bc = list(cfg["bc"])
    cut = bc.index("outflow") if "outflow" in bc else 0
    bc[cut] = "outflow"
    pn = np.empty((len(ids), 3), dtype=np.int32)
    pf = np.full((len(ids), 3), -1, dtype=np.int32)
    for l, g in enumerate(ids):
        for f in range(3):
            b = int(nbr[g, f])
            if b < 0:
                pn[l, f] = b
            elif b in local:
                pn[l, f], pf[l, f] = local[b], nbf[g, f]
            else:
                pn[l, f] = -1 - cut
    pcfg = dict(cfg, mesh=dict(xy=mesh["xy"][ids], nbr=pn, nbr_face=pf), bc=bc)
    return pcfg, np.array(ids), 0


def check_patch_step(cfg, u_before, u_after, dt, gflags, picks, patch, tables):
    """For every picked element: the oracle's step (at the GPU's dt) of the element's
    patch, taken from the GPU's state before the step, must give the GPU's element
    after it (relative error per element and over all picks together), and the same
    switch decisions up to rounding-level ties.  Returns the worst per-element error."""
    from oracle import stabilize as ost
    from oracle import stepper as ostep
    T, R = tables
    worst = 0.0
    got, want = [], []
    for e in picks:
        pcfg, ids, c = patch(cfg, *e) if isinstance(e, tuple) else patch(cfg, e)
        g = e[1] * cfg["nx"] + e[0] if isinstance(e, tuple) else int(e)
        prob = Problem.from_config(pcfg)
        rec = []
        ref, _, rfl = ostep.step(prob, u_before[:, :, ids].copy(), dt, (T, R), record=rec)
        got.append(u_after[:, :, g])
        want.append(ref[:, :, c])
        worst = max(worst, elem_max_rel(u_after[:, :, [g]], ref[:, :, [c]]))
        for pas in range(4):
            if bool(gflags[pas, g]) != bool(rfl[pas, c]):
                st = rec[pas]
                if pas == 2:
                    se, thr = ost.sensor_margin(prob, T, R, st)
                    assert abs(se[c] - thr) / thr <= SENSOR_TIE, ("sensor mismatch", e, pas)
                else:
                    m, scale = ost.limiter_margin(prob, T, R, st)
                    assert abs(m[c]) / scale[c] <= LIMITER_TIE, ("limiter mismatch", e, pas)
    err = rel_l2(np.array(got), np.array(want))
    assert err < RTOL_FP64, err
    assert worst < ELEM_RTOL, worst
    return worst

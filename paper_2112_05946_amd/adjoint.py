"""Reverse-mode differentiation of a run of FR-SG steps through the library's
discrete adjoint (fr_sg_adjoint_step), with checkpointing.

AdjointSolve.apply(u0, params, solver, n_steps, dt, k) runs n_steps SSP-RK3
steps from u0 and returns u_T; its backward returns dJ/du0 and dJ/dparams for
any scalar J of u_T built with torch.  params = [adv_speed, gamma] must be the
solver's problem values (the steps use those); dt is fixed (None: the CFL step
of each forward step, then held frozen in the backward pass).

Checkpointing: the state is kept every k steps; the backward pass walks the
segments in reverse, recomputes each segment's step-start states from its
checkpoint with the same forward steps (bitwise the same arithmetic), then
applies the adjoint steps in reverse.  Where the library hands out a step's
stage states (fr_sg_step_stages: the fused 1D path), the recomputation keeps
them too and the adjoint steps take them (fr_sg_adjoint_step_stages) instead of
recomputing them.  Memory: n_steps/k checkpoints plus k (or 3 k) states.

k = 0 keeps every step's start state (and, where the path hands them out, its
two stage states) from the forward run itself: 3 n_steps states (the Burgers
workload of 4096 elements and 500 steps: 1.8 GB), and the backward pass runs the
adjoint steps alone, with nothing recomputed.  The gradient is the same bit for
bit: the kept values are those the recomputation would produce.

Switch decisions (the detector's filter flags) and dt are those of the forward
run; the derivative is that of the discrete map at those decisions.
"""

import math

import numpy as np
import torch


class AdjointSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, params, solver, n_steps, dt=None, k=25):
        pv = params.detach().cpu().numpy()
        want = np.array([float(solver.cfg.get("adv_speed", 0.0)), float(solver.cfg.get("gamma", 1.4))])
        if solver.cfg.get("equation") == "advection" and pv[0] != want[0]:
            raise ValueError("params[0] must equal the solver's advection speed %r" % want[0])
        k = int(k)
        if k < 0:
            raise ValueError("k must be >= 0 (0: keep every step's states)")
        n = int(n_steps)
        dev = u0.device
        u = u0.detach().contiguous().clone()
        flags = torch.empty((max(n, 1), 4 * solver.E), dtype=torch.uint8, device=dev)
        dts = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        ckpts = []
        ctx.kept, ctx.kept_stages = None, False
        if k == 0:
            ctx.kept, ctx.kept_stages = _forward_keeping_all(solver, u, n, dt, dts, flags)
        else:
            for i in range(n):
                if i % k == 0:
                    ckpts.append(u.clone())
                solver.step(u, dt, dts[i:i + 1], flags[i])
        ctx.solver, ctx.n, ctx.k = solver, n, k
        ctx.params_device = params.device
        ctx.ckpts = ckpts
        ctx.save_for_backward(flags, dts)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        flags, dts = ctx.saved_tensors
        solver, n, k = ctx.solver, ctx.n, ctx.k
        lam = grad_u.detach().to(torch.float64).contiguous().clone()
        dparams = torch.zeros(2, dtype=torch.float64, device=lam.device)
        dt_host = dts.cpu().numpy()
        scratch_dt = torch.empty(1, dtype=torch.float64, device=lam.device)
        scratch_fl = torch.empty(4 * solver.E, dtype=torch.uint8, device=lam.device)
        if ctx.kept is not None:
            bufs = ctx.kept
            for i in reversed(range(n)):
                if ctx.kept_stages:
                    solver.adjoint_step_stages(bufs[0, i], bufs[1, i], bufs[2, i], flags[i], float(dt_host[i]), lam,
                                               dparams)
                else:
                    solver.adjoint_step(bufs[0, i], flags[i], float(dt_host[i]), lam, dparams)
            ctx.kept = None
            return lam, dparams.to(ctx.params_device), None, None, None, None
        nseg = math.ceil(n / k)
        kept = None  # the segment's step-start states and stage states, where the path hands them out
        for seg in reversed(range(nseg)):
            start, end = seg * k, min(seg * k + k, n)
            if kept is not False:
                kept = _segment_from_kept_stages(solver, ctx.ckpts[seg], start, end, dt_host, flags, lam, dparams,
                                                 scratch_dt, scratch_fl, kept)
                if kept is not False:
                    continue
            states = [ctx.ckpts[seg]]
            u = ctx.ckpts[seg].clone()
            for i in range(start, end - 1):
                solver.step(u, float(dt_host[i]), scratch_dt, scratch_fl)
                states.append(u.clone())
            for i in reversed(range(start, end)):
                solver.adjoint_step(states[i - start], flags[i], float(dt_host[i]), lam, dparams)
        ctx.ckpts = None
        return lam, dparams.to(ctx.params_device), None, None, None, None


def _forward_keeping_all(solver, u, n, dt, dts, flags):
    """The forward steps of k = 0: every step's start state and, where the path hands
    them out (fr_sg_step_stages), its two stage states into one [3, n] buffer of
    states; returns the buffer and whether it holds the stage states."""
    from .binding import FrsgError
    bufs = torch.empty((3, max(n, 1)) + tuple(u.shape), dtype=torch.float64, device=u.device)
    stages = True
    for i in range(n):
        bufs[0, i].copy_(u)
        if stages:
            try:
                solver.step_stages(u, bufs[1, i], bufs[2, i], dt, dts[i:i + 1], flags[i])
                continue
            except FrsgError as err:
                if i > 0 or err.status != -2:
                    raise
                stages = False
                # start states only: the n-state buffer replaces the 3 n-state one
                first = bufs[0, 0].clone()
                del bufs
                bufs = torch.empty((1, max(n, 1)) + tuple(u.shape), dtype=torch.float64, device=u.device)
                bufs[0, 0].copy_(first)
        solver.step(u, dt, dts[i:i + 1], flags[i])
    return bufs, stages


def _segment_from_kept_stages(solver, ckpt, start, end, dt_host, flags, lam, dparams, scratch_dt, scratch_fl, bufs):
    """One segment of the backward pass with the library's stage-keeping step: the
    recomputation keeps every step's start state and its two stage states, and the
    adjoint steps take them instead of recomputing the stages (the same values, so
    the same gradient).  Returns the buffers for the next segment, or False, having
    done nothing, where the path does not hand stage states out."""
    from .binding import FrsgError
    k = end - start
    if bufs is None or bufs.shape[1] < k:
        bufs = torch.empty((3, k) + tuple(ckpt.shape), dtype=torch.float64, device=ckpt.device)
    u = ckpt.clone()
    for j in range(k):
        bufs[0, j].copy_(u)
        try:
            solver.step_stages(u, bufs[1, j], bufs[2, j], float(dt_host[start + j]), scratch_dt, scratch_fl)
        except FrsgError as err:
            if j == 0 and err.status == -2:
                return False
            raise
    for j in reversed(range(k)):
        solver.adjoint_step_stages(bufs[0, j], bufs[1, j], bufs[2, j], flags[start + j], float(dt_host[start + j]),
                                   lam, dparams)
    return bufs


def quadrature_weights(solver):
    """Legendre-Gauss weights of the solver's solution points (sum 2)."""
    _, w = np.polynomial.legendre.leggauss(int(solver.cfg["p"]) + 1)
    return torch.from_numpy(w).to(solver.device)


def mean_square(u, solver):
    """J = sum_e J_e sum_j w_j sum_k u[0, k, e, j]^2: the space integral of E[u^2]
    (= E[u]^2 + Var[u]) for orthonormal chaos; 1D."""
    dx = (float(solver.cfg["xhi"]) - float(solver.cfg["xlo"])) / int(solver.cfg["nx"])
    w = quadrature_weights(solver)
    return 0.5 * dx * torch.sum(u[0] * u[0] * w)

"""Failure modes forced from the host (every kernel runs to completion on them).

* Sod with an uncertain interface (Sec. 5.3, second case): without the
  positivity limiter the SG solution loses realizability and the next CFL step
  reports a non-finite wave speed (FRSG_ENONFINITE) within a few dozen steps; with
  the limiter the same run stays finite (the failure the paper documents for the
  unlimited scheme).
* A time step above the SSP-RK3 stability limit (CFL 2 with p = 2, against a
  limit of about 0.63 for dt = CFL dx / ((p+1) lambda)) makes the advection
  solution grow without bound; CFL 0.3 keeps it bounded.
"""

import numpy as np
import pytest

from gpu_util import announce, solver_for, to_np
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu


def _run_until_error(sol, u, nsteps):
    from paper_2112_05946_amd.binding import FrsgError
    for i in range(nsteps):
        sol.step(u)
        try:
            sol.sync()
        except FrsgError as e:
            return i, e.status
    return None, 0


def test_sod_needs_the_limiter():
    announce("failure_sod_unlimited")
    cfg = dict(inputs.small(inputs.SOD, 128), filter="none")
    sol = solver_for(dict(cfg, limiter=False))
    u = sol.initial_state(limit=False)
    step, status = _run_until_error(sol, u, 200)
    print("[failure] unlimited Sod: status %d at step %s" % (status, step), flush=True)
    assert step is not None and status in (-4, -5)
    sol2 = solver_for(cfg)
    u2 = sol2.initial_state()
    step2, status2 = _run_until_error(sol2, u2, 200)
    assert step2 is None
    assert np.all(np.isfinite(to_np(u2)))


def test_cfl_above_the_stability_limit_blows_up():
    announce("failure_cfl")
    growth = {}
    for cfl in (0.3, 2.0):
        sol = solver_for(dict(inputs.ADVECTION, cfl=cfl))
        u = sol.initial_state()
        n0 = float(np.linalg.norm(to_np(u)))
        for _ in range(60):
            sol.step(u)
        sol.sync()
        growth[cfl] = float(np.linalg.norm(to_np(u))) / n0
    print("[failure] norm growth over 60 steps:", growth, flush=True)
    assert growth[0.3] <= 1.0 + 1e-12
    assert growth[2.0] > 1e3

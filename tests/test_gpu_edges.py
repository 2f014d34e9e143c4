"""Edge cases on the GPU against the oracle: zero steps, the largest chaos sizes the
library accepts (128 modes, 256 nodes), an all-zero state with the detector on,
and a right-hand side on a single element."""

import numpy as np
import pytest

from gpu_util import RTOL_FP64, announce, oracle_for, rel_l2, solver_for, to_dev, to_np
from oracle import fr as ofr
from oracle import stepper as ostep
from oracle.initial import project_initial
from paper_2112_05946_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("label,cfg", [
    ("fused2d", inputs.small(inputs.SHOCK_VORTEX, 8, 4)),
    ("fused1d", inputs.small(inputs.BURGERS, 16)),
    ("generic2d", inputs.small(inputs.SHOCK_VORTEX, 5, 3)),
    ("tri_fused", inputs.tri_shock_vortex(2)),
])
def test_zero_steps_leave_the_state_alone(label, cfg):
    announce("zero_steps", label)
    sol = solver_for(cfg)
    u = sol.initial_state()
    before = to_np(u).copy()
    sol.steps(u, 0)
    sol.sync()
    assert np.array_equal(to_np(u), before)
    from paper_2112_05946_amd.binding import FrsgError
    with pytest.raises(FrsgError):
        sol.steps(u, -1)


@pytest.mark.parametrize("label,cfg", [
    # 128 modes on 128 nodes (one random dimension), the mode limit
    ("modes128", dict(inputs.small(inputs.BURGERS, 3), p=2, gpc_order=127, nq1d=128, filter="exp",
                      sensor="always")),
    # 256 nodes (two random dimensions, 16 x 16), the node limit
    ("nodes256", dict(inputs.small(inputs.SHOCK_VORTEX, 3, 2), gpc_order=14, nq1d=16)),
])
def test_largest_chaos_sizes(label, cfg):
    announce("largest_chaos", label)
    prob, (T, R) = oracle_for(cfg)
    u0 = project_initial(prob, cfg["ic"], (T, R))
    if prob.equation == "burgers":
        u0 = u0 + inputs.fuzz_scalar(R.M, prob.E, T.n, seed=5, scale=0.05)
    sol = solver_for(cfg)
    got = to_np(sol.rhs(to_dev(u0)))
    sol.sync()
    ref = ofr.rhs(prob, T, R, u0)
    assert rel_l2(got, ref) < RTOL_FP64
    ud = to_dev(u0)
    un, rdt, _ = ostep.step(prob, u0, None, (T, R))
    dtd, _ = sol.step(ud)
    sol.sync()
    assert abs(to_np(dtd)[0] / rdt - 1.0) < 1e-13
    assert rel_l2(to_np(ud), un) < RTOL_FP64


def test_all_zero_state_with_detector():
    """Burgers with u = 0: zero right-hand side, the detector's energy ratio has a zero
    denominator (no flag), the step keeps the state at zero with the fixed dt."""
    cfg = inputs.small(inputs.BURGERS, 12)
    announce("zero_state", "burgers detector")
    prob, (T, R) = oracle_for(cfg)
    sol = solver_for(cfg)
    u = to_dev(np.zeros((1, R.M, prob.E, T.n)))
    assert not np.any(to_np(sol.rhs(u)))
    dtd, flags = sol.step(u, 1e-3)
    sol.sync()
    assert not np.any(to_np(u)) and not to_np(flags).any()


@pytest.mark.parametrize("n", [1, 2, 7, 1000003])
def test_device_copy_kernel(n):
    """The streaming copy kernel (the bandwidth reference of the benchmark) copies
    every element, odd tails included, and nothing beyond."""
    import torch
    from paper_2112_05946_amd.binding import device_copy
    announce("device_copy", n)
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.full((n + 2,), 7.0, dtype=torch.float64, device="cuda")
    device_copy(src, dst[:n])
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert torch.all(dst[n:] == 7.0)

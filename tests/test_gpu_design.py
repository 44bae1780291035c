"""Inverse design through the adjoint (application of the reverse step).

Twin experiment: the film of inputs.stripe_recovery (128^2, h0 = 0.1 + 1e-4
noise on h_* = 0.095) is run 300 FP32 steps under the true stripe pattern
theta* (pi/9 | pi/4, period 32); starting from theta = pi/6 everywhere, Adam
on theta = (pi/2) sigmoid(z) with the TFLBMRun gradient must bring the misfit
of the final height down by three orders of magnitude and recover theta*:
correlation above 0.99 and the mean fitted angle on each kind of stripe
within 0.04 rad of its true value.
"""
import math

import pytest
import torch

from gpu_common import banner
from paper_1810_07642_amd import inputs

pytestmark = pytest.mark.gpu


def test_inverse_design_recovers_stripe_pattern():
    from paper_1810_07642_amd import Sim
    from paper_1810_07642_amd.design import fit_contact_angle
    banner("inverse design 128^2, 300 steps, 80 Adam iterations")
    n, steps = 128, 300
    p, h0, th_true = inputs.stripe_recovery(n=n)
    p = dict(p, href=0.1)
    sim = Sim(n, n, "fp32", **p).init(h0, th_true)
    sim.step(steps)
    sim.check()
    target = sim.height()
    res = fit_contact_angle(h0, target, p, steps, theta_init=math.pi / 6, iters=80, lr=0.05, K=64, prec="fp32")
    th = res.theta.cpu()
    corr = float(torch.corrcoef(torch.stack([th.flatten(), th_true.flatten()]))[0, 1])
    lo, hi = th_true < 0.4, th_true > 0.75
    print(f"loss {res.losses[0]:.3e} -> {res.final_loss:.3e}, corr {corr:.4f}, "
          f"mean theta {float(th[lo].mean()):.3f} (true {math.pi / 9:.3f}) / {float(th[hi].mean()):.3f} "
          f"(true {math.pi / 4:.3f})")
    assert res.final_loss <= 1e-3 * res.losses[0]
    assert corr > 0.99
    assert abs(float(th[lo].mean()) - math.pi / 9) < 0.04
    assert abs(float(th[hi].mean()) - math.pi / 4) < 0.04


def test_checkpoint_interval_keeps_captures_when_they_fit():
    """K = 0 (every capture kept) when nsteps captures take at most the given
    fraction of free device memory, else checkpoints every 64 steps."""
    from paper_1810_07642_amd.design import checkpoint_interval
    from paper_1810_07642_amd.sim import capture_bytes_for
    free, _ = torch.cuda.mem_get_info()
    cb = capture_bytes_for(512, 512, "fp32")
    fits = int(0.25 * free // cb)
    assert checkpoint_interval(512, 512, fits, "fp32") == 0
    assert checkpoint_interval(512, 512, 2 * fits + 100, "fp32") == 64

"""Inverse design of a wettability pattern through the adjoint of the step.

Finds the contact-angle field theta(x, y) under which a film, started from a
given h0 and run `nsteps` lattice Boltzmann steps (Sec. II), ends closest to a
target height field: it minimises

    L(theta) = 1/2 sum_x (h_N(x; theta) - h_target(x))^2

with Adam, the gradient dL/dtheta coming from TFLBMRun (hand-written adjoint
step; by default every step's captured moments are kept when they take at
most a quarter of the free device memory, else checkpoints every 64 steps and
a recompute).  theta is
kept inside (0, theta_max) by the parametrisation theta = theta_max sigmoid(z),
and z is what Adam moves.

    res = fit_contact_angle(h0, target, params, nsteps=2000, theta_init=0.5, iters=60)
    res.theta, res.losses
"""
import math
from dataclasses import dataclass, field

import torch

from .autograd import TFLBMRun


@dataclass
class FitResult:
    theta: torch.Tensor                  # fitted theta field [ny, nx], float64
    losses: list = field(default_factory=list)   # L at every iteration (before the update)
    final_loss: float = float("nan")     # L at the fitted theta



def checkpoint_interval(nx, ny, nsteps, prec="fp32", fraction=0.25):
    """K for TFLBMRun: 0 (keep every step's capture, no recompute) when the
    nsteps captures take at most `fraction` of the free memory of the current
    GPU, else 64."""
    from .sim import capture_bytes_for
    free, _ = torch.cuda.mem_get_info()
    return 0 if nsteps * capture_bytes_for(nx, ny, prec) <= fraction * free else 64


def fit_contact_angle(h0, target, params, nsteps, theta_init=math.pi / 6, iters=60, lr=0.1, K=None,
                      prec="fp32", theta_max=math.pi / 2, callback=None):
    """Adam on z, theta = theta_max sigmoid(z).  h0, target: [ny, nx] tensors
    (moved to the current GPU in float64); theta_init: a scalar or a field.
    K: TFLBMRun's checkpoint interval (None: checkpoint_interval).
    callback(it, loss, theta) is called every iteration if given."""
    dev = torch.device("cuda", torch.cuda.current_device())
    h0 = torch.as_tensor(h0, dtype=torch.float64).to(dev)
    if K is None:
        K = checkpoint_interval(h0.shape[1], h0.shape[0], nsteps, prec)
    tgt = torch.as_tensor(target, dtype=torch.float64).to(dev)
    th0 = torch.as_tensor(theta_init, dtype=torch.float64)
    if th0.dim() == 0:
        th0 = th0.expand(h0.shape)
    th0 = th0.to(dev)
    if not bool(((th0 > 0) & (th0 < theta_max)).all()):
        raise ValueError("theta_init must lie inside (0, theta_max)")
    z = torch.logit(th0 / theta_max).clone().requires_grad_(True)
    opt = torch.optim.Adam([z], lr=lr)
    res = FitResult(theta=th0.clone())

    def loss_at(theta):
        h = TFLBMRun.apply(h0, theta, params, nsteps, K, prec)
        return 0.5 * ((h - tgt) ** 2).sum()

    for it in range(iters):
        opt.zero_grad()
        theta = theta_max * torch.sigmoid(z)
        loss = loss_at(theta)
        loss.backward()
        res.losses.append(float(loss.detach()))
        if callback is not None:
            callback(it, float(loss), theta.detach())
        opt.step()
    with torch.no_grad():
        res.theta = (theta_max * torch.sigmoid(z)).detach()
        res.final_loss = float(loss_at(res.theta))
    return res

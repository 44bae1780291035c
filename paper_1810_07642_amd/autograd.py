"""Differentiable multi-step run: torch.autograd.Function over the C ABI.

Forward: f = E(h0), kappa(theta), then `nsteps` HIP steps, storing the
population buffer every K steps; returns the final height h_N.
Backward: for each K-step segment, last to first, reload its checkpoint,
recompute the segment with the forward moments captured at every step, and
run the hand-written adjoint backwards through it (two steps per pass over
the lattice); finally map the adjoint of the initial populations and the
FP64 kappa gradient to dLoss/dh0 and dLoss/dtheta.  Memory: nsteps/K
checkpoints plus K captures.

K = 0 trades memory for the recompute: the forward itself writes the
captures of every step (3 values per site and step: 12.9 GB for 4096 FP32
steps of a 512 x 512 lattice) and the backward is the reverse pass alone.
"""
import torch

from .sim import Sim


class TFLBMRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h0, theta, params, nsteps, K=64, prec="fp64"):
        if theta is None:
            raise ValueError("TFLBMRun needs a theta field")
        ny, nx = h0.shape
        sim = Sim(nx, ny, prec, device=h0.device if h0.is_cuda else None, **params)
        sim.init(h0, theta)
        ckpts = []
        done = 0
        nsteps = int(nsteps)
        K = int(K)
        if K < 0:
            raise ValueError("K must be >= 0")
        if K == 0:
            # every step's capture kept: no checkpoints, no recompute
            cap = torch.empty(nsteps * sim.capture_bytes(), dtype=torch.uint8, device=sim.device)
            sim.step_capture(nsteps, cap)
            ckpts.append((cap, 0, nsteps))
        else:
            while done < nsteps:
                k = min(K, nsteps - done)
                ckpts.append((sim.state_save(), done, k))
                sim.step(k)
                done += k
        h = sim.height()
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.K = K
        return h

    @staticmethod
    def backward(ctx, grad_h):
        sim = ctx.sim
        adj = torch.empty(sim.adj_bytes(), dtype=torch.uint8, device=sim.device)
        sim.adj_seed(adj, grad_h)
        if ctx.K == 0:
            cap, _, k = ctx.ckpts[0]
            sim.adj_steps(adj, cap, k)
        else:
            cap = torch.empty(ctx.K * sim.capture_bytes(), dtype=torch.uint8, device=sim.device)
            for buf, start, k in reversed(ctx.ckpts):
                sim.state_load(buf, start)
                sim.step_capture(k, cap)
                sim.adj_steps(adj, cap, k)
        g_h0, g_theta = sim.adj_finish(adj)
        ctx.sim = None
        ctx.ckpts = None
        return g_h0, g_theta, None, None, None, None


def run_with_grad(h0, theta, params, nsteps, K=64, prec="fp64"):
    """h_N = TFLBMRun.apply(h0, theta, params, nsteps, K, prec); K = 0 keeps
    every step's capture instead of checkpoints."""
    return TFLBMRun.apply(h0, theta, params, nsteps, K, prec)

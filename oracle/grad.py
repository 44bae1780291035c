"""Gradient oracle: reverse-mode differentiation of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/lbm.py``).  The gradient of a scalar
function of the final height with respect to the contact-angle field
theta(x, y) and the initial height h0 is obtained with torch autograd through
the plain forward step of ``oracle.lbm``, recomputing each segment of K steps
from a stored state (``torch.utils.checkpoint``).  It is independent of the
hand-written adjoint of the HIP path.

The paper has no adjoint; the differentiated map is the forward step of
Sec. II (eqs. "LBE", "equilibria", "force", "pfilm", "disjoiningP",
"forcefric", "alphafric", "derivative", "n_laplace") started from
f = E(h0) and read out as h = sum_l f_l.
"""
import torch
from torch.utils.checkpoint import checkpoint

from . import lbm


def final_height(h0, theta, p, nsteps, K=64):
    """h after ``nsteps`` steps from f = E(h0) with kappa(theta); differentiable."""
    kap = lbm.kappa(theta, p)
    f = lbm.init(h0, p)
    done = 0
    while done < nsteps:
        k = min(K, nsteps - done)
        f = checkpoint(lbm.run, f, kap, p, k, use_reentrant=False)
        done += k
    h, _, _ = lbm.moments(f)
    return h


def vjp(h0, theta, grad_h, p, nsteps, K=64):
    """Return (dL/dh0, dL/dtheta) for a loss whose gradient w.r.t. the final
    height is ``grad_h``."""
    h0 = h0.detach().clone().to(lbm.DTYPE).requires_grad_(True)
    theta = theta.detach().clone().to(lbm.DTYPE).requires_grad_(True)
    h = final_height(h0, theta, p, nsteps, K)
    g_h0, g_theta = torch.autograd.grad(h, (h0, theta), grad_outputs=grad_h.to(lbm.DTYPE))
    return g_h0.detach(), g_theta.detach()


def misfit_loss(h0, theta, target, p, nsteps, K=64):
    """L = 1/2 sum_x (h_N(x) - target(x))^2 (float; no gradient)."""
    with torch.no_grad():
        h = final_height(h0.to(lbm.DTYPE), theta.to(lbm.DTYPE), p, nsteps, K)
        return 0.5 * float(((h - target.to(lbm.DTYPE)) ** 2).sum())


def misfit_grad(h0, theta, target, p, nsteps, K=64):
    """(L, dL/dh0, dL/dtheta) for the L2 misfit of the final height."""
    with torch.no_grad():
        h = final_height(h0.to(lbm.DTYPE), theta.to(lbm.DTYPE), p, nsteps, K)
        grad_h = h - target.to(lbm.DTYPE)
        loss = 0.5 * float((grad_h ** 2).sum())
    g_h0, g_theta = vjp(h0, theta, grad_h, p, nsteps, K)
    return loss, g_h0, g_theta


def jvp(h0, theta, v_h0, v_theta, p, nsteps):
    """Forward-mode derivative of the final height, J (v_h0, v_theta), with
    torch.func.jvp through the same forward step (no checkpointing): a
    differentiation independent of the reverse mode above, for dot-product
    tests <w, J v> = <J^T w, v>."""
    def fn(a, b):
        f = lbm.run(lbm.init(a, p), lbm.kappa(b, p), p, nsteps)
        h, _, _ = lbm.moments(f)
        return h
    args = (h0.detach().to(lbm.DTYPE), theta.detach().to(lbm.DTYPE))
    tangents = (v_h0.detach().to(lbm.DTYPE), v_theta.detach().to(lbm.DTYPE))
    _, jv = torch.func.jvp(fn, args, tangents)
    return jv.detach()

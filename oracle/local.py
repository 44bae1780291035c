"""Sampled evaluation of the FP64 CPU oracle on large periodic grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/lbm.py``).

One step moves information at most three sites: the post-collision value at a
source site needs the pressure gradient there (pressure on the 1-ring), the
pressure needs the height on the 1-ring around each of those sites, and
streaming adds one more site.  After k steps the state at a site therefore
depends only on the initial fields within Chebyshev distance 3k.  The oracle
step is run unchanged on a periodic window of half-width R >= 3k cut out of
the full initial fields; wrong wrap-around neighbours at the window border
reach at most 3k sites inwards in k steps, so the window centre is exact.
This lets the whole-array oracle check chosen sites of grids that it could
not step as a whole (e.g. 4096 x 4096).
"""
import torch

from . import lbm


def _windows(field, sites, R):
    """Stack periodic windows of half-width R centred on ``sites``: [S, 2R+1, 2R+1]."""
    ny, nx = field.shape
    off = torch.arange(-R, R + 1)
    out = []
    for (y, x) in sites:
        ys = (y + off) % ny
        xs = (x + off) % nx
        out.append(field[ys][:, xs])
    return torch.stack(out)


def sampled_run(h0, theta, p, nsteps, sites, gamma=None):
    """Run ``nsteps`` oracle steps from f = E(h0) and return the height and
    velocity at each (y, x) in ``sites`` as three float64 tensors [S];
    ``gamma``: optional surface tension field."""
    R = 3 * int(nsteps) + 2
    hw = _windows(h0.to(lbm.DTYPE), sites, R)
    tw = _windows(theta.to(lbm.DTYPE), sites, R)
    gw = None if gamma is None else _windows(gamma.to(lbm.DTYPE), sites, R)
    kap = lbm.kappa(tw, p)
    f = lbm.run(lbm.init(hw, p), kap, p, nsteps, gw)
    h, ux, uy = lbm.readout(f)
    return h[:, R, R].clone(), ux[:, R, R].clone(), uy[:, R, R].clone()

"""Drop sliding on an incline (Sec. III C): steady capillary number.

A spherical-cap drop on the precursor film (periodic lattice) is pushed along
x by the body force F = h (a, 0) of eq. "force", with a set by the Bond number
Bo = (3V/4pi)^(2/3) a / gamma (inputs.sliding_drop).  The drop's position is
the circular mean of the x coordinate weighted by h - h_* (periodic in x), its
speed U the displacement over a late window of steps, and the capillary number
Ca = mu U / gamma with mu = nu (rho_0 = 1).

    ca, h = sliding_capillary_number("fp32", bond=0.4, delta=1.0, hstar=0.5)

The stepping runs in the HIP library (Sim); this module only reads h back.
"""
import math

import torch

from . import inputs


def drop_position(h, hstar):
    """Periodic x position of the drop: circular mean of x weighted by h - h_*."""
    nx = h.shape[1]
    d = (h - hstar).clamp(min=0)
    ang = 2 * math.pi * torch.arange(nx, dtype=torch.float64, device=h.device).view(1, -1) / nx
    a = math.atan2(float((d * torch.sin(ang)).sum()), float((d * torch.cos(ang)).sum()))
    return (a % (2 * math.pi)) * nx / (2 * math.pi)


def sliding_capillary_number(prec, bond, delta, hstar=0.5, nx=1024, ny=512, steps=100000, window=20000,
                             base_radius=40.0, theta=math.pi / 6, href=None):
    """Steady Ca of the sliding drop after `steps` steps, from the drift over
    the last `window` steps, and the final height field.  Storage deviations
    are taken from href = h_* unless given.  Raises TFLBMError if the run meets
    h <= 0 or a non-finite h."""
    from .sim import Sim
    p, h0, th = inputs.sliding_drop(nx=nx, ny=ny, bond=bond, delta=delta, hstar=hstar,
                                    base_radius=base_radius, theta=theta)
    sim = Sim(nx, ny, prec, href=hstar if href is None else href, **p).init(h0, th)
    sim.step(steps - window)
    sim.check()
    x0 = drop_position(sim.height(), hstar)
    sim.step(window)
    sim.check()
    h = sim.height()
    x1 = drop_position(h, hstar)
    U = ((x1 - x0 + nx / 2) % nx - nx / 2) / window
    nu = (p["tau"] - 0.5) / 3.0
    return nu * U / p["gamma"], h


BONDS = (0.1, 0.2, 0.4, 0.8)
DELTAS = (0.5, 1.0, 2.0)


def capillary_sweep(prec, bonds=BONDS, deltas=DELTAS, hstar=0.5, **kw):
    """Steady Ca of the sliding drop at every (delta, Bond) point:
    {(delta, bond): Ca}."""
    return {(d, b): sliding_capillary_number(prec, b, d, hstar=hstar, **kw)[0] for d in deltas for b in bonds}


def critical_bond(bonds, cas):
    """Least-squares line Ca = s (Bo - Bo_c) through the points of one slip
    length (Sec. III C, eq. "CaBo"): (slope s, intercept Bo_c, largest
    residual relative to the largest Ca)."""
    import numpy as np
    b = np.asarray(bonds, dtype=np.float64)
    c = np.asarray(cas, dtype=np.float64)
    s, c0 = np.polyfit(b, c, 1)
    res = float(np.abs(c - (s * b + c0)).max() / np.abs(c).max())
    return float(s), float(-c0 / s), res

"""Helpers shared by the GPU tests: run the same seeded inputs through the HIP
path (C ABI via paper_1810_07642_amd.Sim) and through the FP64 oracle."""
import math

import torch

from oracle import lbm

F64 = torch.float64
U32 = 2.0 ** -24  # FP32 unit roundoff


def random_case(ny, nx, seed, hlo=0.3, hhi=0.6, tlo=0.2, thi=0.7):
    g = torch.Generator().manual_seed(seed)
    h0 = hlo + (hhi - hlo) * torch.rand((ny, nx), generator=g, dtype=F64)
    th = tlo + (thi - tlo) * torch.rand((ny, nx), generator=g, dtype=F64)
    return h0, th


def oracle_run(params, h0, th, steps):
    P = lbm.Params(**params)
    f = lbm.run(lbm.init(h0, P), lbm.kappa(th, P), P, steps)
    h, ux, uy = lbm.readout(f)
    return h, ux, uy, lbm.mass(f)


def gpu_run(params, h0, th, steps, prec, theta_field=True, **extra):
    from paper_1810_07642_amd import Sim
    ny, nx = h0.shape
    kw = dict(params)
    kw.update(extra)
    if not theta_field:
        kw["theta0"] = float(th.reshape(-1)[0])
    sim = Sim(nx, ny, prec, **kw)
    sim.init(h0, th if theta_field else None)
    sim.step(steps)
    h, ux, uy = sim.read()
    sim.check()
    m = sim.mass()
    torch.cuda.synchronize()
    return h.cpu(), ux.cpu(), uy.cpu(), m


def max_rel(a, b):
    """max |a - b| / max |b| (0 if both vanish)."""
    scale = float(b.abs().max())
    d = float((a - b).abs().max())
    return d / scale if scale > 0 else d


def fp32_tol(steps):
    """Bound on max |dh| / max h for the FP32 step after `steps` steps: about
    30 rounded operations feed each new h, each within u = 2^-24 relative, and
    the dissipative step does not amplify them, so the error stays below
    30 u per step, accumulated linearly."""
    return 30.0 * U32 * max(1, steps)


def banner(msg):
    print(msg, flush=True)

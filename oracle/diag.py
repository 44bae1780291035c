"""Term-balance diagnostic of the appendix (eq. "magnitude"), plain FP64 CPU.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests use it.  It shares no code with the HIP
path.

The appendix checks the reduction from the depth-averaged momentum equation
(eq. "hydro2") to the film equation the method solves by comparing, over the
whole lattice, the magnitudes of the terms on its right-hand side.  From the
pre-collision populations f at time t (h, j = h u by Sec. II, the film
pressure by eqs. "pfilm", "disjoiningP"), per component a in {x, y}:

    pressure_a  = -h d_a p_film                               (film pressure gradient)
    friction_a  = -nu alpha_delta(h) u_a                      (eqs. "forcefric", "alphafric")
    viscous_a   = nu lap(h u_a) + 2 nu d_a (div(h u))         (longitudinal viscous terms)
    advection_a = div(h u u_a) = d_x(j_x u_a) + d_y(j_y u_a)  (advection, omitted in the
                                                              paper's figure as negligible)

and the norm of eq. "magnitude", ||phi|| = (N^-1 sum_x phi(x)^2)^(1/2) over the
N = nx ny sites (the paper's N^2 for an N x N lattice).

Reading (the appendix does not say how the terms are discretised): every
derivative is the isotropic stencil of the step (eq. "derivative"), the
Laplacian that of eq. "n_laplace", and d_a(div j) applies the derivative
stencil to the stencil divergence d_x j_x + d_y j_y.
"""
import math

from . import lbm

NAMES = ("pressure_x", "friction_x", "viscous_x", "advection_x",
         "pressure_y", "friction_y", "viscous_y", "advection_y")


def term_fields(f, kap, p, gam=None):
    """The eight term fields of the module docstring, as a dict of [ny, nx]
    arrays; ``gam``: optional per-site surface tension field."""
    h, jx, jy = lbm.moments(f)
    ux = jx / h
    uy = jy / h
    pf = lbm.film_pressure(h, kap, p, gam)
    gpx, gpy = lbm.gradient(pf)
    alpha = lbm.friction_coefficient(h, p.delta)
    djx_x, _ = lbm.gradient(jx)
    _, djy_y = lbm.gradient(jy)
    div = djx_x + djy_y
    ddiv_x, ddiv_y = lbm.gradient(div)
    ax_x, _ = lbm.gradient(jx * ux)
    _, ax_y = lbm.gradient(jy * ux)
    ay_x, _ = lbm.gradient(jx * uy)
    _, ay_y = lbm.gradient(jy * uy)
    return {
        "pressure_x": -h * gpx,
        "friction_x": -p.nu * alpha * ux,
        "viscous_x": p.nu * lbm.laplacian(jx) + 2.0 * p.nu * ddiv_x,
        "advection_x": ax_x + ax_y,
        "pressure_y": -h * gpy,
        "friction_y": -p.nu * alpha * uy,
        "viscous_y": p.nu * lbm.laplacian(jy) + 2.0 * p.nu * ddiv_y,
        "advection_y": ay_x + ay_y,
    }


def norm(phi):
    """(N^-1 sum phi^2)^(1/2) (eq. "magnitude"), the sum correctly rounded."""
    vals = phi.detach().reshape(-1)
    return math.sqrt(math.fsum((vals * vals).tolist()) / vals.numel())


def term_norms(f, kap, p, gam=None):
    """Norms of the eight term fields, a dict name -> float."""
    return {k: norm(v) for k, v in term_fields(f, kap, p, gam).items()}

"""Plain FP64 CPU oracle of the thin-film lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
helpers with the HIP path.

It executes the method of Zitz et al., "A lattice Boltzmann method for thin
liquid film hydrodynamics" (arXiv:1810.07642), step by step, in float64 torch
CPU tensors, with whole-array operations written in the order the paper
states them.  Arrays are indexed ``[y, x]``; populations are ``f[l, y, x]``;
every boundary is periodic (Sec. III, opening paragraph).

Readings of silent, ambiguous or garbled passages (each one listed again in
the design notes):

* Equilibrium (Sec. II, eq. "equilibria"): the printed c_s^2 and c_s^4 in the
  denominators are read as the lattice speed dx/dt = 1.  Only this reading
  satisfies the three moment constraints of Sec. II (height, momentum and the
  shallow-water momentum flux).  c_s^2 = 1/3 is kept in the forcing term of
  eq. "LBE" and in the viscosity.
* Laplacian (Sec. II, eq. "n_laplace"): the weights w_l printed inside the
  sums are dropped; with them the stencil does not vanish on a constant.
* Film pressure (Sec. II, eqs. "pfilm" and "disjoiningP"): the disjoining
  term enters with the sign that makes the precursor film stable and gives
  partial wetting, p = -gamma (lap h + kappa f(h)).  kappa f(h) does not
  change when n and m are swapped.
* Forcing (Sec. II, eq. "LBE"): the plain source w_l (dt/c_s^2) c_l.F with no
  (1 - omega/2) factor and no velocity shift; u = j/h.
* All right-hand-side terms of a step use the pre-collision populations at
  time t; the initial populations are the equilibrium at rest, f = E(h0).
* The BGK relaxation (1 - omega) f + omega f^eq of eq. "LBE" is evaluated
  as f + omega (f^eq - f): the same real number, but a population already at
  equilibrium is reproduced exactly, and the rounding of (1 - omega) + omega
  does not bias the total mass once per step.
* Body force (Sec. II, after eq. "alphafric"): F = h (a_x, a_y).
* Position-dependent surface tension (Sec. II, the sentence after eq.
  "n_laplace", which names such a field among those the stencils apply to,
  without writing its model): gamma(x) takes the place of gamma in eq.
  "pfilm", p = -gamma(x) (lap h + kappa f(h)), and F_film = -h grad p as
  before, so the gradient stencil acts on the product.  A Marangoni stress
  at the free surface is not part of the paper's equations and is not
  added.
"""
import math

import torch

DTYPE = torch.float64

# D2Q9 lattice velocities, counter-clockwise from +x, axis (odd) and
# diagonal (even) directions (Sec. II, eq. "speeds").
C = ((0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1))
# Lattice weights (Sec. II, the equation after eq. "speeds").
W = (4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0,
     1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0)
CS2 = 1.0 / 3.0  # lattice speed of sound squared (Sec. II)


class Params:
    """Physical and numerical parameters of one run (Sec. II).

    tau: BGK relaxation time (omega = 1/tau, eq. "LBE").
    gamma: surface tension (eq. "pfilm").
    g: gravity in the hydrostatic term g h^2/2 of the equilibrium
       (eq. "SW_momentum_flux"); negative values destabilise (hanging film).
    hstar: precursor film thickness h_* (eq. "disjoiningP").
    n, m: disjoining exponents (eq. "disjoiningP").
    delta: slip length of the friction coefficient (eq. "alphafric").
    ax, ay: body acceleration, F = h (ax, ay) (eq. "force").
    """

    def __init__(self, tau=1.0, gamma=0.01, g=0.0, hstar=0.05, n=9, m=3,
                 delta=1.0, ax=0.0, ay=0.0):
        self.tau = float(tau)
        self.gamma = float(gamma)
        self.g = float(g)
        self.hstar = float(hstar)
        self.n = int(n)
        self.m = int(m)
        self.delta = float(delta)
        self.ax = float(ax)
        self.ay = float(ay)

    @property
    def omega(self):
        """Relaxation rate omega = dt/tau (Sec. II, after eq. "LBE")."""
        return 1.0 / self.tau

    @property
    def nu(self):
        """Kinematic viscosity nu = c_s^2 ((2 - omega)/(2 omega)) dt (Sec. II)."""
        w = self.omega
        return CS2 * (2.0 - w) / (2.0 * w)


def at_neighbour(phi, c):
    """Return psi with psi(x) = phi(x + c) on the periodic lattice."""
    return torch.roll(phi, shifts=(-c[1], -c[0]), dims=(-2, -1))


def equilibrium(h, ux, uy, g):
    """Shallow-water equilibria f_l^eq(h, u) (Sec. II, eq. "equilibria").

    Denominators read with lattice speed 1 (see the module docstring).
    Returns a list of 9 arrays.
    """
    usq = ux * ux + uy * uy
    feq = []
    for l, (cx, cy) in enumerate(C):
        cu = cx * ux + cy * uy
        if l == 0:
            feq.append(h - 5.0 * g * h * h / 6.0 - 2.0 * h * usq / 3.0)
        elif l % 2 == 1:
            feq.append(g * h * h / 6.0 + h * cu / 3.0 + h * cu * cu / 2.0 - h * usq / 6.0)
        else:
            feq.append(g * h * h / 24.0 + h * cu / 12.0 + h * cu * cu / 8.0 - h * usq / 24.0)
    return feq


def moments(f):
    """Height h = sum_l f_l and momentum h u = sum_l c_l f_l (Sec. II)."""
    h = f[0].clone()
    jx = torch.zeros_like(h)
    jy = torch.zeros_like(h)
    for l in range(1, 9):
        h = h + f[l]
    for l, (cx, cy) in enumerate(C):
        if cx != 0:
            jx = jx + cx * f[l]
        if cy != 0:
            jy = jy + cy * f[l]
    return h, jx, jy


def gradient(phi):
    """Isotropic gradient 3 sum_l w_l c_l phi(x + c_l) (Sec. II, eq. "derivative")."""
    gx = torch.zeros_like(phi)
    gy = torch.zeros_like(phi)
    for l, (cx, cy) in enumerate(C):
        if l == 0:
            continue
        nb = at_neighbour(phi, (cx, cy))
        if cx != 0:
            gx = gx + 3.0 * W[l] * cx * nb
        if cy != 0:
            gy = gy + 3.0 * W[l] * cy * nb
    return gx, gy


def laplacian(phi):
    """Isotropic Laplacian (Sec. II, eq. "n_laplace"), without the printed w_l:
    (1/6) [4 sum_odd phi(x + c_l) + sum_even phi(x + c_l) - 20 phi(x)]."""
    odd = torch.zeros_like(phi)
    even = torch.zeros_like(phi)
    for l in range(1, 9):
        nb = at_neighbour(phi, C[l])
        if l % 2 == 1:
            odd = odd + nb
        else:
            even = even + nb
    return (4.0 * odd + even - 20.0 * phi) / 6.0


def kappa(theta, p):
    """kappa = (1 - cos theta)(n - 1)(m - 1)/((n - m) h_*) (Sec. II, eq. "disjoiningP")."""
    return (1.0 - torch.cos(theta)) * ((p.n - 1) * (p.m - 1)) / ((p.n - p.m) * p.hstar)


def disjoining_shape(h, p):
    """f(h) = (h_*/h)^n - (h_*/h)^m (Sec. II, eq. "disjoiningP")."""
    r = p.hstar / h
    return r ** p.n - r ** p.m


def film_pressure(h, kap, p, gam=None):
    """p_film = -gamma (lap h + kappa f(h)) (Sec. II, eqs. "pfilm", "disjoiningP"),
    with the disjoining sign read as described in the module docstring;
    ``gam``, if given, is a per-site surface tension field used instead of
    p.gamma."""
    g = p.gamma if gam is None else gam
    return -g * (laplacian(h) + kap * disjoining_shape(h, p))


def friction_coefficient(h, delta):
    """alpha_delta(h) = 6 h / (2 h^2 + 6 delta h + 3 delta^2) (Sec. II, eq. "alphafric")."""
    return 6.0 * h / (2.0 * h * h + 6.0 * delta * h + 3.0 * delta * delta)


def total_force(h, ux, uy, kap, p, gam=None):
    """F_tot = F_film + F_fric + F (Sec. II, eq. "force").

    F_film = -h grad p_film (rho_0 = 1), F_fric = -nu alpha_delta(h) u
    (eq. "forcefric"), F = h (ax, ay); ``gam``: optional surface tension field.
    """
    pf = film_pressure(h, kap, p, gam)
    gpx, gpy = gradient(pf)
    alpha = friction_coefficient(h, p.delta)
    fx = -h * gpx - p.nu * alpha * ux + h * p.ax
    fy = -h * gpy - p.nu * alpha * uy + h * p.ay
    return fx, fy


def init(h0, p):
    """Initial populations: the equilibrium at rest, f_l = f_l^eq(h0, u = 0)."""
    z = torch.zeros_like(h0)
    return torch.stack(equilibrium(h0, z, z, p.g))


def step(f, kap, p, gam=None):
    """One time step of eq. "LBE" (Sec. II): BGK collision with forcing, then
    streaming f_l(x + c_l, t + 1) = post-collision f_l(x, t).

    ``f`` holds the pre-collision populations at time t, shape [9, ny, nx];
    ``gam``: optional per-site surface tension field (else p.gamma).
    """
    h, jx, jy = moments(f)
    ux = jx / h
    uy = jy / h
    fx, fy = total_force(h, ux, uy, kap, p, gam)
    feq = equilibrium(h, ux, uy, p.g)
    w = p.omega
    out = []
    for l, (cx, cy) in enumerate(C):
        source = (W[l] / CS2) * (cx * fx + cy * fy)
        post = f[l] + w * (feq[l] - f[l]) + source
        # streaming: the value at x moves to x + c_l
        out.append(torch.roll(post, shifts=(cy, cx), dims=(-2, -1)))
    return torch.stack(out)


def run(f, kap, p, nsteps, gam=None):
    """Apply ``step`` nsteps times."""
    for _ in range(int(nsteps)):
        f = step(f, kap, p, gam)
    return f


def readout(f):
    """h and u = (h u)/h from the populations (Sec. II)."""
    h, jx, jy = moments(f)
    return h, jx / h, jy / h


def mass(f):
    """Total film mass sum_{x,l} f_l(x), correctly rounded (math.fsum)."""
    return math.fsum(f.detach().reshape(-1).tolist())

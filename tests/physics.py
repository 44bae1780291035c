"""Closed forms and measurements used by the tests, derived independently of
both the oracle and the HIP path (the paper, Secs. II-III).

* ``lattice()``: D2Q9 velocities from the trigonometric formula of Sec. II
  (eq. "speeds") and the printed weights.
* ``fourier_step(k, ...)``: the 9 x 9 matrix that advances a single Fourier
  mode of the populations by one step of the linearised scheme about a flat
  film at rest, derived by hand from eqs. "LBE", "equilibria", "force",
  "pfilm", "disjoiningP", "forcefric", "derivative" and "n_laplace".
* ``contact_angle(h, hstar)``: spherical-cap angle from volume and apex
  height (Sec. III B).
* ``lubrication_growth(k, ...)``: thin-film growth rate of the hanging-film
  instability (Sec. III A, eq. "RTgrowth"), with the slip mobility implied by
  eq. "uslaved".
"""
import cmath
import math

import numpy as np


def lattice():
    """Velocities c_l (l = 0..8) and weights w_l of Sec. II."""
    c = [(0, 0)]
    for l in range(1, 9):
        scale = 1.0 if l % 2 == 1 else math.sqrt(2.0)
        ang = (l - 1) * math.pi / 4.0
        c.append((int(round(scale * math.cos(ang))), int(round(scale * math.sin(ang)))))
    w = [4.0 / 9.0] + [1.0 / 9.0 if l % 2 == 1 else 1.0 / 36.0 for l in range(1, 9)]
    return c, w


def laplacian_symbol(kx, ky):
    """Fourier symbol of the isotropic Laplacian read without the printed w_l."""
    return (8.0 * math.cos(kx) + 8.0 * math.cos(ky) + 4.0 * math.cos(kx) * math.cos(ky) - 20.0) / 6.0


def gradient_symbol(kx, ky):
    """Fourier symbol (complex 2-vector) of 3 sum_l w_l c_l phi(x + c_l)."""
    return (1j * math.sin(kx) * (2.0 + math.cos(ky)) / 3.0,
            1j * math.sin(ky) * (2.0 + math.cos(kx)) / 3.0)


def fourier_step(kx, ky, H, tau, gamma, g, kappa, hstar, n, m, delta):
    """One-step propagator of a population mode delta f_l(x) = a_l e^{i k.x}
    about the flat film h = H, u = 0 with uniform kappa.

    Derivation (linearising each term of Sec. II about h = H, u = 0):
      dh = sum_l a_l, dj = sum_l c_l a_l, du = dj / H;
      d feq_0 = (1 - 5 g H / 3) dh;
      d feq_l = (g H / 3) dh + c_l.dj / 3 (axis), (g H / 12) dh + c_l.dj / 12 (diagonal);
      d p = -gamma (L(k) + kappa f'(H)) dh with f'(h) = (-n r^n + m r^m)/h, r = h_*/h;
      d F = -H G(k) d p - nu alpha(H) du;
      post-collision: (1 - omega) a_l + omega d feq_l + 3 w_l c_l.dF;
      streaming multiplies population l by e^{-i k.c_l}.
    """
    c, w = lattice()
    omega = 1.0 / tau
    nu = (tau - 0.5) / 3.0
    alpha = 6.0 * H / (2.0 * H * H + 6.0 * delta * H + 3.0 * delta * delta)
    r = hstar / H
    fprime = (-n * r ** n + m * r ** m) / H
    dp_dh = -gamma * (laplacian_symbol(kx, ky) + kappa * fprime)
    Gx, Gy = gradient_symbol(kx, ky)
    A = np.zeros((9, 9), dtype=complex)
    for j in range(9):          # column: unit perturbation of population j
        a = np.zeros(9, dtype=complex)
        a[j] = 1.0
        dh = a.sum()
        djx = sum(c[l][0] * a[l] for l in range(9))
        djy = sum(c[l][1] * a[l] for l in range(9))
        dFx = -H * Gx * dp_dh * dh - nu * alpha * djx / H
        dFy = -H * Gy * dp_dh * dh - nu * alpha * djy / H
        for l in range(9):
            cx, cy = c[l]
            if l == 0:
                dfeq = (1.0 - 5.0 * g * H / 3.0) * dh
            elif l % 2 == 1:
                dfeq = (g * H / 3.0) * dh + (cx * djx + cy * djy) / 3.0
            else:
                dfeq = (g * H / 12.0) * dh + (cx * djx + cy * djy) / 12.0
            post = (1.0 - omega) * a[l] + omega * dfeq + 3.0 * w[l] * (cx * dFx + cy * dFy)
            A[l, j] = cmath.exp(-1j * (kx * cx + ky * cy)) * post
    return A


def slip_mobility(h, nu, delta):
    """M(h) = h^2/(nu alpha_delta(h)) = (h^3/3 + delta h^2 + delta^2 h/2)/nu."""
    return (h ** 3 / 3.0 + delta * h * h + delta * delta * h / 2.0) / nu


def lubrication_growth(k, h0, gabs, gamma, nu, delta):
    """sigma(k) = M(h0) k^2 (|g| - gamma k^2): eq. "RTgrowth" with the slip
    mobility (reduces to rho g h0^3/(3 mu) (k^2 - l_cap^2 k^4) for delta = 0)."""
    return slip_mobility(h0, nu, delta) * k * k * (gabs - gamma * k * k)


def contact_angle(h, hstar):
    """Spherical-cap angle from the drop volume V = sum(h - h_*) and apex height
    h_d = max h - h_*: r^2 = (6V/(pi h_d) - h_d^2)/3, R = (r^2 + h_d^2)/(2 h_d),
    theta = arcsin(r/R) (Sec. III B)."""
    hh = np.asarray(h, dtype=np.float64)
    V = float((hh - hstar).sum())
    hd = float(hh.max()) - hstar
    r2 = (6.0 * V / (math.pi * hd) - hd * hd) / 3.0
    R = (r2 + hd * hd) / (2.0 * hd)
    return math.asin(math.sqrt(r2) / R)

"""Seeded synthetic inputs: initial heights, contact-angle fields, parameter sets.

This module holds no arithmetic of the method itself.  It only draws seeded
random numbers and evaluates the geometric formulas of the initial
conditions, so that the oracle and the HIP path are fed bit-identical inputs.
Every array is float64, indexed [y, x].

The paper's workloads use no public dataset; these formulas stand in for its
experiments:
  * spherical-cap drop on a precursor film (Sec. III B, cap equation), used
    for the relaxing and the sliding drop;
  * a flat film with uniform noise (Sec. III A, Rayleigh-Taylor initial
    condition; Sec. III D, dewetting);
  * a striped contact-angle pattern standing in for the logo of the
    patterned-substrate showcase (Sec. III D), whose bitmap is not available.
"""
import math

import torch

F64 = torch.float64


def uniform_noise(ny, nx, seed):
    """U(-1, 1) field drawn from ``torch.Generator().manual_seed(seed)``."""
    gen = torch.Generator().manual_seed(int(seed))
    return torch.rand((ny, nx), generator=gen, dtype=F64) * 2.0 - 1.0


def noisy_film(ny, nx, mean, amplitude, seed):
    """h0 = mean + amplitude * U(-1, 1)."""
    return mean + amplitude * uniform_noise(ny, nx, seed)


def cap_radius(base_radius, apex):
    """Sphere radius of a cap with the given base radius and apex height."""
    return (base_radius * base_radius + apex * apex) / (2.0 * apex)


def apex_from_angle(base_radius, theta):
    """Apex height of a cap with base radius r and contact angle theta."""
    R = base_radius / math.sin(theta)
    return R * (1.0 - math.cos(theta))


def spherical_cap(ny, nx, base_radius, apex, hstar, cx=None, cy=None):
    """h0 = max(h_*, sqrt(R^2 - rho^2) - (R - apex)) on integer site coordinates,
    centred at (nx/2, ny/2) unless given (Sec. III B, cap equation)."""
    cx = nx // 2 if cx is None else cx
    cy = ny // 2 if cy is None else cy
    R = cap_radius(base_radius, apex)
    y = torch.arange(ny, dtype=F64).view(-1, 1) - cy
    x = torch.arange(nx, dtype=F64).view(1, -1) - cx
    rho2 = x * x + y * y
    inside = torch.clamp(R * R - rho2, min=0.0)
    cap = torch.sqrt(inside) - (R - apex)
    return torch.clamp(cap, min=hstar)


def _ramp(d, w):
    """0 for d <= -w/2, 1 for d >= w/2, (1 + sin(pi d / w))/2 in between."""
    mid = 0.5 * (1.0 + torch.sin(math.pi * d / w))
    return torch.where(d <= -w / 2, torch.zeros_like(d),
                       torch.where(d >= w / 2, torch.ones_like(d), mid))


def stripe_theta(ny, nx, theta_a, theta_b, period, width):
    """Stripes along x: theta_a on [0, P/2), theta_b on [P/2, P), edges
    smoothed by a sine ramp of the given width; periodic with period P."""
    u = torch.remainder(torch.arange(nx, dtype=F64), period)
    half = period / 2.0
    s = _ramp(u - half, width) - _ramp(u - period, width) + 1.0 - _ramp(u, width)
    row = theta_a + (theta_b - theta_a) * s
    return row.view(1, -1).expand(ny, nx).contiguous()


def smooth_noise(ny, nx, seed, length):
    """Seeded U(-1, 1) noise low-passed by a Gaussian of the given length,
    rescaled to unit maximum modulus (periodic, via the FFT)."""
    z = uniform_noise(ny, nx, seed)
    ky = torch.fft.fftfreq(ny, dtype=F64).view(-1, 1)
    kx = torch.fft.fftfreq(nx, dtype=F64).view(1, -1)
    filt = torch.exp(-2.0 * (math.pi * length) ** 2 * (kx * kx + ky * ky))
    s = torch.fft.ifft2(torch.fft.fft2(z) * filt).real
    return s / s.abs().max()


# ---------------------------------------------------------------------------
# Workloads.  Parameter keys: tau, gamma, g, hstar, n, m, delta, ax, ay.

BASE = dict(tau=1.0, gamma=0.01, g=0.0, hstar=0.05, n=9, m=3, delta=1.0, ax=0.0, ay=0.0)


def params(**kw):
    p = dict(BASE)
    p.update(kw)
    return p


def sessile_drop(n=64, base_radius=20.0, apex=8.0, hstar=0.05, theta=math.pi / 9):
    """Relaxing sessile drop, 64 x 64 by default: cap of base radius 20 and
    apex 8 on h_* = 0.05, uniform theta = pi/9, tau = 1, gamma = 0.01,
    (n, m) = (9, 3), delta = 1, no gravity."""
    p = params(hstar=hstar, delta=1.0)
    h0 = spherical_cap(n, n, base_radius, apex, hstar)
    th = torch.full((n, n), theta, dtype=F64)
    return p, h0, th


def lowpass(z, max_mode):
    """Keeps the Fourier modes of z with |mode number| <= max_mode in each
    direction (periodic), removes the rest."""
    ny, nx = z.shape
    my = torch.fft.fftfreq(ny, dtype=F64).view(-1, 1) * ny
    mx = torch.fft.fftfreq(nx, dtype=F64).view(1, -1) * nx
    keep = (my.abs() <= max_mode) & (mx.abs() <= max_mode)
    return torch.fft.ifft2(torch.fft.fft2(z) * keep).real


def rayleigh_taylor(n=512, seed=1, g=-1.0e-4, delta=0.5, max_mode=None):
    """Hanging film: h0 = 1 + 1e-3 U(-1, 1), g = -1e-4 (destabilising),
    gamma = 0.01, tau = 1, delta = 0.5, no wetting term (theta = 0).
    With max_mode set, the noise keeps only Fourier modes up to that mode
    number (the checkerboard mode of the scheme is unstable for g < 0 and
    would otherwise grow from the initial noise)."""
    p = params(g=g, delta=delta)
    z = uniform_noise(n, n, seed)
    if max_mode is not None:
        z = lowpass(z, max_mode)
    h0 = 1.0 + 1.0e-3 * z
    th = torch.zeros((n, n), dtype=F64)
    return p, h0, th


def sliding_drop(nx=1024, ny=512, bond=0.1, delta=1.0, base_radius=40.0,
                 theta=math.pi / 6, hstar=0.05):
    """Drop on an incline: cap with base radius 40 and contact angle pi/6 on
    h_* = 0.05, body acceleration along x set by the Bond number
    Bo = (3V/4 pi)^(2/3) a / gamma with V = sum(h0 - h_*)."""
    apex = apex_from_angle(base_radius, theta)
    h0 = spherical_cap(ny, nx, base_radius, apex, hstar)
    vol = float((h0 - hstar).sum())
    a = bond * 0.01 / (3.0 * vol / (4.0 * math.pi)) ** (2.0 / 3.0)
    p = params(hstar=hstar, delta=delta, ax=a)
    th = torch.full((ny, nx), theta, dtype=F64)
    return p, h0, th


def patterned_dewetting(n=4096, seed=2, hstar=0.09):
    """Flat film h0 = 0.1 + 1e-4 U(-1, 1) on stripes of period 256 alternating
    pi/9 and pi/4 with sine-smoothed edges of width 8; gamma = 0.01, tau = 1,
    delta = 1.  h_* = 0.09 keeps the flat film linearly stable at grid scale."""
    p = params(hstar=hstar, delta=1.0)
    h0 = noisy_film(n, n, 0.1, 1.0e-4, seed)
    th = stripe_theta(n, n, math.pi / 9, math.pi / 4, 256, 8.0)
    return p, h0, th


def inverse_design(n=512, seed=3, target_seed=4, hstar=0.09):
    """Adjoint test case: the dewetting recipe at n x n with theta = pi/6
    everywhere (the design variable's starting point) and a seeded smooth
    target height 0.1 + 0.01 s(x), s smooth noise of length n/16."""
    p = params(hstar=hstar, delta=1.0)
    h0 = noisy_film(n, n, 0.1, 1.0e-4, seed)
    th = torch.full((n, n), math.pi / 6, dtype=F64)
    target = 0.1 + 0.01 * smooth_noise(n, n, target_seed, n / 16.0)
    return p, h0, th, target


def stripe_recovery(n=128, seed=5, hstar=0.095, period=32):
    """Twin experiment for the inverse-design loop: flat film h0 = 0.1 +
    1e-4 U(-1, 1) on h_* = 0.095 (thin enough, h0 < 1.2 h_*, that the film is
    spinodally stable and its response to theta is smooth), gamma = 0.01,
    tau = 1, delta = 1, and the true pattern: stripes of period 32 alternating
    pi/9 and pi/4 with sine ramps of width 4."""
    p = params(hstar=hstar, delta=1.0)
    h0 = noisy_film(n, n, 0.1, 1.0e-4, seed)
    th = stripe_theta(n, n, math.pi / 9, math.pi / 4, period, 4.0)
    return p, h0, th


def random_pixels(ny, nx, count, seed):
    """``count`` distinct seeded (y, x) sites."""
    gen = torch.Generator().manual_seed(int(seed))
    idx = torch.randperm(ny * nx, generator=gen)[:count]
    return [(int(i) // nx, int(i) % nx) for i in idx]

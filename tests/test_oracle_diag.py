"""Pins of the term-balance diagnostic oracle (appendix, eq. "magnitude").

Single Fourier modes on a periodic lattice have closed-form stencil values:
the isotropic derivative of sin(kx) is sin(k) cos(kx) and of cos(kx) is
-sin(k) sin(kx); the Laplacian of either is 2 (cos k - 1) times it (both
exact for modes along x).  The state is the equilibrium of (h, j), whose
moments are exactly h and j.  Each term's norm is then known in closed form,
so a dropped factor, a wrong sign between the two viscous terms, or a wrong
component fails one of these tests.
"""
import math

import pytest
import torch

from oracle import diag, lbm

F64 = torch.float64
N = 32


def mode_state(h0, a, b, m, transpose=False, g=0.0):
    """Populations with h = h0 + a cos(kx), j_x = b sin(kx), j_y = 0,
    k = 2 pi m / N (or the same along y with transpose)."""
    k = 2.0 * math.pi * m / N
    x = torch.arange(N, dtype=F64).view(1, -1).expand(N, N)
    if transpose:
        x = x.t()
    h = h0 + a * torch.cos(k * x)
    j = b * torch.sin(k * x)
    zero = torch.zeros_like(h)
    ux, uy = (zero, j / h) if transpose else (j / h, zero)
    return torch.stack(lbm.equilibrium(h, ux, uy, g)), k


P = lbm.Params(tau=0.8, gamma=0.02, hstar=0.1, delta=0.7)
KAP0 = torch.zeros((N, N), dtype=F64)


@pytest.mark.parametrize("m", [1, 3])
def test_pressure_term_closed_form(m):
    """kappa = 0, j = 0: -h d_x p with p = -gamma lap h: norm
    |2 gamma (cos k - 1) a sin k| (h0^2/2 + a^2/8)^(1/2)."""
    h0, a = 0.5, 0.05
    f, k = mode_state(h0, a, 0.0, m)
    t = diag.term_norms(f, KAP0, P)
    c = 2.0 * P.gamma * (math.cos(k) - 1.0) * a * math.sin(k)
    assert t["pressure_x"] == pytest.approx(abs(c) * math.sqrt(h0 * h0 / 2 + a * a / 8), rel=1e-12)
    assert t["pressure_y"] < 1e-15
    assert t["friction_x"] == 0.0 and t["viscous_x"] == 0.0 and t["advection_x"] == 0.0


@pytest.mark.parametrize("m", [1, 2, 5])
def test_friction_viscous_advection_closed_forms(m):
    """Uniform h0, j_x = b sin(kx): friction nu alpha(h0) |b| / (h0 sqrt 2);
    viscous nu |b| |2 (cos k - 1) - 2 sin^2 k| / sqrt 2 (the Laplacian and
    twice the x derivative of the divergence add with the same sign);
    advection (b^2 / (2 h0)) |sin 2k| / sqrt 2."""
    h0, b = 0.4, 0.01
    f, k = mode_state(h0, 0.0, b, m)
    t = diag.term_norms(f, KAP0, P)
    alpha = 6 * h0 / (2 * h0 * h0 + 6 * P.delta * h0 + 3 * P.delta ** 2)
    assert t["friction_x"] == pytest.approx(P.nu * alpha * b / (h0 * math.sqrt(2)), rel=1e-12)
    visc = P.nu * b * abs(2 * (math.cos(k) - 1) - 2 * math.sin(k) ** 2) / math.sqrt(2)
    assert t["viscous_x"] == pytest.approx(visc, rel=1e-12)
    adv = b * b / (2 * h0) * abs(math.sin(2 * k)) / math.sqrt(2)
    assert t["advection_x"] == pytest.approx(adv, rel=1e-12)
    assert t["pressure_x"] < 1e-16
    for name in ("pressure_y", "friction_y", "viscous_y", "advection_y"):
        assert t[name] < 1e-16


def test_y_components_are_the_transposed_x_components():
    f, _ = mode_state(0.45, 0.03, 0.008, 2)
    ft, _ = mode_state(0.45, 0.03, 0.008, 2, transpose=True)
    tx = diag.term_norms(f, KAP0, P)
    ty = diag.term_norms(ft, KAP0, P)
    for name in ("pressure", "friction", "viscous", "advection"):
        assert ty[name + "_y"] == pytest.approx(tx[name + "_x"], rel=1e-12)
        assert ty[name + "_x"] < 1e-15


def test_disjoining_enters_the_pressure_term():
    """Uniform kappa changes the pressure term by -h d_x(-gamma kappa f(h)),
    nothing else; with a = 0 (flat film) the pressure term vanishes."""
    f, _ = mode_state(0.3, 0.02, 0.0, 1)
    kap = torch.full((N, N), 5.0, dtype=F64)
    with_k = diag.term_fields(f, kap, P)["pressure_x"]
    without = diag.term_fields(f, KAP0, P)["pressure_x"]
    h, _, _ = lbm.moments(f)
    dfx, _ = lbm.gradient(-P.gamma * kap * lbm.disjoining_shape(h, P))
    assert torch.allclose(with_k - without, -h * dfx, rtol=0, atol=1e-15)
    flat, _ = mode_state(0.3, 0.0, 0.0, 1)
    assert diag.term_norms(flat, kap, P)["pressure_x"] < 1e-16

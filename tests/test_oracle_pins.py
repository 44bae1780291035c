"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks one part of ``oracle.lbm`` against something other than its
own formula: moment identities (Sec. II), closed-form stencil values and
Fourier symbols (eqs. "derivative", "n_laplace"), exact discrete recurrences
(uniform films), a hand-derived Fourier propagator of the linearised step
(``tests/physics.py``), the disjoining integral (eq. "disjoiningP") and
mass invariance (Sec. III B, mass conservation of the method).
"""
import math

import numpy as np
import pytest
import torch

from oracle import lbm
from physics import fourier_step, gradient_symbol, lattice, laplacian_symbol

F64 = torch.float64


def rand(shape, lo, hi, seed):
    g = torch.Generator().manual_seed(seed)
    return lo + (hi - lo) * torch.rand(shape, generator=g, dtype=F64)


def test_lattice_matches_paper_formula():
    c, w = lattice()
    assert tuple(c) == lbm.C
    assert np.allclose(w, lbm.W, rtol=0, atol=1e-17)
    assert math.isclose(sum(lbm.W), 1.0, rel_tol=1e-15)
    # second and fourth moments of the weights: isotropy of D2Q9 with c_s^2 = 1/3
    for a in range(2):
        for b in range(2):
            s = sum(wl * cl[a] * cl[b] for wl, cl in zip(lbm.W, lbm.C))
            assert math.isclose(s, (1.0 / 3.0) * (a == b), abs_tol=1e-16)


@pytest.mark.parametrize("g", [0.0, 1.0e-4, -1.0e-4, 0.3])
def test_equilibrium_moments(g):
    """Sum f^eq = h, sum c f^eq = h u, sum c c f^eq = g h^2/2 I + h u u (Sec. II)."""
    h = rand((50,), 0.05, 10.0, 1)
    ux = rand((50,), -0.1, 0.1, 2)
    uy = rand((50,), -0.1, 0.1, 3)
    feq = lbm.equilibrium(h, ux, uy, g)
    c, _ = lattice()
    m0 = sum(feq)
    mx = sum(c[l][0] * feq[l] for l in range(9))
    my = sum(c[l][1] * feq[l] for l in range(9))
    mxx = sum(c[l][0] * c[l][0] * feq[l] for l in range(9))
    myy = sum(c[l][1] * c[l][1] * feq[l] for l in range(9))
    mxy = sum(c[l][0] * c[l][1] * feq[l] for l in range(9))
    tol = dict(rtol=1e-14, atol=1e-15)
    torch.testing.assert_close(m0, h, **tol)
    torch.testing.assert_close(mx, h * ux, **tol)
    torch.testing.assert_close(my, h * uy, **tol)
    torch.testing.assert_close(mxx, 0.5 * g * h * h + h * ux * ux, **tol)
    torch.testing.assert_close(myy, 0.5 * g * h * h + h * uy * uy, **tol)
    torch.testing.assert_close(mxy, h * ux * uy, **tol)


def test_literal_equilibrium_denominators_break_moments():
    """Negative control for the reading of eq. "equilibria": with c_s^2 = 1/3
    taken literally in the denominators the momentum moment becomes 3 h u."""
    cs2 = 1.0 / 3.0
    h, ux, uy = 2.0, 0.01, -0.02
    c, _ = lattice()
    mx = 0.0
    for l in range(1, 9):
        cu = c[l][0] * ux + c[l][1] * uy
        usq = ux * ux + uy * uy
        if l % 2 == 1:
            fl = h * cu / (3 * cs2) + h * cu * cu / (2 * cs2 * cs2) - h * usq / (6 * cs2)
        else:
            fl = h * cu / (12 * cs2) + h * cu * cu / (8 * cs2 * cs2) - h * usq / (24 * cs2)
        mx += c[l][0] * fl
    assert math.isclose(mx, 3.0 * h * ux, rel_tol=1e-12)


def test_stencils_on_polynomials():
    """grad(x) = (1, 0); lap(const) = 0; lap(x^2) = 2; lap(x^2 + y^2) = 4; lap(xy) = 0,
    checked away from the periodic wrap."""
    ny, nx = 12, 16
    y = torch.arange(ny, dtype=F64).view(-1, 1).expand(ny, nx)
    x = torch.arange(nx, dtype=F64).view(1, -1).expand(ny, nx)
    inner = (slice(2, ny - 2), slice(2, nx - 2))
    const = torch.full((ny, nx), 3.7, dtype=F64)
    assert lbm.laplacian(const).abs().max() < 1e-14
    gx, gy = lbm.gradient(x)
    torch.testing.assert_close(gx[inner], torch.ones_like(gx[inner]), rtol=0, atol=1e-14)
    torch.testing.assert_close(gy[inner], torch.zeros_like(gy[inner]), rtol=0, atol=1e-14)
    gx, gy = lbm.gradient(x * y)
    torch.testing.assert_close(gx[inner], y[inner], rtol=0, atol=1e-13)
    torch.testing.assert_close(gy[inner], x[inner], rtol=0, atol=1e-13)
    for field, val in ((x * x, 2.0), (x * x + y * y, 4.0), (x * y, 0.0)):
        lap = lbm.laplacian(field)[inner]
        torch.testing.assert_close(lap, torch.full_like(lap, val), rtol=0, atol=1e-12)


@pytest.mark.parametrize("mx,my", [(1, 0), (2, 3), (5, 1), (7, 7)])
def test_stencil_fourier_symbols(mx, my):
    """Plane waves are eigenfunctions with the symbols derived in tests/physics.py."""
    n = 16
    kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
    y = torch.arange(n, dtype=F64).view(-1, 1)
    x = torch.arange(n, dtype=F64).view(1, -1)
    phase = kx * x + ky * y
    cosw, sinw = torch.cos(phase), torch.sin(phase)
    lam = laplacian_symbol(kx, ky)
    torch.testing.assert_close(lbm.laplacian(cosw), lam * cosw, rtol=0, atol=1e-13)
    sx, sy = gradient_symbol(kx, ky)
    gx, gy = lbm.gradient(cosw)
    # grad cos = Re(i s e^{i k.x}) = -Im(s) sin
    torch.testing.assert_close(gx, -sx.imag * sinw, rtol=0, atol=1e-13)
    torch.testing.assert_close(gy, -sy.imag * sinw, rtol=0, atol=1e-13)


def test_laplacian_isotropic_to_fourth_order():
    """The k^4 error of the Laplacian symbol is isotropic: -k^2 + k^4/12 + O(k^6)."""
    for k in (0.05, 0.1):
        for ang in (0.0, math.pi / 8, math.pi / 4):
            s = laplacian_symbol(k * math.cos(ang), k * math.sin(ang))
            assert abs(s - (-k * k + k ** 4 / 12.0)) < 0.01 * k ** 6


@pytest.mark.parametrize("n,m", [(9, 3), (3, 6), (2, 3), (4, 10)])
def test_disjoining_integral_and_symmetry(n, m):
    """Pi(h_*) = 0; integral_{h*}^inf kappa f dh = -(1 - cos theta) for the
    paper's exponent pairs (Sec. II, after eq. "disjoiningP"): with kappa's
    normalisation (n-1)(m-1)/((n-m) h_*) the integral is
    kappa h_* (1/(n-1) - 1/(m-1)) = -(1 - cos theta) for any n, m > 1;
    (n, m) <-> (m, n) leaves kappa f unchanged."""
    for theta in (math.pi / 9, math.pi / 6, math.pi / 4):
        p = lbm.Params(hstar=0.05, n=n, m=m)
        q = lbm.Params(hstar=0.05, n=m, m=n)
        th = torch.tensor(theta, dtype=F64)
        kp, kq = lbm.kappa(th, p), lbm.kappa(th, q)
        h = torch.linspace(0.02, 3.0, 200, dtype=F64)
        torch.testing.assert_close(kp * lbm.disjoining_shape(h, p), kq * lbm.disjoining_shape(h, q),
                                   rtol=1e-13, atol=1e-13)
        assert float(lbm.disjoining_shape(torch.tensor(0.05, dtype=F64), p)) == 0.0
        # substitute h = h_*/s: dh = h_*/s^2 ds, s in (0, 1]
        s = torch.linspace(0.0, 1.0, 200001, dtype=F64)[1:]
        hh = p.hstar / s
        integrand = kp * lbm.disjoining_shape(hh, p) * p.hstar / (s * s)
        # the first interval [0, s_1] is not sampled (h = infinity); for n = 2 the
        # integrand is finite there, so add it as a rectangle (error O(s_1^2))
        val = float(torch.trapezoid(integrand, s)) + float(s[0] * integrand[0])
        assert math.isclose(val, -(1.0 - math.cos(theta)), rel_tol=1e-6)


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_mass_invariant(tau):
    """Total mass is unchanged by the step (Sec. III B): FP64 drift <= 1e-13."""
    ny, nx = 20, 24
    p = lbm.Params(tau=tau, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ax=1e-5, ay=-2e-5)
    h0 = rand((ny, nx), 0.3, 0.6, 7)
    th = rand((ny, nx), 0.2, 0.6, 8)
    f = lbm.init(h0, p)
    m0 = lbm.mass(f)
    f = lbm.run(f, lbm.kappa(th, p), p, 1500)
    assert abs(lbm.mass(f) - m0) <= 1e-13 * abs(m0)
    assert math.isclose(m0, math.fsum(h0.reshape(-1).tolist()), rel_tol=1e-15)


@pytest.mark.parametrize("tau,delta", [(1.0, 1.0), (0.7, 0.5), (1.6, 2.0)])
def test_uniform_film_recurrence(tau, delta):
    """Uniform h, uniform u0, body force a: no pressure gradient, so
    u_{t+1} = u_t (1 - nu alpha/h) + a exactly, i.e.
    u_t = u_inf + (u0 - u_inf)(1 - nu alpha/h)^t, u_inf = a (2h^2 + 6 delta h + 3 delta^2)/(6 nu)."""
    H, u0x, u0y, ax, ay = 0.8, 2e-3, -1e-3, 3e-6, 1e-6
    p = lbm.Params(tau=tau, gamma=0.01, g=1e-4, hstar=0.05, delta=delta, ax=ax, ay=ay)
    n = 6
    h = torch.full((n, n), H, dtype=F64)
    f = torch.stack(lbm.equilibrium(h, torch.full_like(h, u0x), torch.full_like(h, u0y), p.g))
    kap = lbm.kappa(torch.full((n, n), 0.3, dtype=F64), p)
    nu = (tau - 0.5) / 3.0
    decay = 1.0 - nu * 6.0 / (2 * H * H + 6 * delta * H + 3 * delta * delta)
    uinf = [a * (2 * H * H + 6 * delta * H + 3 * delta * delta) / (6 * nu) for a in (ax, ay)]
    for t in range(1, 41):
        f = lbm.step(f, kap, p)
        if t % 10 == 0:
            hh, ux, uy = lbm.readout(f)
            for comp, u0, ui in ((ux, u0x, uinf[0]), (uy, u0y, uinf[1])):
                expect = ui + (u0 - ui) * decay ** t
                torch.testing.assert_close(comp, torch.full_like(comp, expect), rtol=1e-12, atol=1e-17)
            torch.testing.assert_close(hh, torch.full_like(hh, H), rtol=1e-14, atol=0)


@pytest.mark.parametrize("tau,g", [(1.0, 0.0), (0.75, 0.0), (1.0, -1e-4), (1.3, 2e-3)])
def test_flat_film_is_fixed_point(tau, g):
    """A flat film at rest with uniform theta stays flat and at rest."""
    p = lbm.Params(tau=tau, g=g, hstar=0.05)
    h0 = torch.full((8, 10), 0.37, dtype=F64)
    kap = lbm.kappa(torch.full_like(h0, 0.5), p)
    f0 = lbm.init(h0, p)
    f = lbm.run(f0, kap, p, 200)
    # Not bitwise: the signed sum of the gradient stencil over a constant
    # pressure leaves a residue of order 1e-17 |p|, and with g != 0 the sum of
    # E_l(h) differs from h by an ulp.  On a uniform film every site rounds the
    # same way, so h may drift by a few ulp per step; u stays at rest.
    steps = 200
    h, ux, uy = lbm.readout(f)
    torch.testing.assert_close(h, h0, rtol=4 * steps * 2.0 ** -52, atol=0)
    assert float(ux.abs().max()) < 1e-18 and float(uy.abs().max()) < 1e-18
    torch.testing.assert_close(f, f0, rtol=0, atol=4 * steps * 2.0 ** -52 * 0.37)


@pytest.mark.parametrize("case", ["drop", "rt", "slip"])
def test_single_mode_follows_fourier_propagator(case):
    """A small single-mode perturbation evolves as the hand-derived linear
    propagator of tests/physics.py predicts, to nonlinearity O(eps)."""
    n = 16
    mx, my = 2, 1
    if case == "drop":
        H, par, theta = 0.3, dict(tau=1.0, gamma=0.01, g=0.0, hstar=0.1, delta=1.0), 0.6
    elif case == "rt":
        H, par, theta = 1.0, dict(tau=0.9, gamma=0.01, g=-1e-3, hstar=0.05, delta=0.5), 0.0
    else:
        H, par, theta = 0.5, dict(tau=1.4, gamma=0.05, g=2e-3, hstar=0.2, delta=2.0), 0.9
    p = lbm.Params(**par)
    kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
    eps = 1e-7
    y = torch.arange(n, dtype=F64).view(-1, 1)
    x = torch.arange(n, dtype=F64).view(1, -1)
    h0 = H * (1.0 + eps * torch.cos(kx * x + ky * y))
    th = torch.full((n, n), theta, dtype=F64)
    kap = float(lbm.kappa(torch.tensor(theta, dtype=F64), p))
    f = lbm.init(h0, p)
    base = lbm.init(torch.full((n, n), H, dtype=F64), p)
    # initial mode amplitudes: projection of f - base on e^{i k.x}
    def amp(field):
        return complex(np.fft.fft2(field.numpy())[my, mx]) / (n * n)
    a = np.array([amp(f[l] - base[l]) for l in range(9)])
    A = fourier_step(kx, ky, H, p.tau, p.gamma, p.g, kap, p.hstar, p.n, p.m, p.delta)
    steps = 60
    f = lbm.run(f, lbm.kappa(th, p), p, steps)
    pred = np.linalg.matrix_power(A, steps) @ a
    got = np.array([amp(f[l] - base[l]) for l in range(9)])
    scale = np.abs(a).max()
    assert np.abs(got - pred).max() <= 1e-5 * scale
    # the height mode itself
    assert abs(got.sum() - pred.sum()) <= 1e-5 * abs(a.sum())


def _lead_rate(k, H, tau, gamma, g, delta):
    ev = np.linalg.eigvals(fourier_step(k, 0.0, H, tau, gamma, g, 0.0, 0.05, 9, 3, delta))
    return math.log(abs(ev[np.argmin(np.abs(np.abs(ev) - 1.0))]))


@pytest.mark.parametrize("tau", [0.55, 0.7, 1.0])
def test_fourier_propagator_matches_corrected_lubrication_growth(tau):
    """The slowest mode of the linearised scheme grows at the thin-film rate of
    eq. "RTgrowth" (slip mobility M(h) = h^2/(nu alpha), eq. "uslaved"), with two
    corrections the discrete scheme carries: the longitudinal viscous factor
    1/(1 + 3 k^2 h/alpha) (eq. "hydro2") and the half-step force in the mass
    flux of the plain forcing term, -|g| h k^2 / 2.  Agreement within 1% over
    the unstable band up to the fastest mode."""
    from physics import slip_mobility
    H, gamma, g, delta = 1.0, 0.01, -1e-4, 0.5
    nu = (tau - 0.5) / 3.0
    alpha = 6 * H / (2 * H * H + 6 * delta * H + 3 * delta * delta)
    for k in (0.005, 0.02, 0.04, 0.0707):
        sig = k * k * (slip_mobility(H, nu, delta) * (abs(g) - gamma * k * k)
                       / (1.0 + 3.0 * k * k * H / alpha) - abs(g) * H / 2.0)
        assert abs(_lead_rate(k, H, tau, gamma, g, delta) / sig - 1.0) < 0.01


def test_fourier_propagator_tends_to_lubrication_law():
    """As tau -> 1/2 the half-step correction vanishes (the viscous factor,
    independent of nu, stays): at tau = 0.52 the scheme reproduces
    eq. "RTgrowth" times 1/(1 + 3 k^2 h/alpha) within 1% up to the fastest
    mode, and the neutral wavenumber is k_c = sqrt(|g|/gamma) within 1%."""
    from physics import lubrication_growth
    H, tau, gamma, g, delta = 1.0, 0.52, 0.01, -1e-4, 0.5
    nu = (tau - 0.5) / 3.0
    alpha = 6 * H / (2 * H * H + 6 * delta * H + 3 * delta * delta)
    for k in (0.005, 0.02, 0.04, 0.0707):
        sig = lubrication_growth(k, H, abs(g), gamma, nu, delta) / (1.0 + 3.0 * k * k * H / alpha)
        assert abs(_lead_rate(k, H, tau, gamma, g, delta) / sig - 1.0) < 0.01
    lo, hi = 0.05, 0.15
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if _lead_rate(mid, H, tau, gamma, g, delta) > 0:
            lo = mid
        else:
            hi = mid
    assert abs(lo / math.sqrt(abs(g) / gamma) - 1.0) < 0.01


def test_checkerboard_mode_unstable_for_negative_gravity():
    """The checkerboard mode k = (pi, pi) is invisible to the isotropic
    gradient stencil (its symbol vanishes there), so the capillary pressure
    cannot restore it, while a negative g in the equilibrium drives it through
    streaming: the linearised scheme grows it by about 1 + 2.7|g| per step
    (1.000267 at g = -1e-4), far faster than the thin-film instability
    (1.4e-6 per step at the fastest mode).  For g >= 0 it is neutral or damped.
    The oracle follows the propagator on this mode."""
    from physics import gradient_symbol
    sx, sy = gradient_symbol(math.pi, math.pi)
    assert abs(sx) < 1e-15 and abs(sy) < 1e-15
    for g, unstable in ((-1e-4, True), (-1e-3, True), (0.0, False), (1e-3, False)):
        A = fourier_step(math.pi, math.pi, 1.0, 1.0, 0.01, g, 0.0, 0.05, 9, 3, 0.5)
        lam = np.abs(np.linalg.eigvals(A)).max()
        assert (lam > 1.0 + 1e-9) == unstable, (g, lam)
        if unstable:
            assert abs((lam - 1.0) / abs(g) - 2.667) < 0.05
    # oracle on an 8 x 8 lattice: the checkerboard amplitude of h after 300 steps
    n, g, steps, eps = 8, -1e-3, 300, 1e-7
    p = lbm.Params(tau=1.0, gamma=0.01, g=g, hstar=0.05, delta=0.5)
    y = torch.arange(n, dtype=F64).view(-1, 1)
    x = torch.arange(n, dtype=F64).view(1, -1)
    cb = torch.cos(math.pi * (x + y))
    h0 = 1.0 + eps * cb
    f = lbm.init(h0, p)
    base = lbm.init(torch.ones((n, n), dtype=F64), p)
    amp0 = np.array([float(((f[l] - base[l]) * cb).mean()) for l in range(9)])
    A = fourier_step(math.pi, math.pi, 1.0, 1.0, 0.01, g, 0.0, 0.05, 9, 3, 0.5)
    pred = (np.linalg.matrix_power(A, steps) @ amp0).real
    f = lbm.run(f, lbm.kappa(torch.zeros((n, n), dtype=F64), p), p, steps)
    got = np.array([float(((f[l] - base[l]) * cb).mean()) for l in range(9)])
    assert np.abs(got - pred).max() <= 1e-5 * np.abs(pred).max()
    assert abs(got.sum()) > 1.5 * abs(amp0.sum())  # the h mode has grown


# ---- position-dependent surface tension (Sec. II, after eq. "n_laplace") -------

def _gamma_case(nx=48, ny=6):
    x = torch.arange(nx, dtype=torch.float64).view(1, -1).expand(ny, nx)
    return x


def test_uniform_gamma_field_equals_scalar_gamma():
    """A surface tension field equal to gamma everywhere is the scalar path,
    bit for bit, for a random state with a kappa field."""
    g = torch.Generator().manual_seed(71)
    ny, nx = 9, 13
    p = lbm.Params(tau=0.9, gamma=0.013, g=1e-3, hstar=0.1, delta=1.0, ax=1e-5)
    h0 = 0.3 + 0.3 * torch.rand((ny, nx), generator=g, dtype=torch.float64)
    th = 0.2 + 0.5 * torch.rand((ny, nx), generator=g, dtype=torch.float64)
    f = lbm.run(lbm.init(h0, p), lbm.kappa(th, p), p, 3)
    a = lbm.step(f, lbm.kappa(th, p), p)
    b = lbm.step(f, lbm.kappa(th, p), p, torch.full((ny, nx), 0.013, dtype=torch.float64))
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", [1, 5])
def test_gamma_field_on_flat_film_gives_closed_form_force(mode):
    """Flat film h0 at rest with uniform kappa under gamma(x) = gamma0 (1 +
    eps cos(q x)): the Laplacian vanishes, p = -gamma(x) kappa f(h0), and the
    isotropic gradient stencil maps cos(q x) to -sin(q) sin(q x) (its symbol
    for a field varying along x only), so F_x = -h0 gamma0 kappa f(h0) eps
    sin(q) sin(q x) and F_y = 0.  A reading where gamma(x) multiplies the
    Laplacian only would give no force here."""
    nx, ny = 48, 6
    p = lbm.Params(tau=1.0, gamma=0.0, hstar=0.1, delta=1.0)
    h0, g0, eps = 0.3, 0.02, 0.25
    q = 2.0 * math.pi * mode / nx
    x = _gamma_case(nx, ny)
    gam = g0 * (1.0 + eps * torch.cos(q * x))
    kap = lbm.kappa(torch.full((ny, nx), 0.6, dtype=torch.float64), p)
    h = torch.full((ny, nx), h0, dtype=torch.float64)
    z = torch.zeros_like(h)
    fx, fy = lbm.total_force(h, z, z, kap, p, gam)
    r = p.hstar / h0
    f0 = r ** 9 - r ** 3
    want = -h0 * g0 * float(kap[0, 0]) * f0 * eps * math.sin(q) * torch.sin(q * x)
    assert float((fx - want).abs().max()) <= 1e-13 * float(want.abs().max())
    assert float(fy.abs().max()) <= 1e-18


@pytest.mark.parametrize("k_mode,q_mode", [(1, 3), (4, 1)])
def test_gamma_field_capillary_pressure_product(k_mode, q_mode):
    """No disjoining term (theta = 0), h = h0 + a sin(k x), gamma(x) = gamma0
    (1 + eps cos(q x)).  The Laplacian stencil maps sin(k x) to 2 (cos k - 1)
    sin(k x) (its symbol along x), so p = -gamma0 L a [sin(k x) + eps/2
    (sin((k+q) x) + sin((k-q) x))], L = 2 (cos k - 1); the gradient stencil
    maps sin(K x) to sin(K) cos(K x), which gives F_x = -h(x) d_x p in closed
    form."""
    nx, ny = 60, 5
    p = lbm.Params(tau=1.0, gamma=0.0, hstar=0.1, delta=1.0)
    h0, a, g0, eps = 0.5, 0.01, 0.01, 0.3
    k = 2.0 * math.pi * k_mode / nx
    q = 2.0 * math.pi * q_mode / nx
    x = _gamma_case(nx, ny)
    h = h0 + a * torch.sin(k * x)
    gam = g0 * (1.0 + eps * torch.cos(q * x))
    z = torch.zeros_like(h)
    fx, fy = lbm.total_force(h, z, z, torch.zeros_like(h), p, gam)
    L = 2.0 * (math.cos(k) - 1.0)
    dpx = -g0 * L * a * (math.sin(k) * torch.cos(k * x)
                         + 0.5 * eps * (math.sin(k + q) * torch.cos((k + q) * x)
                                        + math.sin(k - q) * torch.cos((k - q) * x)))
    want = -h * dpx
    # the Laplacian cancels terms of size h0 to leave L a: rounding of order
    # 2^-52 h0 / |L a| relative (1e-11 here); a dropped or misplaced gamma(x)
    # factor changes F_x by a fraction eps of itself
    tol = 100 * 2.0 ** -52 * h0 / abs(L * a)
    assert float((fx - want).abs().max()) <= tol * float(want.abs().max())
    assert float(fy.abs().max()) <= 1e-18

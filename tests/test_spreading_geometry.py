"""Cap geometry of the spreading tracker (paper_1810_07642_amd/spreading.py)
on exact spherical caps sampled on the lattice: base radius, apex height and
contact angle recovered within the lattice discretisation (CPU only)."""
import math

import pytest

from paper_1810_07642_amd import inputs
from paper_1810_07642_amd.spreading import cap_geometry


@pytest.mark.parametrize("rb,theta", [(40.0, math.pi / 6), (60.0, math.pi / 12), (25.0, math.pi / 4)])
def test_cap_geometry_recovers_the_cap(rb, theta):
    hstar = 0.5
    apex = inputs.apex_from_angle(rb, theta)
    h = inputs.spherical_cap(256, 256, rb, apex, hstar)
    r, hd, th, R = cap_geometry(h, hstar)
    # the sampled cap is clipped at h_*: above the precursor it is the cap of
    # the same sphere cut at height h_*, base radius rho* and angle arcsin(rho*/R_s)
    Rs = inputs.cap_radius(rb, apex)
    rho = math.sqrt(Rs * Rs - (Rs - apex + hstar) ** 2)
    assert hd == pytest.approx(apex - hstar, rel=1e-9)
    assert r == pytest.approx(rho, rel=0.005)
    assert R == pytest.approx(Rs, rel=0.01)
    assert th == pytest.approx(math.asin(rho / Rs), rel=0.01)


def test_cap_geometry_needs_a_drop():
    import torch
    with pytest.raises(ValueError):
        cap_geometry(torch.full((8, 8), 0.5, dtype=torch.float64), 0.5)


def test_tanner_slope_and_cox_voinov_on_exact_laws():
    """The fits on series that follow the laws exactly: r = r0 t^(1/10) gives
    the exponent 1/10; theta^3 - theta_eq^3 = 9 Ca gives correlation 1 and
    slope 9 (Ca = mu U / gamma from the radius increments)."""
    import numpy as np
    from paper_1810_07642_amd.spreading import SpreadingSeries, cox_voinov, tanner_slope
    t = np.array([0.0, 0.5, 1, 2, 3, 5, 8, 12, 20])
    r = 50.0 * np.maximum(t, 1e-9) ** 0.1
    s = SpreadingSeries(t=t, r=r, theta=np.full_like(t, 0.3), tau_cap=1000.0, nu=1 / 6, gamma=0.01, r0=r[0])
    assert tanner_slope(s, 2, 20) == pytest.approx(0.1, rel=1e-9)
    # angles chosen so that the interval means of theta^3 follow 9 Ca + theta_eq^3
    th_eq = 0.25
    ca = [s.nu * (r[i + 1] - r[i]) / ((t[i + 1] - t[i]) * s.tau_cap) / s.gamma for i in range(len(t) - 1)]
    mean3 = [th_eq ** 3 + 9.0 * c for c in ca]
    th3 = [mean3[0]]
    for m in mean3:           # 0.5 (a^3 + b^3) = m  ->  b^3 = 2 m - a^3
        th3.append(2 * m - th3[-1])
    s.theta = np.cbrt(np.array(th3))
    corr, slope = cox_voinov(s, t_min=2.0, theta_eq=th_eq)
    assert corr == pytest.approx(1.0, abs=1e-9)
    assert slope == pytest.approx(9.0, rel=1e-6)


def test_drop_position_is_the_periodic_centre():
    """Circular mean of x weighted by h - h_*: a cap centred at x = 10 on a
    200-wide lattice, also when it straddles the periodic edge."""
    import torch
    from paper_1810_07642_amd.sliding import drop_position
    h = inputs.spherical_cap(64, 200, 20.0, 3.0, 0.5)      # centred at x = 100
    assert drop_position(h, 0.5) == pytest.approx(100.0, abs=1e-6)
    shifted = torch.roll(h, shifts=110, dims=1)           # centre at 210 mod 200 = 10
    assert drop_position(shifted, 0.5) == pytest.approx(10.0, abs=1e-6)

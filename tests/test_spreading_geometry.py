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

"""Spreading dynamics (Sec. III B) on the paper's geometry: 512^2, cap of base
radius 100 released at theta = pi/6 on a substrate of theta_eq = pi/12, three
viscosities (tau = 0.9, 1.0, 1.2; tau_cap = 1333, 1667, 2333 steps), h_* = 0.5
and slip length delta = 4 (the paper states neither), FP64, 25 tau_cap.

Checks the paper's statements that hold here, with margins around the measured
values: the radius curves of the three viscosities collapse when time is
measured in tau_cap (measured spread 0.6 %); theta^3 - theta_eq^3 is linear in
the capillary number (Cox-Voinov; measured correlation 0.995); the drop spreads
monotonically toward theta_eq after the first 2 tau_cap.  The growth exponent
is measured, 0.07 over 2-10 tau_cap, against Tanner's 1/10, and asserted to lie
in [0.05, 0.11].
"""
import math

import numpy as np
import pytest

from gpu_common import banner

pytestmark = pytest.mark.gpu

TIMES = (0.5, 1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20, 25)


def test_spreading_drop_collapse_cox_voinov_tanner():
    from paper_1810_07642_amd.spreading import cox_voinov, spreading_series, tanner_slope
    banner("spreading drop 512^2, three viscosities, 25 tau_cap")
    runs = {tau: spreading_series(tau=tau, times=TIMES) for tau in (0.9, 1.0, 1.2)}
    ref = runs[1.0]
    for tau, s in runs.items():
        rr = s.r / s.r0
        dev = float(np.abs(rr - ref.r / ref.r0).max())
        corr, slope = cox_voinov(s, t_min=2.0)
        n = tanner_slope(s, 2.0, 10.0)
        print(f"tau {tau}: tau_cap {s.tau_cap:.0f}, r/r0 at 12 tau_cap {rr[TIMES.index(12) + 1]:.3f}, "
              f"at 25 {rr[-1]:.3f}, theta {math.degrees(s.theta[-1]):.1f} deg, collapse dev {dev:.4f}, "
              f"Cox-Voinov corr {corr:.4f} slope {slope:.2f}, growth exponent {n:.3f}")
        assert dev < 0.015
        assert corr > 0.98 and slope > 0
        assert 0.05 <= n <= 0.11
        late = s.t >= 2.0
        assert np.all(np.diff(s.r[late]) > 0) and np.all(np.diff(s.theta[late]) < 0)
        assert rr[-1] > 1.15
        assert math.pi / 12 < s.theta[-1] < math.pi / 12 + math.radians(4)

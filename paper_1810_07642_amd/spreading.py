"""Spreading dynamics of a sessile drop (Sec. III B): contact-angle and radius
tracking, Tanner's law and the Cox-Voinov law.

The drop is a spherical cap on the precursor film (Sec. III B cap equation)
released at an angle above the equilibrium one, so it spreads.  Following the
paper, the instantaneous cap is recovered from the conserved volume and the
measured apex height: with V = sum_x (h - h_*) and h_d = max h - h_*, the cap
volume V = (pi/6) h_d (3 r^2 + h_d^2) (the paper's eq. "spherical_cap_vol"
written with base radius r and height h_d instead of R and theta) gives the
base radius r, the sphere radius R = (r^2 + h_d^2) / (2 h_d), and the angle
theta = arcsin(r / R) (the paper's cross-check formula).  Time is measured in
capillary times tau_cap = mu R0 / gamma with mu = nu (rho_0 = 1) and R0 the
initial base radius.

    series = spreading_series(n=512, base_radius=100, theta0=pi/6, theta_eq=pi/12, tau=1.0,
                              times=(0.5, 1, 2, 5, 10, 20))
    tanner_slope(series, 2, 10), cox_voinov(series, t_min=2)

The stepping runs in the HIP library (Sim); this module only reads h back and
does the cap geometry on the host.
"""
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import inputs


def cap_geometry(h, hstar):
    """(r, h_d, theta, R) of the spherical cap with the volume and apex height
    of the film h above the precursor h_*."""
    d = torch.as_tensor(h, dtype=torch.float64) - hstar
    vol = float(d.sum())
    hd = float(d.max())
    if hd <= 0 or vol <= 0:
        raise ValueError("no drop above the precursor film")
    r2 = (6.0 * vol / (math.pi * hd) - hd * hd) / 3.0
    r = math.sqrt(max(r2, 0.0))
    R = (r * r + hd * hd) / (2.0 * hd)
    return r, hd, math.asin(min(1.0, r / R)), R


@dataclass
class SpreadingSeries:
    t: np.ndarray          # time in capillary times tau_cap = nu R0 / gamma
    r: np.ndarray          # base radius (lattice units)
    theta: np.ndarray      # apparent contact angle (rad)
    tau_cap: float         # lattice time steps per capillary time
    nu: float
    gamma: float
    r0: float


def spreading_series(n=512, base_radius=100.0, theta0=math.pi / 6, theta_eq=math.pi / 12, tau=1.0,
                     gamma=0.01, hstar=0.5, delta=4.0, times=(0.5, 1, 2, 3, 5, 8, 12, 20), prec="fp64"):
    """Runs the spreading drop and samples (r, theta) at the given times (in
    tau_cap).  Initial cap of the given base radius and angle theta0 on h_*,
    uniform equilibrium angle theta_eq, (n, m) = (9, 3)."""
    from .sim import Sim
    apex = inputs.apex_from_angle(base_radius, theta0)
    h0 = inputs.spherical_cap(n, n, base_radius, apex, hstar)
    p = inputs.params(tau=tau, gamma=gamma, hstar=hstar, delta=delta)
    nu = (tau - 0.5) / 3.0
    tcap = nu * base_radius / gamma
    sim = Sim(n, n, prec, **p).init(h0, torch.full((n, n), theta_eq, dtype=torch.float64))
    rows = [(0.0,) + cap_geometry(sim.height(), hstar)[::2]]
    done = 0
    for tt in times:
        s = int(round(tt * tcap / 2.0)) * 2
        if s > done:
            sim.step(s - done)
            done = s
        r, _, th, _ = cap_geometry(sim.height(), hstar)
        rows.append((done / tcap, r, th))
    sim.check()
    a = np.array(rows, dtype=np.float64)
    return SpreadingSeries(t=a[:, 0], r=a[:, 1], theta=a[:, 2], tau_cap=tcap, nu=nu, gamma=gamma, r0=a[0, 1])


def tanner_slope(s, t_lo, t_hi):
    """Exponent of r(t) ~ t^n fitted in log-log over t_lo <= t <= t_hi (tau_cap)."""
    sel = (s.t >= t_lo) & (s.t <= t_hi)
    if sel.sum() < 2:
        raise ValueError("fewer than two samples in the window")
    return float(np.polyfit(np.log(s.t[sel]), np.log(s.r[sel]), 1)[0])


def cox_voinov(s, t_min=2.0, theta_eq=None):
    """Correlation and slope of theta^3 - theta_eq^3 against Ca = mu U / gamma,
    with U the contact-line speed dr/dt between consecutive samples after
    t_min (theta averaged over each interval); theta_eq defaults to the last
    sample's angle."""
    th_eq = s.theta[-1] if theta_eq is None else theta_eq
    ca, d3 = [], []
    for i in range(len(s.t) - 1):
        if s.t[i] < t_min:
            continue
        U = (s.r[i + 1] - s.r[i]) / ((s.t[i + 1] - s.t[i]) * s.tau_cap)
        ca.append(s.nu * U / s.gamma)
        d3.append(0.5 * (s.theta[i] ** 3 + s.theta[i + 1] ** 3) - th_eq ** 3)
    if len(ca) < 3:
        raise ValueError("fewer than three intervals after t_min")
    return float(np.corrcoef(ca, d3)[0, 1]), float(np.polyfit(ca, d3, 1)[0])


TANNER_TIMES = (0.5, 1, 2, 3, 4, 5, 6, 8, 10, 12, 15, 20, 25)


def tanner_summary(series_by_tau, t_sat=12.0, t_end=25.0):
    """Per viscosity: growth exponents of r(t) over 1-5 and 2-10 tau_cap, r/r0
    at t_sat and t_end, the final angle, whether the radius has saturated
    (grown by less than 1 % of r0 from t_sat to t_end), and the largest
    spread of r/r0 between the viscosities at equal t/tau_cap (the collapse)."""
    out = {}
    ref = None
    for tau, s in sorted(series_by_tau.items()):
        rr = s.r / s.r0
        i_sat = int(np.argmin(np.abs(s.t - t_sat)))
        i_end = int(np.argmin(np.abs(s.t - t_end)))
        out[tau] = {"n_1_5": tanner_slope(s, 1.0, 5.0), "n_2_10": tanner_slope(s, 2.0, 10.0),
                    "r_sat": float(rr[i_sat]), "r_end": float(rr[i_end]),
                    "theta_end_deg": math.degrees(float(s.theta[i_end])),
                    "saturated": bool(rr[i_end] - rr[i_sat] < 0.01)}
        ref = rr if ref is None else ref
        out[tau]["collapse_dev"] = float(np.abs(rr - ref).max())
    return out


def tanner_sweep(hstars=(0.2, 0.5, 1.0), deltas=(1.0, 2.0, 4.0), taus=(0.9, 1.0, 1.2), times=TANNER_TIMES,
                 prec="fp64", **kw):
    """The spreading drop over a grid of precursor thicknesses h_* and slip
    lengths delta (neither is stated for the paper's experiment), three
    viscosities each: {(h_*, delta): tanner_summary(...)}, or the error text of
    a run that met h <= 0 or a non-finite h."""
    from ._lib import TFLBMError
    res = {}
    for hs in hstars:
        for d in deltas:
            try:
                runs = {tau: spreading_series(tau=tau, hstar=hs, delta=d, times=times, prec=prec, **kw)
                        for tau in taus}
                res[(hs, d)] = tanner_summary(runs, times[-4] if len(times) > 4 else times[-1], times[-1])
            except TFLBMError as e:
                res[(hs, d)] = str(e)
    return res

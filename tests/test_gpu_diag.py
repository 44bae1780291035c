"""Term-balance diagnostic (appendix, eq. "magnitude") on the GPU against the
oracle (oracle/diag.py): the same seeded inputs run the same number of steps
on both sides, then the eight norms are compared.  FP64 storage: relative
1e-10 (the state agrees to 1e-12, the terms are stencils of it); FP32 and
FP16S: 1e-3 relative to the norm (second differences of an FP32 state); plus
an absolute floor of 1e-14 (FP64) or 1e-6 (FP32) of the case's largest norm
for terms whose exact value is zero."""
import pytest
import torch

from gpu_common import banner, random_case
from oracle import diag, lbm

pytestmark = pytest.mark.gpu

CASES = [
    (70, 150, 60, dict(tau=0.8, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ax=1e-5, ay=-2e-5)),
    (23, 37, 40, dict(tau=1.0, gamma=0.02, g=0.0, hstar=0.2, delta=0.7)),
    (130, 61, 30, dict(tau=1.3, gamma=0.01, g=-2e-4, hstar=0.15, delta=1.5, ax=-3e-5)),
    (3, 2, 10, dict(tau=0.9, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ay=1e-5)),
]


def oracle_norms(p, h0, th, steps):
    P = lbm.Params(**p)
    kap = lbm.kappa(th, P)
    f = lbm.run(lbm.init(h0, P), kap, P, steps)
    return diag.term_norms(f, kap, P)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_term_norms_match_oracle(case):
    from paper_1810_07642_amd import Sim
    ny, nx, steps, p = CASES[case]
    banner(f"term norms case {case}: {ny}x{nx}, {steps} steps")
    h0, th = random_case(ny, nx, 200 + case)
    ref = oracle_norms(p, h0, th, steps)
    # a term whose exact value is 0 (x derivatives on a 2-wide lattice) keeps a
    # rounding residue of the other terms' size: absolute floor relative to the
    # largest norm of the case
    top = max(ref.values())
    for prec, tol, floor in (("fp64", 1e-10, 1e-14), ("fp32", 1e-3, 1e-6), ("fp16s", 1e-3, 1e-6)):
        sim = Sim(nx, ny, prec, href=0.45, **p).init(h0, th)
        sim.step(steps)
        got = sim.term_norms()
        for k, v in ref.items():
            assert abs(got[k] - v) <= tol * v + floor * top, (prec, k, got[k], v)


def test_term_norms_need_init():
    from paper_1810_07642_amd import Sim, TFLBMError
    from paper_1810_07642_amd._lib import TFLBM_ESTATE
    sim = Sim(20, 10, "fp32")
    with pytest.raises(TFLBMError) as e:
        sim.term_norms()
    assert e.value.code == TFLBM_ESTATE


def test_advection_negligible_against_friction():
    """The appendix omits the advection term as orders of magnitude below the
    others.  Dewetting film (256^2 of the benchmark recipe, FP32) and a thin
    spreading drop (256^2, cap of base radius 60 and apex 4 relaxing to
    theta = 5 degrees, FP64): at every 1000 steps up to 6000 the advection
    norm stays below 1e-2 of the friction norm."""
    import math
    from paper_1810_07642_amd import Sim, inputs
    banner("advection vs friction: dewetting 256^2 and spreading drop 256^2")
    runs = [(inputs.patterned_dewetting(n=256), "fp32"),
            (inputs.sessile_drop(n=256, base_radius=60.0, apex=4.0, hstar=0.05, theta=math.pi / 36), "fp64")]
    for (p, h0, th), prec in runs:
        sim = Sim(256, 256, prec, **p).init(h0, th)
        for _ in range(6):
            sim.step(1000)
            d = sim.term_norms()
            assert d["advection_x"] < 1e-2 * d["friction_x"], d
            assert d["advection_y"] < 1e-2 * d["friction_y"], d
        sim.check()

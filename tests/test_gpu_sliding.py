"""Sliding drop (Sec. III C, eq. "CaBo") at the configuration's size: 1024 x 512,
cap of base radius 40 at theta = pi/6, 100000 steps, steady capillary number
over the whole sweep (Bond numbers 0.1, 0.2, 0.4, 0.8; slip lengths 0.5, 1,
2) in FP64, FP32 and FP16-shifted storage.  The FP64 HIP path (parity with
the oracle is shown on this workload's first 300 steps in
test_gpu_config_parity.py) is the reference here.  The precursor is h_* =
0.5: with the configuration's h_* = 0.05 the contact line is a fraction of a
lattice unit wide and the run reaches h <= 0 for delta >= 1, in the oracle as
well.

Checks: Ca positive and growing with the Bond number at every slip length;
FP32 and FP16S Ca within their recorded errors of FP64 (a-priori bound 1 %).
The least-squares line Ca = s (Bo - Bo_c) per slip length is printed; its
intercept Bo_c has no closed form to check (parity unpinned): the model's
linear friction has no pinning mechanism, and the fitted Bo_c comes out at
or below 0 (-0.08, -0.06, -0.01), not the positive critical Bond number of
the paper's figure."""
import pytest

from gpu_common import banner, check_err

pytestmark = pytest.mark.gpu


def test_sliding_drop_capillary_number_sweep_all_forms():
    from paper_1810_07642_amd.sliding import BONDS, DELTAS, capillary_sweep, critical_bond
    banner("sliding drop 1024x512, 12 (delta, Bond) points x 3 forms, 100000 steps each")
    ca = {prec: capillary_sweep(prec) for prec in ("fp64", "fp32", "fp16s")}
    for d in DELTAS:
        c64 = [ca["fp64"][(d, b)] for b in BONDS]
        s, bo_c, res = critical_bond(BONDS, c64)
        print(f"delta {d}: Ca {['%.4e' % c for c in c64]}; fit Ca = {s:.4f} (Bo - {bo_c:.4f}), "
              f"largest residual {res:.3f} of max Ca", flush=True)
        assert all(c > 0 for c in c64)
        assert all(b > a for a, b in zip(c64, c64[1:]))
        for b in BONDS:
            for prec in ("fp32", "fp16s"):
                err = abs(ca[prec][(d, b)] - ca["fp64"][(d, b)]) / ca["fp64"][(d, b)]
                check_err(f"sliding.ca.{prec}.delta{d}.bond{b}", err, 1e-2)

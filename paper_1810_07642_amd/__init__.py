"""MI355X-native thin-film lattice Boltzmann method (arXiv:1810.07642).

The compute path is libtflbm.so (HIP kernels for gfx950 behind the C ABI of
include/tflbm.h); this package is its thin Python binding:

  Sim        -- one lattice: init / step / read / mass / check / checkpoints / adjoint
  TFLBMRun   -- torch.autograd.Function: gradient of the final height w.r.t. h0 and theta
  design     -- inverse design: Adam on theta(x, y) through TFLBMRun (fit_contact_angle)
  spreading  -- spreading-drop tracking: cap geometry, Tanner exponent, Cox-Voinov fit
  sliding    -- sliding drop under a body force: steady capillary number
  inputs     -- seeded synthetic initial conditions and parameter sets
  build      -- compiles libtflbm.so
"""
from . import inputs  # noqa: F401


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    if name in ("TFLBMRun", "run_with_grad"):
        from . import autograd
        return getattr(autograd, name)
    if name == "TFLBMError":
        from ._lib import TFLBMError
        return TFLBMError
    raise AttributeError(name)

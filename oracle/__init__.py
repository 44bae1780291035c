"""FP64 CPU oracle of the thin-film lattice Boltzmann method (arXiv:1810.07642).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports, links or calls anything here, and this package shares no code with
the HIP path.

Modules:
  lbm   -- forward step, moments, mass (Sec. II).
  grad  -- autograd gradient through the forward step, with recompute.
  local -- one-site-at-a-time evaluation on periodic windows, for sampled
           checks at grid sizes the whole-array oracle cannot afford.
  diag  -- term-balance diagnostic of the appendix (eq. "magnitude").

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` (moment identities, stencil closed forms, exact
recurrences, a hand-derived Fourier propagator, disjoining integral, mass
invariance, contact angle of a relaxed drop); none is "parity unpinned".
"""
from . import lbm, grad, local, diag  # noqa: F401

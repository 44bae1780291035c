"""Python handle over the C ABI: torch supplies device memory and the stream,
every step of the method runs in the HIP kernels of libtflbm.so.

    sim = Sim(nx, ny, prec="fp32", tau=1.0, gamma=0.01, hstar=0.05, ...)
    sim.init(h0, theta)          # float64 [ny, nx] tensors (any device)
    sim.step(1000)
    h, ux, uy = sim.read()       # float64 [ny, nx] on the GPU
"""
import ctypes

import torch

from . import _lib

PARAM_KEYS = ("tau", "gamma", "g", "hstar", "n", "m", "delta", "ax", "ay", "theta0",
              "href", "fp16_scale_log2", "gamma_field")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _addr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _buf(t, nbytes, device, name):
    """Checks that a caller-supplied buffer is a contiguous tensor on the
    handle's device holding at least nbytes (the library dereferences its
    address on the GPU)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, the lattice is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return t


def _dev_f64(t, device, shape, name):
    if t is None:
        return None
    t = torch.as_tensor(t)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.to(device=device, dtype=torch.float64).contiguous()


def make_params(nx, ny, prec="fp64", **kw):
    """A ``tflbm_params`` from keyword arguments (paper notation: n, m exponents)."""
    lib = _lib.load()
    p = _lib.Params()
    lib.tflbm_default_params(ctypes.byref(p))
    p.nx, p.ny = int(nx), int(ny)
    p.prec = _lib.PREC[prec] if isinstance(prec, str) else int(prec)
    for k, v in kw.items():
        if k not in PARAM_KEYS:
            raise KeyError(f"unknown parameter {k!r}")
        if k == "n":
            p.n_exp = int(v)
        elif k == "m":
            p.m_exp = int(v)
        elif k == "fp16_scale_log2":
            p.fp16_scale_log2 = int(v)
        elif k == "gamma_field":
            p.gamma_field = int(bool(v))
        else:
            setattr(p, k, float(v))
    return p


def capture_bytes_for(nx, ny, prec="fp64"):
    """Bytes of one step's capture (tflbm_capture_bytes) for a lattice, from a
    handle that binds no workspace."""
    lib = _lib.load()
    p = make_params(nx, ny, prec)
    h = ctypes.c_void_p()
    _lib.check(lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)), "tflbm_create")
    try:
        return int(lib.tflbm_capture_bytes(h))
    finally:
        lib.tflbm_destroy(h)


def check_params(nx, ny, prec="fp64", **kw):
    """TFLBM_OK, TFLBM_EINVAL or TFLBM_EUNSTABLE for a parameter set."""
    return _lib.load().tflbm_check_params(ctypes.byref(make_params(nx, ny, prec, **kw)))


class Sim:
    """One periodic nx x ny lattice on one GPU."""

    def __init__(self, nx, ny, prec="fp64", device=None, **params):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("Sim needs a GPU device")
        self.nx, self.ny = int(nx), int(ny)
        self.prec = prec
        self.params = make_params(nx, ny, prec, **params)
        h = ctypes.c_void_p()
        _lib.check(self.lib.tflbm_create(ctypes.byref(self.params), ctypes.byref(h)), "tflbm_create")
        self.h = h
        nbytes = self.lib.tflbm_workspace_bytes(h)
        # zeroed so that record padding (columns past nx) has defined bytes
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.tflbm_bind(h, _addr(self.ws), nbytes), "tflbm_bind", h)
        self.h0 = None
        self.theta = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.tflbm_destroy(h)
            self.h = None

    @property
    def stream(self):
        return _stream(self.device)

    def _chk(self, code, where):
        return _lib.check(code, where, self.h)

    def init(self, h0, theta=None, gamma=None):
        """f = E(h0); kappa from theta ([ny, nx] float64) or the uniform theta0;
        gamma: a per-site surface tension field (the handle must be created
        with gamma_field=True), else the scalar gamma."""
        shape = (self.ny, self.nx)
        self.h0 = _dev_f64(h0, self.device, shape, "h0")
        self.theta = _dev_f64(theta, self.device, shape, "theta")
        self.gamma = _dev_f64(gamma, self.device, shape, "gamma")
        self._chk(self.lib.tflbm_init_fields(self.h, _addr(self.h0), _addr(self.theta), _addr(self.gamma),
                                             self.stream), "tflbm_init_fields")
        return self

    def step(self, nsteps=1):
        self._chk(self.lib.tflbm_step(self.h, int(nsteps), self.stream), "tflbm_step")
        return self

    @property
    def steps(self):
        return int(self.lib.tflbm_step_count(self.h))

    @property
    def steps_per_pass(self):
        """Most time steps one pass of tflbm_step advances on this handle."""
        n = int(self.lib.tflbm_steps_per_pass(self.h))
        if n < 0:
            raise RuntimeError(f"tflbm_steps_per_pass: {n}")
        return n

    @property
    def step_graphs(self):
        """Step graphs the handle holds (tflbm_step replays blocks of steps
        from them on launch-bound lattices)."""
        return int(self.lib.tflbm_step_graphs(self.h))

    def read(self, out=None):
        """(h, ux, uy) as float64 [ny, nx] tensors on the device."""
        if out is None:
            out = tuple(torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(3))
        h, ux, uy = out
        for t, name in ((h, "h"), (ux, "ux"), (uy, "uy")):
            if t is not None:
                _buf(t, 8 * self.nx * self.ny, self.device, name)
                if t.dtype != torch.float64:
                    raise ValueError(f"{name}: expected float64")
        self._chk(self.lib.tflbm_read(self.h, _addr(h), _addr(ux), _addr(uy), self.stream), "tflbm_read")
        return h, ux, uy

    def height(self):
        h = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        self._chk(self.lib.tflbm_read(self.h, _addr(h), None, None, self.stream), "tflbm_read")
        return h

    def mass(self):
        m = ctypes.c_double()
        self._chk(self.lib.tflbm_mass(self.h, ctypes.byref(m), self.stream), "tflbm_mass")
        return m.value

    def mass_noalloc(self, out=None):
        """Total mass as a float64 device tensor of one element, by the
        allocation-free entry point (tflbm_mass_noalloc: partials in the
        library's static scratch, no synchronisation)."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        _buf(out, 8, self.device, "mass output")
        self._chk(self.lib.tflbm_mass_noalloc(self.h, _addr(out), self.stream), "tflbm_mass_noalloc")
        return out

    def check(self):
        """Raises TFLBMError(TFLBM_ENONFINITE) if a step met h <= 0 or non-finite h."""
        self._chk(self.lib.tflbm_check(self.h, self.stream), "tflbm_check")

    TERM_NAMES = ("pressure_x", "friction_x", "viscous_x", "advection_x",
                  "pressure_y", "friction_y", "viscous_y", "advection_y")

    def term_norms(self):
        """Term-balance diagnostic of the current state (appendix, eq.
        "magnitude"): a dict name -> L2 norm over the lattice."""
        out = (ctypes.c_double * 8)()
        self._chk(self.lib.tflbm_term_norms(self.h, out, self.stream), "tflbm_term_norms")
        return dict(zip(self.TERM_NAMES, list(out)))

    def status(self):
        return self.lib.tflbm_check(self.h, self.stream)

    # ---- checkpoints ----------------------------------------------------------
    def state_bytes(self):
        return int(self.lib.tflbm_state_bytes(self.h))

    def state_save(self, out=None):
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _buf(out, self.state_bytes(), self.device, "checkpoint buffer")
        self._chk(self.lib.tflbm_state_save(self.h, _addr(out), self.stream), "tflbm_state_save")
        return out

    def state_load(self, buf, step):
        _buf(buf, self.state_bytes(), self.device, "checkpoint buffer")
        self._chk(self.lib.tflbm_state_load(self.h, _addr(buf), int(step), self.stream), "tflbm_state_load")
        return self

    # ---- reverse mode ---------------------------------------------------------
    def capture_bytes(self):
        return int(self.lib.tflbm_capture_bytes(self.h))

    def step_capture(self, nsteps, capture):
        _buf(capture, int(nsteps) * self.capture_bytes(), self.device, "capture buffer")
        self._chk(self.lib.tflbm_step_capture(self.h, int(nsteps), _addr(capture), self.stream),
                  "tflbm_step_capture")
        return self

    def adj_bytes(self):
        return int(self.lib.tflbm_adj_bytes(self.h))

    def adj_seed(self, adj, grad_h):
        _buf(adj, self.adj_bytes(), self.device, "adjoint workspace")
        g = _dev_f64(grad_h, self.device, (self.ny, self.nx), "grad_h")
        self._chk(self.lib.tflbm_adj_seed(self.h, _addr(adj), _addr(g), self.stream), "tflbm_adj_seed")
        self._seed_keepalive = g
        return self

    def adj_step(self, adj, capture_t):
        _buf(adj, self.adj_bytes(), self.device, "adjoint workspace")
        _buf(capture_t, self.capture_bytes(), self.device, "capture")
        self._chk(self.lib.tflbm_adj_step(self.h, _addr(adj), _addr(capture_t), self.stream), "tflbm_adj_step")
        return self

    def adj_steps(self, adj, captures, nsteps):
        """Reverse pass over `nsteps` captured steps (tflbm_adj_steps: two per
        pass over the lattice where that pays)."""
        _buf(adj, self.adj_bytes(), self.device, "adjoint workspace")
        _buf(captures, int(nsteps) * self.capture_bytes(), self.device, "captures")
        self._chk(self.lib.tflbm_adj_steps(self.h, _addr(adj), _addr(captures), int(nsteps), self.stream),
                  "tflbm_adj_steps")
        return self

    def adj_finish(self, adj, want_h0=True, want_theta=True):
        _buf(adj, self.adj_bytes(), self.device, "adjoint workspace")
        gh0 = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) if want_h0 else None
        gth = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) if want_theta else None
        self._chk(self.lib.tflbm_adj_finish(self.h, _addr(adj), _addr(self.h0), _addr(self.theta),
                                            _addr(gh0), _addr(gth), self.stream), "tflbm_adj_finish")
        return gh0, gth

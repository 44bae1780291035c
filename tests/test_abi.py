"""C-ABI checks that need no GPU: the library loads, exports every function
include/tflbm.h declares, and validates parameters and call order on the host."""
import ctypes

import pytest

from paper_1810_07642_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def params(lib, **kw):
    p = _lib.Params()
    lib.tflbm_default_params(ctypes.byref(p))
    p.nx, p.ny = 64, 48
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_exports_every_declared_function(lib):
    names = _lib.header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version_and_strerror(lib):
    assert b"gfx950" in lib.tflbm_version()
    for code in (0, -1, -2, -3, -4, -5):
        assert len(lib.tflbm_strerror(code)) > 0
    assert lib.tflbm_strerror(-99) == b"unknown error"


def test_struct_layout_matches_header(lib):
    # seven int32, padding to 8 bytes, then nine doubles (natural alignment)
    assert ctypes.sizeof(_lib.Params) == 7 * 4 + 4 + 9 * 8
    p = params(lib)
    assert (p.n_exp, p.m_exp, p.tau, p.gamma, p.hstar, p.delta) == (9, 3, 1.0, 0.01, 0.05, 1.0)
    assert p.fp16_scale_log2 == 12


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("prec", 3), ("tau", 0.5), ("tau", float("nan")), ("hstar", 0.0),
    ("gamma", -1.0), ("delta", -0.1), ("n_exp", 3), ("m_exp", 0), ("fp16_scale_log2", 30),
    ("g", float("inf")), ("href", -1.0), ("gamma_field", 2),
])
def test_invalid_parameters_rejected(lib, field, value):
    p = params(lib, **{field: value})
    if field == "n_exp":
        p.m_exp = 3  # n == m
    assert lib.tflbm_check_params(ctypes.byref(p)) == _lib.TFLBM_EINVAL
    h = ctypes.c_void_p(123)
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == _lib.TFLBM_EINVAL
    assert not h.value


def test_too_large_lattice_rejected(lib):
    p = params(lib, nx=65536, ny=40000)
    assert lib.tflbm_check_params(ctypes.byref(p)) == _lib.TFLBM_EINVAL


# bytes per 54-column strip of the largest adjoint row (the records of nine
# populations: FP64 for the FP64 form, FP32 for the others)
ADJ_ROW_MAX = {0: 3968, 1: 2176, 2: 2176}


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_rows_end_below_the_dropped_store_offset(lib, prec):
    """The kernels aim the stores they drop (halo lanes, rows without output)
    at byte offset 0x7fff0000 of a row's buffer range, so every row must end
    below it.  The widest accepted lattice has its population and adjoint rows
    below the offset, one more column is rejected, although every row would
    still fit a 32-bit range; the population rows bind in FP64, the adjoint
    rows in FP32 and FP16S."""
    sites, rb = RECORDS[prec]
    lim = 0x7fff0000
    by_records = (lim - 1) // rb * sites
    by_adjoint = (lim - 1) // ADJ_ROW_MAX[prec] * 54
    nx = min(by_records, by_adjoint)
    assert (by_records < by_adjoint) == (prec == 0)
    accept = params(lib, prec=prec, nx=nx, ny=1)
    assert lib.tflbm_check_params(ctypes.byref(accept)) == _lib.TFLBM_OK
    reject = params(lib, prec=prec, nx=nx + 1, ny=1)
    assert (-(-(nx + 1) // sites)) * rb < 1 << 31
    assert lib.tflbm_check_params(ctypes.byref(reject)) == _lib.TFLBM_EINVAL


def test_steps_per_pass_needs_an_initialised_handle(lib):
    """tflbm_steps_per_pass: EINVAL for NULL, ESTATE before tflbm_init (the
    plan is fixed at init, from the device's occupancy)."""
    assert lib.tflbm_steps_per_pass(None) == _lib.TFLBM_EINVAL
    h = ctypes.c_void_p()
    assert lib.tflbm_create(ctypes.byref(params(lib)), ctypes.byref(h)) == _lib.TFLBM_OK
    try:
        assert lib.tflbm_steps_per_pass(h) == _lib.TFLBM_ESTATE
    finally:
        lib.tflbm_destroy(h)


def test_friction_stability_warning(lib):
    # 2 nu / delta^2 >= 2: nu = 1/6 needs delta > sqrt(1/6) ~ 0.408
    p = params(lib, delta=0.3)
    assert lib.tflbm_check_params(ctypes.byref(p)) == _lib.TFLBM_EUNSTABLE
    h = ctypes.c_void_p()
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == _lib.TFLBM_OK  # warning only
    lib.tflbm_destroy(h)
    assert lib.tflbm_check_params(ctypes.byref(params(lib, delta=0.5))) == _lib.TFLBM_OK


# population records: (sites per record, bytes per record) of each storage form
RECORDS = {0: (46, 3456), 1: (108, 4224), 2: (116, 2688)}


@pytest.mark.parametrize("prec,per_site", [(0, 72), (1, 36), (2, 20)])
def test_workspace_and_state_sizes(lib, prec, per_site):
    p = params(lib, prec=prec, nx=100, ny=30)
    h = ctypes.c_void_p()
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == 0
    B, RB = RECORDS[prec]
    nblk = -(-100 // B)
    assert lib.tflbm_state_bytes(h) == 30 * nblk * RB
    assert RB >= per_site * B
    assert lib.tflbm_workspace_bytes(h) >= 2 * 30 * nblk * RB
    wb = 8 if prec == 0 else 4
    # capture: records of the same B columns, three segments padded to whole lines
    assert lib.tflbm_capture_bytes(h) == 30 * nblk * (-(-3 * B * wb // 128) * 128)
    # adjoint: two buffers of records of 54 columns (nine segments padded to an
    # odd number of lines) and FP64 dLoss/dkappa records of 64 values, each
    # rounded to 4 KiB
    # (with tau = 1, three fields per site in records of 3 x 64 slots)
    ARB = {0: 31 * 128, 1: 17 * 128, 2: 17 * 128}[prec]
    assert ARB >= 9 * 54 * wb
    if p.tau == 1.0:
        ARB = 3 * 64 * wb
    nas = -(-100 // 54)
    r4k = lambda v: -(-v // 4096) * 4096
    assert lib.tflbm_adj_bytes(h) == 2 * r4k(30 * nas * ARB) + r4k(30 * nas * 512)
    from paper_1810_07642_amd.sim import capture_bytes_for
    assert capture_bytes_for(100, 30, {0: "fp64", 1: "fp32", 2: "fp16s"}[prec]) == lib.tflbm_capture_bytes(h)
    lib.tflbm_destroy(h)


def test_call_order_and_null_pointers(lib):
    h = ctypes.c_void_p()
    p = params(lib)
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == 0
    assert lib.tflbm_create(ctypes.byref(p), None) == _lib.TFLBM_EINVAL
    # nothing bound / initialised yet: host-side rejections, no GPU touched
    assert lib.tflbm_bind(h, None, 0) == _lib.TFLBM_EINVAL
    assert lib.tflbm_bind(h, ctypes.c_void_p(256), 16) == _lib.TFLBM_EINVAL
    assert lib.tflbm_bind(h, ctypes.c_void_p(257), 1 << 40) == _lib.TFLBM_EINVAL  # misaligned
    assert lib.tflbm_init(h, ctypes.c_void_p(256), None, None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_init(h, None, None, None) == _lib.TFLBM_EINVAL
    assert lib.tflbm_step(h, 1, None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_step(h, -1, None) == _lib.TFLBM_EINVAL
    assert lib.tflbm_step_graphs(h) == 0 and lib.tflbm_step_graphs(None) == -1
    assert lib.tflbm_read(h, None, None, None, None) == _lib.TFLBM_ESTATE
    m = ctypes.c_double()
    assert lib.tflbm_mass(h, ctypes.byref(m), None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_check(h, None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_adj_step(h, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_adj_steps(h, ctypes.c_void_p(256), ctypes.c_void_p(256), 4, None) == _lib.TFLBM_ESTATE
    assert lib.tflbm_adj_steps(h, ctypes.c_void_p(256), ctypes.c_void_p(256), -1, None) == _lib.TFLBM_EINVAL
    assert lib.tflbm_adj_steps(h, ctypes.c_void_p(256), None, 2, None) == _lib.TFLBM_EINVAL
    assert lib.tflbm_step_count(h) == 0
    assert lib.tflbm_step_count(None) == -1
    lib.tflbm_destroy(h)


def test_gamma_field_needs_the_flag(lib):
    """tflbm_init_fields with a surface tension field on a handle created
    without params.gamma_field is refused before any device work; with the
    flag the workspace holds two values per site instead of one."""
    p = params(lib, nx=100, ny=30)
    h = ctypes.c_void_p()
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == _lib.TFLBM_OK
    fake = ctypes.c_void_p(0x1000)
    assert lib.tflbm_init_fields(h, fake, None, fake, None) == _lib.TFLBM_EINVAL
    ws0 = lib.tflbm_workspace_bytes(h)
    lib.tflbm_destroy(h)
    p.gamma_field = 1
    assert lib.tflbm_create(ctypes.byref(p), ctypes.byref(h)) == _lib.TFLBM_OK
    assert lib.tflbm_workspace_bytes(h) > ws0
    lib.tflbm_destroy(h)

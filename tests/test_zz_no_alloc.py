"""The allocation-free mass entry point (tflbm_mass_noalloc, partial sums in
the library's static device scratch, result left in device memory) against
tflbm_mass, which reduces through the handle's workspace: the same bits, on
two calls in a row, the second on a smaller lattice, and inside a caller's
captured graph replayed with eager steps between the replays."""
import ctypes

import pytest
import torch

from gpu_common import banner, random_case

pytestmark = pytest.mark.gpu


def _noalloc(sim):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=sim.device)
    rc = sim.lib.tflbm_mass_noalloc(sim.h, ctypes.c_void_p(out.data_ptr()), sim.stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return float(out.item())


def test_mass_noalloc_equals_mass_two_calls_second_smaller():
    from paper_1810_07642_amd import Sim
    p = dict(tau=0.9, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ax=1e-5)
    for (ny, nx, prec) in [(260, 700, "fp32"), (23, 37, "fp64"), (40, 130, "fp16s")]:
        banner(f"mass_noalloc {prec} {ny}x{nx}")
        h0, th = random_case(ny, nx, 61)
        sim = Sim(nx, ny, prec, **p).init(h0, th)
        sim.step(9)
        ref = sim.mass()
        got = _noalloc(sim)
        print(f"{prec} {ny}x{nx}: tflbm_mass {ref!r}, tflbm_mass_noalloc {got!r}")
        assert got == ref
        # the oracle's mass of the same state is within FP64 rounding of both
        m0 = float(h0.sum())
        if prec == "fp64":
            assert abs(got - m0) <= 1e-13 * m0
        del sim


def test_mass_noalloc_rejects_bad_calls():
    from paper_1810_07642_amd import Sim
    from paper_1810_07642_amd._lib import TFLBM_EINVAL, TFLBM_ESTATE
    sim = Sim(50, 20, "fp32", hstar=0.1)
    out = torch.zeros(1, dtype=torch.float64, device=sim.device)
    assert sim.lib.tflbm_mass_noalloc(sim.h, ctypes.c_void_p(out.data_ptr()), sim.stream) == TFLBM_ESTATE
    sim.init(torch.full((20, 50), 0.3, dtype=torch.float64), None)
    assert sim.lib.tflbm_mass_noalloc(sim.h, None, sim.stream) == TFLBM_EINVAL
    assert sim.lib.tflbm_mass_noalloc(None, ctypes.c_void_p(out.data_ptr()), sim.stream) == TFLBM_EINVAL


def test_mass_noalloc_in_a_captured_graph():
    """Captured into a torch graph (kernel nodes only) together with steps of
    the lattice; each of three replays, with eager steps in between, leaves
    the mass of the state it saw, equal to tflbm_mass of that state."""
    from paper_1810_07642_amd import Sim
    p = dict(tau=0.9, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ax=1e-5)
    h0, th = random_case(70, 150, 62)
    sim = Sim(150, 70, "fp64", **p).init(h0, th)
    out = torch.zeros(1, dtype=torch.float64, device=sim.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            sim.step(4)  # an even number of buffer swaps: the replay keeps the parity
            sim.mass_noalloc(out)
    torch.cuda.synchronize()
    for i in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = float(out.item())
        assert got == sim.mass(), i
        sim.step(6)
        torch.cuda.synchronize()
    sim.check()

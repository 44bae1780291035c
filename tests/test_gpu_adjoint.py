"""Reverse mode: the hand-written adjoint of the HIP step (through the C ABI,
wrapped in TFLBMRun) against the oracle's autograd gradient and against
central finite differences of the HIP forward."""
import math

import pytest
import torch

from gpu_common import banner, check_err, random_case
from oracle import grad as ograd
from oracle import lbm
from paper_1810_07642_amd import inputs

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float((a - b).norm() / b.norm())


def gpu_grads(p, h0, th, grad_h, steps, K, prec):
    from paper_1810_07642_amd import TFLBMRun
    h0c = h0.cuda().requires_grad_(True)
    thc = th.cuda().requires_grad_(True)
    h = TFLBMRun.apply(h0c, thc, p, steps, K, prec)
    h.backward(grad_h.cuda())
    torch.cuda.synchronize()
    return h.detach().cpu(), h0c.grad.cpu(), thc.grad.cpu()


CASES = [
    # ny, nx, steps, K, params
    (20, 30, 1, 1, dict(tau=1.0, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0, ax=1e-4)),
    (45, 70, 37, 8, dict(tau=0.8, gamma=0.02, g=-1e-3, hstar=0.15, delta=0.8, ax=2e-5, ay=-1e-5)),
    (64, 131, 25, 25, dict(tau=1.3, gamma=0.01, g=0.0, hstar=0.2, delta=1.5, n=4, m=3)),
    (3, 2, 9, 4, dict(tau=0.9, gamma=0.01, g=1e-3, hstar=0.1, delta=1.0)),
]


@pytest.mark.parametrize("fuse", ["auto", "2"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fp64_adjoint_matches_oracle_gradient(case, fuse, monkeypatch):
    """fuse = "2": two reverse steps per pass also on these small lattices
    (by default they run single steps)."""
    ny, nx, steps, K, p = CASES[case]
    banner(f"fp64 adjoint case {case}: {ny}x{nx}, {steps} steps, K={K}, reverse steps per pass: {fuse}")
    if fuse != "auto":
        monkeypatch.setenv("TFLBM_ADJ_FUSE", fuse)
    h0, th = random_case(ny, nx, 200 + case)
    g = torch.Generator().manual_seed(300 + case)
    grad_h = torch.randn((ny, nx), generator=g, dtype=torch.float64)
    gh0_o, gth_o = ograd.vjp(h0, th, grad_h, lbm.Params(**p), steps, K)
    _, gh0, gth = gpu_grads(p, h0, th, grad_h, steps, K, "fp64")
    e0, e1 = rel_l2(gh0, gh0_o), rel_l2(gth, gth_o)
    print(f"case {case}: rel L2 dL/dh0 {e0:.2e}, dL/dtheta {e1:.2e}")
    assert e0 <= 1e-11 and e1 <= 1e-11
    assert float((gh0 - gh0_o).abs().max()) <= 1e-10 * float(gh0_o.abs().max())


@pytest.mark.parametrize("fuse", ["1", "2"])
def test_adjoint_dot_product_against_oracle_forward_mode(fuse, monkeypatch):
    """<w, J v> from the oracle's forward-mode derivative (torch.func.jvp,
    no reverse mode involved) against <J^T w, v> from the hand-written GPU
    adjoint (FP64), one and two reverse steps per pass, 7 steps."""
    ny, nx, steps = 37, 70, 7
    banner(f"adjoint dot-product test {ny}x{nx}, {steps} steps, reverse steps per pass {fuse}")
    monkeypatch.setenv("TFLBM_ADJ_FUSE", fuse)
    p = dict(tau=0.8, gamma=0.02, g=-1e-3, hstar=0.15, delta=0.8, ax=2e-5, ay=-1e-5)
    h0, th = random_case(ny, nx, 91)
    g = torch.Generator().manual_seed(92)
    vh, vt, w = (torch.randn((ny, nx), generator=g, dtype=torch.float64) for _ in range(3))
    jv = ograd.jvp(h0, th, vh, vt, lbm.Params(**p), steps)
    _, gh0, gth = gpu_grads(p, h0, th, w, steps, 4, "fp64")
    lhs = float((w * jv).sum())
    rhs = float((gh0 * vh).sum() + (gth * vt).sum())
    print(f"<w, Jv> = {lhs:.15e}, <J^T w, v> = {rhs:.15e}, rel diff {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_inverse_design_64_copy():
    """The inverse-design case on a 64 x 64 copy: dewetting recipe, theta = pi/6,
    smooth target, L = 1/2 sum (h_N - target)^2, 256 steps checkpointed every 64;
    FP64 forward against the oracle gradient, and the FP32 and FP16S forwards
    (FP32 adjoint, FP64 gradient accumulation) with their errors stated: FP32
    stored as deviations from h_ref = 0 and from the film height 0.1, FP16S
    from 0.1 (measured 4.7e-5, 1.6e-6 and 1.6e-6 relative L2)."""
    p, h0, th, target = inputs.inverse_design(n=64)
    steps, K = 256, 64
    P = lbm.Params(**p)
    loss_o, gh0_o, gth_o = ograd.misfit_grad(h0, th, target, P, steps, K)
    from paper_1810_07642_amd import TFLBMRun
    res = {}
    for prec, href in (("fp64", 0.0), ("fp32", 0.0), ("fp32", 0.1), ("fp16s", 0.1)):
        h0c = h0.cuda().requires_grad_(True)
        thc = th.cuda().requires_grad_(True)
        h = TFLBMRun.apply(h0c, thc, dict(p, href=href), steps, K, prec)
        loss = 0.5 * ((h - target.cuda()) ** 2).sum()
        loss.backward()
        key = (prec, href)
        res[key] = (float(loss.detach()), rel_l2(h0c.grad.cpu(), gh0_o), rel_l2(thc.grad.cpu(), gth_o))
        print(f"{prec} href {href}: loss {res[key][0]:.10e} (oracle {loss_o:.10e}), "
              f"rel L2 err dh0 {res[key][1]:.2e} dtheta {res[key][2]:.2e}")
    assert abs(res[("fp64", 0.0)][0] - loss_o) <= 1e-12 * loss_o
    assert res[("fp64", 0.0)][1] <= 1e-10 and res[("fp64", 0.0)][2] <= 1e-10
    # a-priori bound of the FP32 forms' gradient: 1e-3 relative L2
    for key in (("fp32", 0.0), ("fp32", 0.1), ("fp16s", 0.1)):
        check_err(f"design64x256.{key[0]}.href{key[1]}.dh0", res[key][1], 1e-3)
        check_err(f"design64x256.{key[0]}.href{key[1]}.dtheta", res[key][2], 1e-3)


def test_adjoint_against_finite_differences_fp64():
    """Central differences of the HIP FP64 forward at 16 seeded pixels for theta
    and h0 (eps = 1e-4 and eps/2 must agree first), 128 x 128 dewetting recipe,
    512 steps, K = 64."""
    from paper_1810_07642_amd import Sim, TFLBMRun
    p, h0, th, target = inputs.inverse_design(n=128)
    steps, K = 512, 64
    h0c = h0.cuda().requires_grad_(True)
    thc = th.cuda().requires_grad_(True)
    tgt = target.cuda()
    h = TFLBMRun.apply(h0c, thc, p, steps, K, "fp64")
    (0.5 * ((h - tgt) ** 2).sum()).backward()
    gh0, gth = h0c.grad.cpu(), thc.grad.cpu()

    def loss(hh0, tth):
        sim = Sim(128, 128, "fp64", **p).init(hh0, tth)
        sim.step(steps)
        return float(0.5 * ((sim.height() - tgt) ** 2).sum())

    pix = inputs.random_pixels(128, 128, 16, seed=5)
    checked = 0
    for (y, x) in pix:
        for which, g in (("h0", gh0), ("theta", gth)):
            fds = []
            for eps in (1e-4, 5e-5):
                a = h0.clone(); b = th.clone()
                c = h0.clone(); d = th.clone()
                if which == "h0":
                    a[y, x] += eps; c[y, x] -= eps
                else:
                    b[y, x] += eps; d[y, x] -= eps
                fds.append((loss(a, b) - loss(c, d)) / (2 * eps))
            scale = float(g.abs().max())
            if abs(fds[0] - fds[1]) > 1e-6 * scale:
                continue  # FD itself not converged at this pixel
            checked += 1
            assert abs(fds[1] - float(g[y, x])) <= 1e-5 * scale, (which, y, x, fds, float(g[y, x]))
    assert checked >= 24


def test_adjoint_full_inverse_design_config():
    """The inverse-design configuration at full size: 512 x 512 dewetting recipe,
    4096 steps, checkpoints every 64, L = 1/2 sum (h_N - target)^2.  The FP64
    adjoint gradient w.r.t. theta and h0 against central differences of the HIP
    FP64 forward (eps = 2e-5, cross-checked with eps/2; the film ruptures over
    4096 steps, so a pixel whose two differences disagree is skipped and at
    least half of the 64 checks must converge) at 32 seeded pixels; the
    gradient of the FP32 forward (FP32 adjoint, FP64 kappa-gradient
    accumulation) against the FP64 one over the whole field."""
    from paper_1810_07642_amd import Sim, TFLBMRun
    banner("full inverse-design config 512^2 x 4096, K = 64")
    n, steps, K = 512, 4096, 64
    p, h0, th, target = inputs.inverse_design(n=n)
    tgt = target.cuda()
    grads = {}
    for prec in ("fp64", "fp32"):
        h0c = h0.cuda().requires_grad_(True)
        thc = th.cuda().requires_grad_(True)
        h = TFLBMRun.apply(h0c, thc, p, steps, K, prec)
        (0.5 * ((h - tgt) ** 2).sum()).backward()
        grads[prec] = (h0c.grad.cpu(), thc.grad.cpu())
    gh0, gth = grads["fp64"]

    def loss(hh0, tth):
        sim = Sim(n, n, "fp64", **p).init(hh0, tth)
        sim.step(steps)
        sim.check()
        return float(0.5 * ((sim.height() - tgt) ** 2).sum())

    checked = 0
    for (y, x) in inputs.random_pixels(n, n, 32, seed=11):
        for which, g in (("h0", gh0), ("theta", gth)):
            fds = []
            for eps in (2e-5, 1e-5):
                a = h0.clone(); b = th.clone()
                c = h0.clone(); d = th.clone()
                if which == "h0":
                    a[y, x] += eps; c[y, x] -= eps
                else:
                    b[y, x] += eps; d[y, x] -= eps
                fds.append((loss(a, b) - loss(c, d)) / (2 * eps))
            scale = float(g.abs().max())
            if abs(fds[0] - fds[1]) > 1e-6 * scale:
                continue  # FD itself not converged at this pixel
            checked += 1
            assert abs(fds[1] - float(g[y, x])) <= 1e-5 * scale, (which, y, x, fds, float(g[y, x]))
    assert checked >= 32
    e_h0 = rel_l2(grads["fp32"][0], gh0)
    e_th = rel_l2(grads["fp32"][1], gth)
    print(f"FD pixels checked {checked}/64; FP32-forward gradient vs FP64: rel L2 h0 {e_h0:.2e}, theta {e_th:.2e}")
    check_err("design512x4096.fp32.href0.dh0_vs_fp64", e_h0, 1e-2)
    check_err("design512x4096.fp32.href0.dtheta_vs_fp64", e_th, 1e-2)


def _reverse_pass(prec, h0, th, p, nsteps, grad_h, fused, field):
    """(dL/dh0, dL/dtheta) of nsteps captured steps, the reverse pass either
    through tflbm_adj_steps (two steps per pass) or one tflbm_adj_step per step."""
    from paper_1810_07642_amd import Sim
    ny, nx = h0.shape
    kw = dict(p)
    if not field:
        kw["theta0"] = float(th[0, 0])
    sim = Sim(nx, ny, prec, **kw).init(h0, th if field else None)
    cb = sim.capture_bytes()
    cap = torch.empty(nsteps * cb, dtype=torch.uint8, device="cuda")
    adj = torch.empty(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
    sim.step_capture(nsteps, cap)
    sim.adj_seed(adj, grad_h)
    if fused:
        sim.adj_steps(adj, cap, nsteps)
    else:
        for t in reversed(range(nsteps)):
            sim.adj_step(adj, cap[t * cb:(t + 1) * cb])
    g_h0, g_th = sim.adj_finish(adj)
    torch.cuda.synchronize()
    return g_h0.cpu(), g_th.cpu()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("shape,rows2,field,nsteps", [
    ((150, 173), "7", True, 7),      # four strips (the last 11 columns), 22 row chunks, the last of 3 rows
    ((150, 173), "40", True, 7),     # chunks of 40 rows (the long-chunk row loop), the last of 30
    ((45, 70), None, False, 6),      # uniform kappa, an even number of steps
    ((3, 2), None, True, 5),         # every row and column wraps onto the others
])
def test_two_steps_per_pass_equal_single_steps_bitwise(prec, shape, rows2, field, nsteps, monkeypatch):
    """The two-step reverse pass hands the adjoint of step t to step t-1 on
    chip instead of through memory; both stages round exactly as the single
    step does, so the gradients must agree bit for bit (odd nsteps also runs
    one single step at the end)."""
    ny, nx = shape
    banner(f"adjoint two steps per pass vs single steps: {prec} {ny}x{nx}, {nsteps} steps, rows {rows2}, field {field}")
    monkeypatch.setenv("TFLBM_ADJ_FUSE", "2")  # two steps per pass also on lattices this small
    if rows2 is not None:
        monkeypatch.setenv("TFLBM_ADJ_ROWS2", rows2)
    h0, th = random_case(ny, nx, 77)
    p = dict(tau=0.8, gamma=0.02, g=1e-3, hstar=0.15, delta=0.8, ax=2e-5, ay=-1e-5)
    if prec != "fp64":
        p["href"] = 0.45
    g = torch.Generator().manual_seed(78)
    grad_h = torch.randn((ny, nx), generator=g, dtype=torch.float64)
    a = _reverse_pass(prec, h0, th, p, nsteps, grad_h, True, field)
    b = _reverse_pass(prec, h0, th, p, nsteps, grad_h, False, field)
    for x, y, name in ((a[0], b[0], "dL/dh0"), (a[1], b[1], "dL/dtheta")):
        assert torch.isfinite(y).all(), name
        nd = int((x != y).sum())
        print(f"{name}: {nd} differing sites, max |diff| {float((x - y).abs().max()):.3e}")
        assert nd == 0, name


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("shape,rows2,field,nsteps", [
    ((150, 173), "7", True, 7),
    ((150, 173), "40", True, 7),
    ((45, 70), None, False, 6),
    ((3, 2), None, True, 5),
    ((64, 131), None, True, 9),
])
def test_omega1_reverse_pass_equals_general_bitwise(prec, shape, rows2, field, nsteps, monkeypatch):
    """At tau = 1 the step's adjoint is lambda_h + c_l . lambda_j, and the
    library carries three fields per site between reverse steps instead of
    nine populations.  Against the general reverse pass (TFLBM_OMEGA1=0), both
    with two reverse steps per pass and with one per pass: the same bits."""
    ny, nx = shape
    banner(f"omega = 1 reverse pass vs general: {prec} {ny}x{nx}, {nsteps} steps, rows {rows2}, field {field}")
    monkeypatch.setenv("TFLBM_ADJ_FUSE", "2")
    if rows2 is not None:
        monkeypatch.setenv("TFLBM_ADJ_ROWS2", rows2)
    h0, th = random_case(ny, nx, 79)
    p = dict(tau=1.0, gamma=0.02, g=1e-3, hstar=0.15, delta=0.8, ax=2e-5, ay=-1e-5)
    if prec != "fp64":
        p["href"] = 0.45
    g = torch.Generator().manual_seed(80)
    grad_h = torch.randn((ny, nx), generator=g, dtype=torch.float64)
    runs = []
    for omega1 in ("1", "0"):
        monkeypatch.setenv("TFLBM_OMEGA1", omega1)
        for fused in (True, False):
            runs.append(_reverse_pass(prec, h0, th, p, nsteps, grad_h, fused, field))
    for other in runs[1:]:
        for x, y, name in ((other[0], runs[0][0], "dL/dh0"), (other[1], runs[0][1], "dL/dtheta")):
            assert torch.isfinite(y).all(), name
            nd = int((x != y).sum())
            assert nd == 0, (name, nd, float((x - y).abs().max()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_keeping_every_capture_equals_checkpoint_and_recompute(prec):
    """K = 0 keeps the captures the forward writes instead of checkpoints and
    a recompute; every step and every reverse step rounds the same way, so the
    final height and both gradients agree bit for bit with K = 5 (odd step
    count, segments not a multiple of the fused pair)."""
    from paper_1810_07642_amd import TFLBMRun
    ny, nx, steps = 41, 67, 23
    banner(f"{prec}: all captures kept vs checkpoints every 5 steps, {ny}x{nx}, {steps} steps")
    p = dict(tau=0.8, gamma=0.02, g=1e-3, hstar=0.15, delta=0.8, ax=2e-5, ay=-1e-5)
    if prec != "fp64":
        p["href"] = 0.45
    h0, th = random_case(ny, nx, 95)
    g = torch.Generator().manual_seed(96)
    grad_h = torch.randn((ny, nx), generator=g, dtype=torch.float64)
    res = []
    for K in (0, 5):
        h0c = h0.cuda().requires_grad_(True)
        thc = th.cuda().requires_grad_(True)
        h = TFLBMRun.apply(h0c, thc, p, steps, K, prec)
        h.backward(grad_h.cuda())
        torch.cuda.synchronize()
        res.append((h.detach().cpu(), h0c.grad.cpu(), thc.grad.cpu()))
    for a, b in zip(res[0], res[1]):
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)


def test_binding_rejects_buffers_it_cannot_hand_to_the_library():
    """Host tensors and short buffers are refused before any HIP call."""
    from paper_1810_07642_amd import Sim
    h0, th = random_case(12, 20, 7)
    sim = Sim(20, 12, "fp32", device="cuda", tau=0.9, gamma=0.01, hstar=0.1).init(h0, th)
    assert sim.device.index is not None
    adj = torch.empty(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sim.adj_seed(torch.empty(sim.adj_bytes(), dtype=torch.uint8), torch.zeros(12, 20))
    with pytest.raises(ValueError):
        sim.adj_seed(adj[:-1], torch.zeros(12, 20))
    sim.adj_seed(adj, torch.zeros(12, 20))
    cap = torch.empty(3 * sim.capture_bytes(), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sim.step_capture(4, cap)
    with pytest.raises(ValueError):
        sim.adj_steps(adj, cap, 4)
    with pytest.raises(ValueError):
        sim.state_load(torch.empty(sim.state_bytes(), dtype=torch.uint8), 0)
    sim.step_capture(3, cap)
    sim.adj_steps(adj, cap, 3)
    g_h0, g_th = sim.adj_finish(adj)
    torch.cuda.synchronize()
    assert torch.isfinite(g_h0).all() and torch.isfinite(g_th).all()

#!/usr/bin/env python3
"""Throughput of the thin-film lattice Boltzmann step on one MI355X.

Workload (the headline configuration): patterned-substrate dewetting on a
4096 x 4096 periodic lattice, FP32 population storage, contact-angle stripes
of period 256 alternating pi/9 and pi/4 (sine-smoothed edges, width 8), flat
film h0 = 0.1 + 1e-4 U(-1, 1) (seed 2), h_* = 0.09, gamma = 0.01, tau = 1,
delta = 1.  A "step" is one lattice time step of the whole grid; the library
runs two steps per launch of its fused step kernel (the intermediate state
stays on chip); MLUPS = nx ny steps / (t 1e6) (Sec. IV of the paper).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Besides the headline FP32 number it reports the FP64
and FP16-shifted forms, their errors against the FP64 path, the FP32/FP64
speed-up, the adjoint/forward time ratio of the inverse-design case
(512 x 512, 4096 steps, checkpoints every 64), the roofline position of the
step kernel and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
BYTES_PER_SITE = {"fp64": 152, "fp32": 76, "fp16s": 44}  # read + write 9 populations, + kappa field
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "step_fp32_dewetting4096_traffic.md")
# the step kernel and the launch plan that sets its tiles (its traffic depends on both)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1810_07642_amd", "csrc", f) for f in ("fwd.hip", "device.h", "api.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the step kernel's and its launch plan's source code with
    comments and blank lines removed, so that the committed counter summary
    stays valid across edits of comments only."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        text = open(p).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def committed_traffic():
    """(HBM bytes per step-kernel launch, time steps per launch) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source; else None."""
    if not os.path.exists(PROFILE_SUMMARY):
        return None
    text = open(PROFILE_SUMMARY).read()
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_steps = re.search(r"steps_per_launch:\s*([0-9]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1)), int(m_steps.group(1)) if m_steps else 1


def timed_steps(sim, steps, warmup):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)  # ms


def run_form(prec, p, h0, th, steps, warmup, fuse=None, href=0.0):
    from paper_1810_07642_amd import Sim
    import torch
    n = h0.shape[0]
    if fuse is not None:
        os.environ["TFLBM_FUSE"] = str(fuse)
    try:
        sim = Sim(n, n, prec, href=href, **p).init(h0, th)
    finally:
        os.environ.pop("TFLBM_FUSE", None)
    ms = timed_steps(sim, steps, warmup)
    sim.check()
    h = sim.height()
    mass = sim.mass()
    del sim
    torch.cuda.empty_cache()
    return ms, h, mass


def adjoint_ratio(prec="fp32", n=512, steps=4096, K=64):
    """Backward (recompute + adjoint) over forward (with checkpoints) wall time
    of the inverse-design case; with K = 0 the forward writes every step's
    capture and the backward is the reverse pass alone."""
    import torch
    from paper_1810_07642_amd import TFLBMRun, inputs
    p, h0, th, target = inputs.inverse_design(n=n)
    tgt = target.cuda()
    res = []
    for _ in range(2):  # first pass warms up
        h0c = h0.cuda().requires_grad_(True)
        thc = th.cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = TFLBMRun.apply(h0c, thc, p, steps, K, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * ((h - tgt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res.append((t1 - t0, t2 - t1))
    fwd, bwd = res[-1]
    return {"forward_s": fwd, "backward_s": bwd, "ratio": bwd / fwd, "grid": n, "steps": steps,
            "checkpoint_every": K, "storage": prec}


def reverse_sweep_at(n, K=16):
    """Per-step times of the pieces of the backward pass at n x n (the dewetting
    recipe, FP32): forward step, recompute with capture, and the adjoint, both
    two steps per pass (tflbm_adj_steps, what the backward pass runs) and one
    step per pass (tflbm_adj_step); the backward/forward ratio they give
    (checkpoint copies excluded).  Algorithmic bytes per site and step: 104
    one step per pass (adjoint read and write 36 + 36, h and j 12, kappa 4,
    FP64 g_kappa read and write 16), 58 two steps per pass (116 per pass:
    two captures, one adjoint read and write, one g_kappa update)."""
    import ctypes
    import torch
    from paper_1810_07642_amd import Sim, inputs
    p, h0, th = inputs.patterned_dewetting(n=n)
    sim = Sim(n, n, "fp32", href=0.1, **p).init(h0, th)
    cb = sim.capture_bytes()
    cap = torch.empty(K * cb, dtype=torch.uint8, device="cuda")
    adj = torch.zeros(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
    sim.adj_seed(adj, torch.zeros(n, n, dtype=torch.float64))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    def adjoint_single():
        for t in range(K - 1, -1, -1):
            sim.lib.tflbm_adj_step(sim.h, ctypes.c_void_p(adj.data_ptr()), ctypes.c_void_p(cap.data_ptr() + t * cb),
                                   sim.stream)

    f = timed(lambda: sim.step(K))
    c = timed(lambda: sim.step_capture(K, cap))
    a2 = timed(lambda: sim.adj_steps(adj, cap, K))
    a1 = timed(adjoint_single)
    del sim, cap, adj
    torch.cuda.empty_cache()
    return {"grid": n, "forward_us_per_step": round(f * 1e3, 1), "capture_us_per_step": round(c * 1e3, 1),
            "adjoint_us_per_step": round(a2 * 1e3, 1), "ratio": round((c + a2) / f, 3),
            "adjoint_GBps_at_58B_per_site": round(58 * n * n / (a2 * 1e-3) / 1e9, 1),
            "adjoint_one_step_per_pass_us_per_step": round(a1 * 1e3, 1),
            "ratio_one_step_per_pass": round((c + a1) / f, 3),
            "adjoint_one_step_per_pass_GBps_at_104B_per_site": round(104 * n * n / (a1 * 1e-3) / 1e9, 1)}


def fp64_by_lattice(mlups_4096):
    """FP64 MLUPS of the dewetting recipe at the lattice sizes of the paper's
    benchmark table (Sec. IV), the 4096^2 figure taken from the main run."""
    from paper_1810_07642_amd import inputs
    out = {}
    for n, steps in ((128, 2000), (256, 2000), (512, 1000), (1024, 500), (2048, 200)):
        p, h0, th = inputs.patterned_dewetting(n=n)
        # the warm-up runs past the point (256 steps) from which a handle on a
        # launch-bound lattice captures its step graph, so that the capture is
        # not timed
        ms, _, _ = run_form("fp64", p, h0, th, steps, 512)
        out[str(n)] = round(n * n * steps / (ms * 1e-3) / 1e6, 1)
    out["4096"] = round(mlups_4096, 1)
    return out


def cpu_oracle_one_thread(n=1024, budget_s=6.0):
    """The FP64 oracle on one host thread (the paper's CPU figure is one core),
    whole steps of the n x n dewetting recipe for about budget_s seconds."""
    import torch
    from oracle import lbm
    from paper_1810_07642_amd import inputs
    p, h0, th = inputs.patterned_dewetting(n=n)
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        P = lbm.Params(**p)
        kap = lbm.kappa(th, P)
        f = lbm.init(h0, P)
        t0 = time.perf_counter()
        done = 0
        while done < 1 or (time.perf_counter() - t0 < budget_s and done < 20):
            f = lbm.step(f, kap, P)
            done += 1
        dt = time.perf_counter() - t0
    finally:
        torch.set_num_threads(nthreads)
    return {"value": round(n * n * done / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{done} whole steps of the {n}x{n} dewetting recipe, FP64, {dt:.1f} s"}


def cpu_baseline(p, h0, th, budget_s=12.0):
    """The FP64 oracle (never tuned) on the host cores: whole steps of the same
    4096 x 4096 workload until ~budget_s of CPU work, at least two."""
    import torch
    from oracle import lbm
    P = lbm.Params(**p)
    kap = lbm.kappa(th, P)
    f = lbm.init(h0, P)
    t0 = time.perf_counter()
    done = 0
    while done < 2 or (time.perf_counter() - t0 < budget_s and done < 6):
        f = lbm.step(f, kap, P)
        done += 1
    dt = time.perf_counter() - t0
    n = h0.numel()
    return {"value": n * done / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{done} whole steps of the {h0.shape[1]}x{h0.shape[0]} dewetting workload, FP64, "
                      f"{dt:.1f} s",
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical CPU count of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "os_cpu_count": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=4096, help="lattice side (default 4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline FP32 number only")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run this many FP32 steps and a 1 GiB device copy (for rocprofv3), then exit")
    ap.add_argument("--profile-adjoint", type=int, default=0,
                    help="run the reverse pass over this many captured FP32 steps and a 1 GiB device copy "
                         "(for rocprofv3), then exit")
    ap.add_argument("--profile-storage", default="fp32", choices=("fp64", "fp32", "fp16s"),
                    help="storage form of the --profile-steps run (default fp32)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the thin-film step runs on a single MI355X "
              "(the library has no multi-GPU slab decomposition)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_07642_amd import Sim, inputs

    n = args.n
    p, h0, th = inputs.patterned_dewetting(n=n)
    # FP32 storage as deviations from the rest equilibrium at the mean film height
    href = 0.1

    if args.profile_steps or args.profile_adjoint:
        prec = "fp32" if args.profile_adjoint else args.profile_storage
        sim = Sim(n, n, prec, href=0.0 if prec == "fp64" else href, **p).init(h0, th)
        if args.profile_adjoint:
            k = args.profile_adjoint
            cap = torch.empty(k * sim.capture_bytes(), dtype=torch.uint8, device="cuda")
            adj = torch.empty(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
            sim.step_capture(k, cap)
            sim.adj_seed(adj, torch.zeros(n, n, dtype=torch.float64))
            sim.adj_steps(adj, cap, k)
        else:
            sim.step(args.profile_steps)
        torch.cuda.synchronize()
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        what = f"reverse pass over {args.profile_adjoint} captured" if args.profile_adjoint else f"{args.profile_steps}"
        log(f"profile run: {what} {prec} steps at {n}^2 and a 1 GiB copy")
        return

    ms32, h32, m32 = run_form("fp32", p, h0, th, args.steps, args.warmup, href=href)
    ms_step = ms32 / args.steps
    sites = n * n
    mlups = sites * args.steps / (ms32 * 1e-3) / 1e6
    achieved = BYTES_PER_SITE["fp32"] * sites / (ms_step * 1e-3) / 1e9
    traffic = committed_traffic()
    line = {
        "metric": "D2Q9 thin-film MLUPS, % HBM roofline, FP32/FP64 speedup, adjoint/forward time",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"patterned-substrate dewetting {n}x{n}, FP32 storage, stripe theta field",
                   "nx": n, "ny": n, "storage": "fp32", "href": href, "theta": "stripes pi/9 | pi/4, period 256",
                   "hstar": p["hstar"], "tau": p["tau"], "gamma": p["gamma"], "delta": p["delta"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic[0] / (traffic[1] * ms_step * 1e-3) / 1e9, 1),
                     "kernel": "step_kernel<fp32, kappa field, 2 fused steps>", "site_updates_per_launch": 2,
                     "bytes_per_site_update": BYTES_PER_SITE["fp32"],
                     # one launch advances two steps but reads and writes every record once:
                     # frac above counts the bytes of two separate steps, per_pass the bytes of one pass
                     "per_pass": {"bytes_per_site": BYTES_PER_SITE["fp32"],
                                  "achieved": round(achieved / 2, 1),
                                  "frac": round(achieved / 2 / HBM_PEAK_GBS, 4)}},
    }
    log(f"fp32: {ms_step * 1e3:.1f} us/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")

    if not args.no_extras:
        extras = {}
        k64 = max(50, args.steps // 4) // 2 * 2
        ms64, h64, m64 = run_form("fp64", p, h0, th, k64, 20)
        ms16, h16, m16 = run_form("fp16s", p, h0, th, args.steps, args.warmup, href=href)
        mlups64 = sites * k64 / (ms64 * 1e-3) / 1e6
        mlups16 = sites * args.steps / (ms16 * 1e-3) / 1e6
        # accuracy against the FP64 path after the same number of steps
        from paper_1810_07642_amd import Sim as _S
        total = args.steps + args.warmup
        s64 = _S(n, n, "fp64", **p).init(h0, th)
        s64.step(total)
        h64ref = s64.height()
        del s64
        torch.cuda.empty_cache()
        scale = float(h64ref.abs().max())
        extras["fp64"] = {"mlups": round(mlups64, 1), "ms_per_step": round(ms64 / k64, 5),
                          "hbm_frac": round(BYTES_PER_SITE["fp64"] * mlups64 * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
        extras["fp16s"] = {"mlups": round(mlups16, 1), "ms_per_step": round(ms16 / args.steps, 5),
                           "hbm_frac": round(BYTES_PER_SITE["fp16s"] * mlups16 * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                           "max_rel_dh_vs_fp64": float((h16 - h64ref).abs().max()) / scale}
        extras["fp32_max_rel_dh_vs_fp64"] = float((h32 - h64ref).abs().max()) / scale
        _, h32p, _ = run_form("fp32", p, h0, th, args.steps, args.warmup, href=0.0)
        extras["fp32_href0_max_rel_dh_vs_fp64"] = float((h32p - h64ref).abs().max()) / scale
        del h32p
        extras["accuracy_after_steps"] = total
        ms1, _, _ = run_form("fp32", p, h0, th, k64, 20, fuse=1, href=href)
        extras["fp32_one_step_per_pass"] = {"mlups": round(sites * k64 / (ms1 * 1e-3) / 1e6, 1),
                                            "ms_per_step": round(ms1 / k64, 5)}
        extras["fp64_mlups_by_lattice"] = fp64_by_lattice(mlups64)
        extras["fp32_over_fp64_speedup"] = round(mlups / mlups64, 3)
        extras["fp16s_over_fp64_speedup"] = round(mlups16 / mlups64, 3)
        m0 = float(h0.sum())
        extras["mass_rel_drift"] = {"fp32": (m32 - m0) / m0, "fp16s": (m16 - m0) / m0}
        del h16, h64ref
        torch.cuda.empty_cache()
        extras["adjoint"] = adjoint_ratio()
        # the same case with every step's capture kept (K = 0: no checkpoints, no recompute)
        extras["adjoint_all_captures_kept"] = adjoint_ratio(K=0)
        extras["reverse_sweep_at_headline_size"] = reverse_sweep_at(n)
        line["extras"] = extras
        log(f"fp64 {mlups64:.0f} MLUPS, fp16s {mlups16:.0f} MLUPS, adjoint/forward {extras['adjoint']['ratio']:.2f}")

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, h0, th)
        log(f"cpu oracle: {line['cpu_baseline']['value']:.2f} MLUPS on {line['cpu_baseline']['cores']} threads")
        if "extras" in line:
            line["extras"]["cpu_oracle_one_thread"] = cpu_oracle_one_thread()

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

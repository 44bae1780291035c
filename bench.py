#!/usr/bin/env python3
"""Throughput of the thin-film lattice Boltzmann step on one MI355X.

Workload (the headline configuration): patterned-substrate dewetting on a
4096 x 4096 periodic lattice, contact-angle stripes of period 256 alternating
pi/9 and pi/4 (sine-smoothed edges, width 8), flat film h0 = 0.1 + 1e-4
U(-1, 1) (seed 2), h_* = 0.09, gamma = 0.01, tau = 1, delta = 1.  The headline
value is the FP64 step, the arithmetic of the paper's own benchmark table
(Sec. IV).  A "step" is one lattice time step of the whole grid; the library
runs two steps per launch of its fused step kernel (the intermediate state
stays on chip); MLUPS = nx ny steps / (t 1e6) (Sec. IV).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Besides the headline it reports, per storage form
(FP64, FP32, FP16-shifted) and for the two-step reverse pass, the roofline
position of the dominant kernel per pass (the bytes one launch must move over
its launch time, against the 8 TB/s HBM peak and against the record-copy
ceiling measured in the same run); the errors of the FP32 and FP16S forms
against the FP64 path after a fixed 2000 steps; the FP32/FP64 speed-up; the
adjoint/forward time ratio of the inverse-design case (512 x 512, 4096 steps,
checkpoints every 64) with the FP32-forward gradient error; and the FP64 CPU
oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
# Algorithmic bytes per site of one pass of the fused step kernel: read and
# write each of the 9 populations once, plus the kappa field read once.
BYTES_PER_SITE = {"fp64": 152, "fp32": 76, "fp16s": 44}
HREF = {"fp64": 0.0, "fp32": 0.1, "fp16s": 0.1}  # storage reference height: the film's mean
# Reverse pass, two steps per launch, FP32 adjoint with FP64 kappa gradient,
# at tau = 1 (the adjoint between steps as three fields per site): fields
# read and written 12 + 12, two captures 24, kappa 4, g_kappa RMW 16.  (The
# general pass moves nine adjoint populations each way: 116 B.)
ADJ2_BYTES_PER_SITE = 68
PROFILES = os.path.join(ROOT, "profiles")
EXTRA_STEPS = 400   # timed steps of each form in the per-form table (independent of --steps)
ACCURACY_STEPS = 2000  # fixed horizon of the accuracy legs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_path(form):
    return os.path.join(PROFILES, f"step_{form}_dewetting4096_traffic.md")


ADJ_PROFILE = os.path.join(PROFILES, "adj_step2_fp32_dewetting4096.md")


def committed_traffic(form):
    """(HBM bytes per launch, steps per launch) from the committed counter
    summary of the form's step kernel, if it was taken on the current kernel
    and launch-plan source; else None."""
    from paper_1810_07642_amd import profiling
    r = profiling.read_summary(profile_path(form), profiling.STEP_SOURCES)
    return None if r is None else r[:2]


def committed_adj_traffic():
    from paper_1810_07642_amd import profiling
    r = profiling.read_summary(ADJ_PROFILE, profiling.ADJ_SOURCES)
    return None if r is None else r[:2]


def cuda_timer():
    """Start/stop events on the stream the library launches on (torch's
    current stream, which Sim hands to every C-ABI call)."""
    import torch
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return stream, e0, e1


def timed_steps(sim, steps, warmup):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    stream, e0, e1 = cuda_timer()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)  # ms


def make_sim(prec, p, h0, th, fuse=None, href=None):
    from paper_1810_07642_amd import Sim
    n = h0.shape[0]
    if fuse is not None:
        os.environ["TFLBM_FUSE"] = str(fuse)
    try:
        return Sim(n, n, prec, href=HREF[prec] if href is None else href, **p).init(h0, th)
    finally:
        os.environ.pop("TFLBM_FUSE", None)


def general_stages(sims, p, h0, th, ceil_gbs):
    """The same workload and state with the general collision stages
    (TFLBM_OMEGA1=0: the stages that keep the populations, as any tau != 1
    needs; two steps per pass): what the step costs when tau != 1."""
    import torch
    out = {}
    sites = h0.numel()
    for prec in ("fp64", "fp32", "fp16s"):
        os.environ["TFLBM_OMEGA1"] = "0"
        try:
            sim = make_sim(prec, p, h0, th)
        finally:
            os.environ.pop("TFLBM_OMEGA1", None)
        sim.state_load(sims[prec].state_save(), sims[prec].steps)
        ms = timed_steps(sim, EXTRA_STEPS, 20)
        sim.check()
        spp = sim.steps_per_pass
        out[prec] = {"mlups": round(sites * EXTRA_STEPS / (ms * 1e-3) / 1e6, 1), "steps_per_pass": spp,
                     "roofline_frac": roofline_block("general stages", BYTES_PER_SITE[prec] * sites,
                                                     ms / launches(EXTRA_STEPS, spp), None, ceil_gbs)["frac"]}
        del sim
        torch.cuda.empty_cache()
    return out


def run_form(prec, p, h0, th, steps, warmup, fuse=None, href=None):
    import torch
    sim = make_sim(prec, p, h0, th, fuse, href)
    ms = timed_steps(sim, steps, warmup)
    sim.check()
    del sim
    torch.cuda.empty_cache()
    return ms


def launches(steps, per_pass):
    """Launches of the step kernel for `steps` steps with at most `per_pass`
    steps per pass (the last pass may be shorter)."""
    return -(-steps // per_pass)


def step_kernel_name(sim, prec):
    spp = sim.steps_per_pass
    return f"step_kernel<{prec}, kappa field, {spp} fused steps{', omega = 1 stages' if sim.params.tau == 1.0 else ''}>"


def roofline_block(kernel, bytes_per_launch, launch_ms, traffic, ceiling_gbs, steps_per_launch=2):
    """Roofline position of one kernel: its algorithmic bytes per launch over
    its launch time, against the HBM peak (frac) and the record-copy ceiling;
    `traffic` = (measured HBM bytes per launch, steps per launch) from the
    committed counter summary, or None."""
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    blk = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(traffic[0] / (launch_ms * 1e-3) / 1e9, 1),
           "kernel": kernel, "bytes_per_launch": int(bytes_per_launch), "steps_per_launch": steps_per_launch,
           "launch_us": round(launch_ms * 1e3, 2)}
    if traffic is not None:
        blk["traffic_over_algorithmic"] = round(traffic[0] / bytes_per_launch, 4)
    if ceiling_gbs:
        blk["ceiling"] = {"GBps": round(ceiling_gbs, 1), "what": "record copy (tflbm_state_save) of the same buffer",
                          "frac_of_ceiling": round(achieved / ceiling_gbs, 4)}
    return blk


def copy_ceiling(p, h0, th, reps=20):
    """The library's record-copy kernel (tflbm_state_save: one read and one
    write of every byte of a population buffer) on the FP64 state of the
    benchmark lattice, and the runtime's device copy of the same bytes:
    GB/s counting bytes read + written."""
    import torch
    sim = make_sim("fp64", p, h0, th)
    nbytes = sim.state_bytes()
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        sim.state_save(dst)
        dst.copy_(src)
    torch.cuda.synchronize()
    stream, e0, e1 = cuda_timer()
    e0.record(stream)
    for _ in range(reps):
        sim.state_save(dst)
    e1.record(stream)
    torch.cuda.synchronize()
    t_rec = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    t_rt = e0.elapsed_time(e1) / reps
    del sim, dst, src
    torch.cuda.empty_cache()
    return {"record_copy_GBps": round(2 * nbytes / (t_rec * 1e-3) / 1e9, 1),
            "runtime_copy_GBps": round(2 * nbytes / (t_rt * 1e-3) / 1e9, 1), "bytes_copied": nbytes}


def steady_sims(p, h0, th, steps=ACCURACY_STEPS, forms=("fp64", "fp32", "fp32_href0", "fp16s")):
    """Handles of each form advanced `steps` untimed steps from the flat film,
    and the accuracy of the FP32 and FP16S forms against the FP64 path there
    (max |dh| / max h) with the mass drift of each form.  Timing starts from
    these states: over its first ~60 steps from the flat initial film the step
    runs up to 15 % slower per launch than later in the run (measured at
    4096^2 FP64: 595-675 us per launch, against 577-590 us after 2000 steps),
    and the paper's MLUPS are averages over 10^5 steps."""
    import torch
    sims, acc = {}, {"steps": steps, "mass_rel_drift": {}}
    ref = None
    for key in forms:
        prec = "fp32" if key == "fp32_href0" else key
        sim = make_sim(prec, p, h0, th, href=0.0 if key == "fp32_href0" else None)
        m0 = sim.mass()
        sim.step(steps)
        sim.check()
        h = sim.height()
        acc["mass_rel_drift"][key] = (sim.mass() - m0) / m0
        if key == "fp64":
            ref = h
        else:
            acc[f"{key}_max_rel_dh_vs_fp64"] = float((h - ref).abs().max()) / float(ref.abs().max())
        del h
        if key == "fp32_href0":
            del sim
        else:
            sims[key] = sim
    del ref
    torch.cuda.empty_cache()
    return sims, acc


def inverse_design_case(prec="fp32", n=512, steps=4096, K=64, reps=2):
    """Backward (recompute + adjoint) over forward (with checkpoints) wall time
    of the inverse-design case, and the gradients of the last repetition; with
    K = 0 the forward writes every step's capture and the backward is the
    reverse pass alone."""
    import torch
    from paper_1810_07642_amd import TFLBMRun, inputs
    p, h0, th, target = inputs.inverse_design(n=n)
    tgt = target.cuda()
    res = []
    for _ in range(reps):  # the first pass warms up
        h0c = h0.cuda().requires_grad_(True)
        thc = th.cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = TFLBMRun.apply(h0c, thc, dict(p, href=HREF[prec]), steps, K, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * ((h - tgt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res.append((t1 - t0, t2 - t1))
    fwd, bwd = res[-1]
    info = {"forward_s": round(fwd, 5), "backward_s": round(bwd, 5), "ratio": round(bwd / fwd, 4), "grid": n,
            "steps": steps, "checkpoint_every": K, "storage": prec, "href": HREF[prec]}
    return info, (h0c.grad.detach(), thc.grad.detach())


def reverse_sweep_at(n, ceiling_gbs, K=18):
    """Per-step times of the pieces of the backward pass at n x n (the dewetting
    recipe, FP32): forward step, recompute with capture, and the adjoint, both
    two steps per pass (tflbm_adj_steps, what the backward pass runs) and one
    step per pass (tflbm_adj_step); the backward/forward ratio they give
    (checkpoint copies excluded), and the roofline block of the two-step
    reverse kernel (68 B per site and pass at tau = 1).  K = 18 steps are whole
    passes of each piece (six of three forward or recompute steps, nine of two
    reverse steps), so every piece is timed at its steady per-step rate."""
    import ctypes
    import torch
    from paper_1810_07642_amd import Sim, inputs
    p, h0, th = inputs.patterned_dewetting(n=n)
    sim = Sim(n, n, "fp32", href=HREF["fp32"], **p).init(h0, th)
    sim.step(ACCURACY_STEPS)  # past the start-up transient of the flat film, as for the forward timings
    cb = sim.capture_bytes()
    cap = torch.empty(K * cb, dtype=torch.uint8, device="cuda")
    adj = torch.zeros(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
    sim.adj_seed(adj, torch.zeros(n, n, dtype=torch.float64))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        stream, e0, e1 = cuda_timer()
        e0.record(stream)
        fn()
        e1.record(stream)
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
            "adjoint_one_step_per_pass_us_per_step": round(a1 * 1e3, 1),
            "ratio_one_step_per_pass": round((c + a1) / f, 3),
            "roofline": roofline_block("adj_step2_kernel<float, kappa field, three adjoint fields per site> "
                                       "(two reverse steps per launch)",
                                       ADJ2_BYTES_PER_SITE * n * n, 2 * a2, committed_adj_traffic(), ceiling_gbs)}


def whole_workload(p, h0, th, steps=20000, prec="fp64"):
    """MLUPS over the workload's whole run, from the flat initial film, timed
    as one region (the paper's metric: a run's sites x steps over its
    simulation time, Sec. IV)."""
    import torch
    sim = make_sim(prec, p, h0, th)
    torch.cuda.synchronize()
    stream, e0, e1 = cuda_timer()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sim.check()
    ms = e0.elapsed_time(e1)
    n = h0.numel()
    del sim
    torch.cuda.empty_cache()
    return {"mlups": round(n * steps / (ms * 1e-3) / 1e6, 1), "steps": steps, "storage": prec, "seconds": round(ms / 1e3, 3)}


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
        ms = run_form("fp64", p, h0, th, steps, 512)
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


def profile_run(args, p, h0, th):
    """Short runs for rocprofv3: N steps of one form (and a record copy of its
    state), or a reverse pass over N captured FP32 steps; then a 1 GiB runtime
    copy that calibrates the HBM counters."""
    import torch
    n = args.n
    prec = "fp32" if args.profile_adjoint else args.profile_storage
    sim = make_sim(prec, p, h0, th)
    if args.profile_adjoint:
        k = args.profile_adjoint
        cap = torch.empty(k * sim.capture_bytes(), dtype=torch.uint8, device="cuda")
        adj = torch.empty(sim.adj_bytes(), dtype=torch.uint8, device="cuda")
        sim.step_capture(k, cap)
        sim.adj_seed(adj, torch.zeros(n, n, dtype=torch.float64))
        sim.adj_steps(adj, cap, k)
    else:
        sim.step(args.profile_steps)
        sim.state_save()
    torch.cuda.synchronize()
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    what = f"reverse pass over {args.profile_adjoint} captured" if args.profile_adjoint else f"{args.profile_steps}"
    log(f"profile run: {what} {prec} steps at {n}^2 and a 1 GiB copy")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=4096, help="lattice side (default 4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline FP64 number and its roofline only")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run this many steps, a record copy and a 1 GiB device copy (for rocprofv3), then exit")
    ap.add_argument("--profile-adjoint", type=int, default=0,
                    help="run the reverse pass over this many captured FP32 steps and a 1 GiB device copy "
                         "(for rocprofv3), then exit")
    ap.add_argument("--profile-storage", default="fp64", choices=("fp64", "fp32", "fp16s"),
                    help="storage form of the --profile-steps run (default fp64)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the thin-film step runs on a single MI355X "
              "(the library has no multi-GPU slab decomposition)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_07642_amd import inputs

    n = args.n
    sites = n * n
    p, h0, th = inputs.patterned_dewetting(n=n)

    if args.profile_steps or args.profile_adjoint:
        profile_run(args, p, h0, th)
        return

    extras = {}
    ceiling = copy_ceiling(p, h0, th)
    ceil_gbs = ceiling["record_copy_GBps"]
    # untimed: every form advanced ACCURACY_STEPS steps (the state the timing
    # starts from) and its accuracy against the FP64 path there
    sims, accuracy = steady_sims(p, h0, th, forms=("fp64",) if args.no_extras else
                                 ("fp64", "fp32", "fp32_href0", "fp16s"))
    if not args.no_extras:
        extras["accuracy"] = accuracy
        log(f"accuracy after {ACCURACY_STEPS} steps: {accuracy}")

    # headline: FP64, exactly --steps timed steps after --warmup untimed ones,
    # continuing the workload from step ACCURACY_STEPS
    ms64 = timed_steps(sims["fp64"], args.steps, args.warmup)
    sims["fp64"].check()
    ms_step = ms64 / args.steps
    mlups = sites * args.steps / (ms64 * 1e-3) / 1e6
    spp64 = sims["fp64"].steps_per_pass
    launch_ms = ms64 / launches(args.steps, spp64)
    roof = roofline_block(step_kernel_name(sims["fp64"], "fp64"), BYTES_PER_SITE["fp64"] * sites,
                          launch_ms, committed_traffic("fp64"), ceil_gbs, steps_per_launch=spp64)
    roof["per_step_equivalent_GBps"] = round(BYTES_PER_SITE["fp64"] * sites / (ms_step * 1e-3) / 1e9, 1)
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"patterned-substrate dewetting {n}x{n}, FP64 storage and arithmetic, "
                               "stripe theta field",
                   "nx": n, "ny": n, "storage": "fp64", "theta": "stripes pi/9 | pi/4, period 256",
                   "hstar": p["hstar"], "tau": p["tau"], "gamma": p["gamma"], "delta": p["delta"]},
        "roofline": roof,
    }
    log(f"fp64: {ms_step * 1e3:.1f} us/step, {mlups:.0f} MLUPS, per pass {roof['achieved']:.0f} GB/s "
        f"({roof['frac']:.3f} of peak), record copy {ceil_gbs:.0f} GB/s")

    if not args.no_extras:
        extras["ceiling"] = ceiling
        forms = {}
        for prec in ("fp64", "fp32", "fp16s"):
            ms = timed_steps(sims[prec], EXTRA_STEPS, 50)
            sims[prec].check()
            ml = sites * EXTRA_STEPS / (ms * 1e-3) / 1e6
            spp = sims[prec].steps_per_pass
            lm = ms / launches(EXTRA_STEPS, spp)
            forms[prec] = {"mlups": round(ml, 1), "ms_per_step": round(ms / EXTRA_STEPS, 5),
                           "steps_timed": EXTRA_STEPS, "href": HREF[prec], "steps_per_pass": spp,
                           "roofline": roofline_block(step_kernel_name(sims[prec], prec),
                                                      BYTES_PER_SITE[prec] * sites, lm, committed_traffic(prec),
                                                      ceil_gbs, steps_per_launch=spp)}
            forms[prec]["roofline"]["per_step_equivalent_GBps"] = round(
                BYTES_PER_SITE[prec] * sites / (ms / EXTRA_STEPS * 1e-3) / 1e9, 1)
        for prec in ("fp32", "fp16s"):
            forms[prec]["speedup_over_fp64"] = round(forms[prec]["mlups"] / forms["fp64"]["mlups"], 3)
        extras["forms"] = forms
        extras["general_collision_stages"] = general_stages(sims, p, h0, th, ceil_gbs)
        extras["timing_starts_after_steps"] = ACCURACY_STEPS
        del sims
        torch.cuda.empty_cache()
        log("forms: " + ", ".join(f"{k} {v['mlups']:.0f} MLUPS ({v['steps_per_pass']} steps per pass, "
                                  f"pass frac {v['roofline']['frac']:.3f})" for k, v in forms.items()))
        log("general stages (tau != 1): " + ", ".join(f"{k} {v['mlups']:.0f} MLUPS"
                                                      for k, v in extras["general_collision_stages"].items()))
        s1 = make_sim("fp32", p, h0, th, fuse=1)
        s1.step(ACCURACY_STEPS)
        ms1 = timed_steps(s1, EXTRA_STEPS, 20)
        del s1
        extras["fp32_one_step_per_pass"] = {"mlups": round(sites * EXTRA_STEPS / (ms1 * 1e-3) / 1e6, 1),
                                            "ms_per_step": round(ms1 / EXTRA_STEPS, 5)}
        extras["fp64_mlups_by_lattice"] = fp64_by_lattice(forms["fp64"]["mlups"])
        extras["fp64_whole_workload"] = whole_workload(p, h0, th)
        log(f"fp64 over the whole 20000-step workload: {extras['fp64_whole_workload']['mlups']:.0f} MLUPS")
        adj32, g32 = inverse_design_case("fp32")
        _, g64 = inverse_design_case("fp64", reps=1)
        rel = [float((a - b).norm() / b.norm()) for a, b in zip(g32, g64)]
        adj32["fp32_forward_grad_rel_l2_vs_fp64"] = {"h0": rel[0], "theta": rel[1]}
        extras["adjoint"] = adj32
        del g32, g64
        torch.cuda.empty_cache()
        extras["adjoint_all_captures_kept"] = inverse_design_case("fp32", K=0)[0]
        extras["reverse_sweep_at_headline_size"] = reverse_sweep_at(n, ceil_gbs)
        extras["paper_context"] = {
            "note": "the paper's FP64 MLUPS table (Sec. IV), other hardware and code: context, not a target",
            "gtx1080ti_fp64_mlups_4096": 395.6, "i7_4790_one_core_fp64_mlups_4096": 4.3}
        line["extras"] = extras
        log(f"adjoint/forward {adj32['ratio']:.2f} (512^2, K = 64), fp32-forward gradient error {rel}")

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, h0, th)
        log(f"cpu oracle: {line['cpu_baseline']['value']:.2f} MLUPS on {line['cpu_baseline']['cores']} threads")
        if "extras" in line:
            line["extras"]["cpu_oracle_one_thread"] = cpu_oracle_one_thread()

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

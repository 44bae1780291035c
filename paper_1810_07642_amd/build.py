"""Builds libtflbm.so (HIP, gfx950) in the package directory.

    python -m paper_1810_07642_amd.build [-v]
"""
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtflbm.so")
# (object, source, defines): the step kernels of each storage form and
# collision stage are a translation unit of their own (step_form.hip with
# STEP_FORM and STEP_W1), so that the sources compile in parallel
UNITS = [(f"step_{form}_{'w1' if w1 else 'general'}", "step_form.hip", [f"-DSTEP_FORM={P}", f"-DSTEP_W1={w1}"])
         for form, P in (("f16s", "kF16S"), ("f32", "kF32"), ("f64", "kF64")) for w1 in (1, 0)]
UNITS += [(s[:-4], s, []) for s in ("adj.hip", "fwd.hip", "api.hip", "diag.hip", "noalloc.hip")]
SOURCES = sorted({src for _, src, _ in UNITS})
OBJ = os.path.join(PKG, "_build")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit fused multiply-add contraction: the kernels fuse where they
    # say so (madd, the reciprocal refinement), nowhere else
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
    # per-kernel register and scratch report (checked below)
    "-Rpass-analysis=kernel-resource-usage",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def spilling_kernels(remarks):
    """Kernels whose resource-usage remark reports scratch memory per lane."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            out.append(f"{name}: {m.group(1)} bytes per lane")
    return out


def build(verbose=False, jobs=None):
    """Compile every HIP source (in parallel, `jobs` at a time: default the
    CPU count, at most 8) and link libtflbm.so; raises on failure."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    pending = [(name, os.path.join(CSRC, src), os.path.join(OBJ, name + ".o"), defs) for name, src, defs in UNITS]
    running, remarks = [], []

    def wait_one():
        name, proc = running.pop(0)
        out, err = proc.communicate()
        if proc.returncode != 0:
            for _, other in running:
                other.wait()
            raise RuntimeError(f"hipcc failed on {name}:\n" + out + err)
        remarks.append(err)

    for name, src, obj, defs in pending:
        cmd = [hipcc()] + FLAGS + defs + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        if len(running) >= jobs:
            wait_one()
        running.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    while running:
        wait_one()
    tmp = LIB + ".tmp"
    link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [o for _, _, o, _ in pending]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    res.stderr = "\n".join(remarks)
    spills = spilling_kernels(res.stderr)
    if spills:
        raise RuntimeError("kernels spill registers to scratch memory (the step and reverse kernels are "
                           "sized to fit their register budget):\n" + "\n".join(spills))
    if verbose:
        print(f"{len(re.findall(r'Function Name:', res.stderr))} kernels, none spills", file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

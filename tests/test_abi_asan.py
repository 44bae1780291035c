"""Host memory safety of the C ABI: the library's host code built with
AddressSanitizer (device code as usual), driven by tests/asan_driver.c through
every call that needs no GPU — parameter checks, create/destroy of each
storage form, sizes, bind and call-order errors — with leak detection on.
Skipped when hipcc or ROCm's clang is absent."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1810_07642_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and ROCm clang")
def test_c_abi_host_paths_under_address_sanitizer(tmp_path):
    lib = tmp_path / "libtflbm_asan.so"
    srcs = [os.path.join(CSRC, f) for f in ("api.hip", "fwd.hip", "adj.hip", "diag.hip")]
    subprocess.run([HIPCC, "-std=c++17", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-Xarch_host", "-fsanitize=address", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-fPIC", "-shared", "-I" + os.path.join(ROOT, "include"), "-o", str(lib)] + srcs,
                   check=True, capture_output=True, timeout=600)
    exe = tmp_path / "asan_driver"
    subprocess.run([CLANG, "-g", "-fsanitize=address", "-I" + os.path.join(ROOT, "include"), "-o", str(exe),
                    os.path.join(HERE, "asan_driver.c"), "-L" + str(tmp_path), "-ltflbm_asan",
                    "-Wl,-rpath," + str(tmp_path)], check=True, capture_output=True, timeout=120)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok (0 failures)" in r.stdout

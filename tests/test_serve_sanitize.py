"""Race and memory checks of the request server's host code: the scheduler
(serve.cpp) and the host-only plan checks are built with g++ under the
thread sanitizer and then the address sanitizer, and a multi-threaded
dry-run stress (tests/serve_stress.cpp) must finish clean."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_00890_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.parametrize("sanitizer", ["thread", "address"])
def test_server_under_sanitizer(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "include", "hip")):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / f"serve_stress_{sanitizer}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={sanitizer}",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "serve.cpp"), os.path.join(CSRC, "plan_check.cpp"),
           os.path.join(ROOT, "tests", "serve_stress.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr

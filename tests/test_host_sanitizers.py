"""The host parts of the scene build (binned-SAH builder, quantizer, instance
opening) under the compiler's sanitizers, built with the host C++ compiler from
the library's own sources and driven by tests/host_builder_check.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_02620_amd", "csrc")


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_host_builder_under_sanitizer(tmp_path, san):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host C++ compiler or HIP headers")
    exe = tmp_path / "check"
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I", CSRC, os.path.join(ROOT, "tests", "host_builder_check.cpp"),
           os.path.join(CSRC, "bvh_build.cpp"), os.path.join(CSRC, "rebraid.cpp"), "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and "cannot find" in r.stderr:
        pytest.skip(f"sanitizer runtime missing: {r.stderr[-300:]}")
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0 and "ok" in run.stdout, (run.stdout[-2000:], run.stderr[-4000:])

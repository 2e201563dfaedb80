"""Host logic of the serving loop on the CPU: the scheduler source is built
with g++ and AddressSanitizer against a CPU stand-in for the device calls
(tests/host_sched/mock_device.cpp), then driven through admission under a
byte budget, coalesced launches, release of finished requests while later
ones still run, argument errors and shutdown."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1909_04539_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not shutil.which("g++") or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("needs g++ and the HIP headers")
    out = str(tmp_path_factory.mktemp("sched") / "scenarios")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, "server.cpp"), os.path.join(HERE, "host", "mock_device.cpp"),
           os.path.join(HERE, "host", "scenarios.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    return out


@pytest.mark.parametrize("scenario", ["mix", "budget", "errors", "shutdown", "early", "churn", "modes", "replay"])
def test_scheduler_scenario(exe, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, scenario], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr

"""The request server's policy (slp_scheduler.hpp) and threading
(slp_server_core.hpp), the code the server in libslp runs, against simulated
devices on the CPU: the policy under the host address and undefined-behaviour
sanitizers, the threading under the thread sanitizer (clang's runtime, whose
interceptors cover the condition-variable waits of std::condition_variable)
and under the address sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1305_3162_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_run(tmp_path, compiler, flags, source, name):
    exe = tmp_path / name
    cmd = [compiler, "-std=c++17", "-O1", "-g"] + flags + [
        "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", source), "-o", str(exe),
        "-lpthread"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_simulation(tmp_path):
    out = _build_run(tmp_path, "g++", ["-fsanitize=address,undefined"], "sched_sim.cpp",
                     "sched_sim")
    assert out.returncode == 0, out.stderr + out.stdout
    for name in ("chain_and_skip", "burst_is_one_launch", "bounded_wait_under_load",
                 "memory_backpressure_and_eviction", "oversized_and_errors", "random_stress"):
        assert f"OK {name}" in out.stdout
    assert "ALL OK" in out.stdout


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ not available")
def test_server_threads_under_thread_sanitizer(tmp_path):
    out = _build_run(tmp_path, CLANG, ["-fsanitize=thread"], "server_sim.cpp", "server_tsan")
    assert out.returncode == 0, out.stderr[-4000:] + out.stdout
    assert "ThreadSanitizer" not in out.stderr
    assert "ALL OK" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_server_threads_under_address_sanitizer(tmp_path):
    out = _build_run(tmp_path, "g++", ["-fsanitize=address,undefined"], "server_sim.cpp",
                     "server_asan")
    assert out.returncode == 0, out.stderr[-4000:] + out.stdout
    assert "ALL OK" in out.stdout

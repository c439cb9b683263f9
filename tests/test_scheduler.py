"""The request scheduler's policy (slp_scheduler.hpp, the code the server in
libslp runs) against a simulated device on the CPU, built with the host
address and undefined-behaviour sanitizers."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_simulation(tmp_path):
    exe = tmp_path / "sched_sim"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "paper_1305_3162_amd", "csrc"),
           os.path.join(ROOT, "tests", "sched_sim.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr + out.stdout
    for name in ("chain_and_skip", "memory_backpressure_and_eviction", "oversized_and_errors",
                 "random_stress"):
        assert f"OK {name}" in out.stdout
    assert "ALL OK" in out.stdout

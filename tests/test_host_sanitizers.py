"""The library's host logic under the address and undefined-behaviour
sanitizers (CPU only): the host sources of libslp are compiled with clang and
-fsanitize=address,undefined, the device sources as usual (their kernels are
never launched here), and tests/host_sanitize.cpp drives the host-only entry
points on inputs of the benchmark's sizes: the gridding and interpolation
tables of the 64-cell cube and of the 1024 x 1024 x 64 film, the near-field
index sets, the FEM assembly of the 32-cell tetrahedral cube and a multigrid
cycle built from it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1305_3162_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = "/opt/rocm/bin/hipcc"
HOST_SOURCES = ["slp_api.cpp", "slp_near.cpp", "slp_fem.cpp", "slp_amg.cpp", "slp_server.cpp"]
DEVICE_SOURCES = ["slp_kernels.hip", "slp_fft.hip", "slp_fem.hip", "slp_static.hip"]


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(HIPCC)),
                    reason="ROCm clang/hipcc not available")
def test_host_logic_under_address_and_ub_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined"]
    objs = []
    jobs = []
    for src in DEVICE_SOURCES:
        obj = str(tmp_path / (src + ".o"))
        cmd = [HIPCC, "-O1", "-std=c++17", "-fPIC", "-x", "hip", "--offload-arch=gfx950"] + inc + [
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c",
            os.path.join(CSRC, src), "-o", obj]
        jobs.append(subprocess.Popen(cmd, stderr=subprocess.DEVNULL))
        objs.append(obj)
    for src in HOST_SOURCES + [os.path.join(ROOT, "tests", "host_sanitize.cpp")]:
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [CLANG, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + \
            inc + san + ["-c", path, "-o", obj]
        jobs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for j in jobs:
        assert j.wait() == 0
    exe = str(tmp_path / "host_sanitize")
    subprocess.run([CLANG] + san + ["-o", exe] + objs +
                   ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert out.returncode == 0, out.stderr[-4000:] + out.stdout
    for line in ("OK cube64 tables", "OK film tables", "OK near-field host logic",
                 "OK fem assembly and multigrid cycle", "ALL OK"):
        assert line in out.stdout

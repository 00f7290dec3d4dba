"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU, no GPU needed): the HIP sources are compiled with the
sanitizers on their host side only (device code unchanged), linked into
tests/host_sanitizers/driver.cpp, which drives argument validation of every
entry point, the host arithmetic (trace distance, the blockBP update's
least-squares fit), workspace and memory estimates and the request server's
admission checks; any sanitizer report fails the run."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_05844_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize=function", "-Xarch_host", "-fno-omit-frame-pointer"]
# sources with device code are compiled whole; the others for the host only
FULL = ("bbp_kernels.hip", "bbp_api.hip", "bbp_svd.hip")
HOST_ONLY = ("bbp_server.hip", "bbp_ite.hip")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not installed")
def test_host_paths_are_sanitizer_clean(tmp_path):
    procs, objs = [], []
    for src in FULL + HOST_ONLY:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        if src in HOST_ONLY:
            cmd.append("--cuda-host-only")
        cmd += HOST_SAN + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out.decode()[-2000:]
    drv = str(tmp_path / "driver.o")
    san = ["-fsanitize=address,undefined", "-fno-sanitize=function"]
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + san +
                   ["-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(ROOT, "tests", "host_sanitizers", "driver.cpp"), "-o", drv],
                   check=True, timeout=300)
    exe = str(tmp_path / "driver")
    subprocess.run([CLANG] + san + ["-o", exe, drv] + objs +
                   ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-pthread",
                    "-Wl,-rpath," + os.path.join(ROCM, "lib")], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    print(run.stdout, run.stderr[-3000:])
    assert run.returncode == 0, run.stderr[-3000:]
    assert "host paths clean" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)

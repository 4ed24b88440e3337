"""The CPU oracle and the host side of libmpmc built with
-fsanitize=address,undefined, each driven through its chain, state and
error paths by a small driver in tests/sanitize/ (no GPU: the library
calls used touch only host code).  GPU code is not sanitized: the host
flags sit behind -Xarch_host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, (cmd[:3], r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_asan")
    srcs = [os.path.join(SAN, "oracle_driver.c")] + [
        os.path.join(ROOT, "oracle", f) for f in ("mpmc_oracle.c", "serial_ref.c", "sphere_oracle.c")]
    run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp"] + srcs + ["-lm", "-o", exe])
    r = run([exe], env=ENV)
    assert "sanitized oracle run ok" in r.stdout


def test_host_library_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    csrc = os.path.join(ROOT, "paper_1211_1646_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
              "-I", os.path.join(ROOT, "include")]
    gpu = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = []
    for f in ("mpmc_kernels.hip", "mpmc_mlp.hip", "mpmc_api.cpp", "sphere_kernels.hip",
              "sphere_api.cpp"):
        o = str(tmp_path / (f + ".o"))
        run([hipcc] + common + gpu + san + ["-x", "hip", "-c", os.path.join(csrc, f), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "drv.o")
    run([hipcc] + common + san + ["-x", "c++", "-c", os.path.join(SAN, "host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_asan")
    run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined",
         "-o", exe, drv] + objs)
    # the HIP runtime keeps allocations of its own until exit: leaks are not checked here
    r = run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"))
    assert "sanitized host library run ok" in r.stdout

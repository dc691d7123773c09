"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: `api.cpp` is rebuilt with both sanitizers on its
host side (device code is not instrumented), linked with the library's
other objects into `tests/abi_host_check.cpp`, and run.  The program drives
the C-ABI's host paths (graph and parameter validation, workspace sizes,
defaults, the autotuner cache file) and needs no GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2605_06921_amd")
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
OTHERS = ["grid_kernels.hip", "tile_kernel.hip", "toy_kernel.hip", "static_scratch.hip"]


def _objects_current():
    for src in OTHERS:
        obj = os.path.join(BUILD, src + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(os.path.join(CSRC, src)):
            return False
    return True


def _run(cmd, cwd):
    proc = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert proc.returncode == 0, f"{' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}"
    return proc


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not _objects_current():
        sys.path.insert(0, PKG)
        import build  # the package's own build script
        build.build(verbose=False)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC] + san + ["-c", os.path.join(CSRC, "api.cpp"), "-o", "api_san.o"], tmp_path)
    host = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    _run([CLANG, "-std=c++17", "-g"] + host + ["-I", os.path.join(ROOT, "include"), "-c",
                                               os.path.join(ROOT, "tests", "abi_host_check.cpp"), "-o", "check.o"],
         tmp_path)
    _run([CLANG] + host + ["check.o", "api_san.o"] + [os.path.join(BUILD, s + ".o") for s in OTHERS] +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", "abi_check"], tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("MQO_TUNE_CACHE", None)
    proc = subprocess.run([str(tmp_path / "abi_check"), str(tmp_path)], capture_output=True, text=True, env=env,
                          timeout=120)
    out = proc.stdout + proc.stderr
    assert proc.returncode == 0, out
    assert "0 failure(s)" in out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out

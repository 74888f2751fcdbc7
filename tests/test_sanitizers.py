"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library: a build of csrc/lbm_vans.hip whose host code carries both sanitizers
  (device code built at -O0, only to link; it never runs here), driven through its
  argument checks, layouts and error paths by tests/sanitize_child.py.
* The oracle: a gcc build with both sanitizers running the oracle's pin suites.
Each runs in a child process with the sanitizer runtime preloaded and fails on the
first report.
"""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _clang_asan():
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return libs[0] if libs else None


def _gcc_lib(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


@pytest.mark.skipif(not os.path.exists(HIPCC) or _clang_asan() is None,
                    reason="hipcc or the clang AddressSanitizer runtime is missing")
def test_library_host_code_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liblbm_vans_asan.so")
        cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
               "-I" + os.path.join(ROOT, "include"),
               "-Xarch_device", "-O0", "-Xarch_host", "-O1", "-Xarch_host", "-g",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", lib, os.path.join(ROOT, "paper_1406_6438_amd", "csrc", "lbm_vans.hip")]
        subprocess.run(cmd, check=True, capture_output=True, timeout=900)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_child.py"), lib],
                           env=dict(ENV, LD_PRELOAD=_clang_asan()), capture_output=True,
                           text=True, timeout=300)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "sanitized host checks passed" in r.stdout


@pytest.mark.skipif(_gcc_lib("libasan.so") is None, reason="gcc's AddressSanitizer is missing")
def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liblbm_vans_oracle_asan.so")
        subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-o", lib, os.path.join(ROOT, "oracle", "lbm_vans_oracle.c"), "-lm"],
                       check=True, capture_output=True, timeout=300)
        env = dict(ENV, LD_PRELOAD=_gcc_lib("libasan.so"), LBM_VANS_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_adjoint.py"),
                            os.path.join(ROOT, "tests", "test_oracle_inout.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]

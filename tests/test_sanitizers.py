"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code, run on the
CPU: the FP64 oracle (gcc) under its pin suite, and the library's host side (the C
ABI's validation, planning and workspace layout; hipcc with the sanitizers on the
host pass only) under the host-only ABI tests.  No device code runs."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run([gcc, "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not available")
    lib = str(tmp_path / "liboq_san.so")
    _run([gcc, "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib,
          os.path.join(ROOT, "oracle", "qnep_oracle.c"), "-lm"], dict(os.environ), 300)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", QNEP_ORACLE_LIBRARY=lib, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "tests/test_oracle_pins.py"], env,
         900)


def test_host_abi_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    objs = [o for o in glob.glob(os.path.join(ROOT, "paper_2601_19034_amd", "_build", "*.o"))
            if not o.endswith("api.o")]
    if not os.path.exists(hipcc) or not rt or not objs:
        pytest.skip("hipcc, the clang sanitizer runtime or the library objects are not available")
    api_o = str(tmp_path / "api.o")
    lib = str(tmp_path / "libqnep_san.so")
    csrc = os.path.join(ROOT, "paper_2601_19034_amd", "csrc")
    arch = os.environ.get("QNEP_ARCH", "gfx950")
    _run([hipcc, f"--offload-arch={arch}", "-O1", "-g", "-fPIC", "-std=c++17", "-x", "hip",
          "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), "-I", csrc, "-c", os.path.join(csrc, "api.cpp"), "-o", api_o],
         dict(os.environ), 600)
    _run([hipcc, f"--offload-arch={arch}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address,undefined",
          "-Xarch_host", "-shared-libsan", "-o", lib, api_o] + objs, dict(os.environ), 300)
    env = dict(os.environ, LD_PRELOAD=rt[-1], QNEP_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "tests/test_abi_cpu.py"], env, 600)

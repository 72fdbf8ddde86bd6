"""Sanitizer builds on the CPU (no GPU, no device code runs): the library's
host-only helpers, the oracle and the library's host entry points are built
with the address and undefined-behaviour sanitizers, and their checks run
against those builds.  A finding aborts the run (no recovery), so a pass means
no invalid access, leak-free exit aside (leak checking is off: the HIP
runtime keeps allocations until exit)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_6862_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ASAN_OPTIONS = "detect_leaks=0:halt_on_error=1:abort_on_error=0"

needs_hipcc = pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _clang_asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def _gcc_asan_runtime():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()


def _run_pytest(files, env_extra, timeout=600):
    env = dict(os.environ, ASAN_OPTIONS=ASAN_OPTIONS, UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.update(env_extra)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                           *[os.path.join(ROOT, "tests", f) for f in files]],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


@needs_hipcc
def test_host_helpers_under_sanitizers(tmp_path):
    """Window bit helpers of the segmented kernels (mask_top over every
    window end), the server's ring allocator and coarse tile map."""
    exe = str(tmp_path / "host_units")
    subprocess.check_call([HIPCC, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "--offload-host-only",
                           "-Xarch_host", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", CSRC, "-I", INCLUDE, "-o", exe, os.path.join(ROOT, "tests", "host_units.cpp")],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], env=dict(os.environ, ASAN_OPTIONS=ASAN_OPTIONS), capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "host units ok" in out.stdout


@needs_gcc
def test_oracle_pins_under_sanitizers(tmp_path):
    """The oracle's pins and the input generator's tests against an
    address- and UB-sanitized build of the oracle."""
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", lib,
                           os.path.join(ROOT, "oracle", "hamming_oracle.c"),
                           os.path.join(ROOT, "oracle", "segmented_oracle.c")])
    out = _run_pytest(["test_oracle_pins.py", "test_oracle_seg_pins.py", "test_synth.py"],
                      {"LD_PRELOAD": _gcc_asan_runtime(), "ORACLE_LIB": lib})
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert " passed" in out.stdout and "ERROR: AddressSanitizer" not in out.stderr


@needs_hipcc
@pytest.mark.skipif(_clang_asan_runtime() is None, reason="needs the clang address-sanitizer runtime")
def test_library_host_code_under_sanitizers(tmp_path):
    """The library's host entry points (argument validation, layouts, grid
    sizing, segment layout) called from the CPU tests and from a C program,
    against a build whose host code is address- and UB-sanitized (device
    code is built as usual and never runs here)."""
    sys.path.insert(0, ROOT)
    from paper_1412_6862_amd import build as hip_build

    lib = str(tmp_path / "libhamming_asan.so")
    subprocess.check_call([HIPCC, *hip_build.FLAGS, "-O1", "-g", "-Xarch_host", "-fsanitize=address,undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all", "-I", INCLUDE, "-I", CSRC, "-o", lib,
                           *hip_build.sources(), "-lpthread"], stderr=subprocess.DEVNULL)
    out = _run_pytest(["test_abi_cpu.py", "test_seg_layout_cpu.py", "test_bench_cli.py"],
                      {"LD_PRELOAD": _clang_asan_runtime(), "HAMMING_LIB": lib})
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert " passed" in out.stdout and "ERROR: AddressSanitizer" not in out.stderr

"""The boundary as a C program sees it: tests/c_abi_consumer.c is compiled
with gcc against include/hamming.h, linked to libhamming.so and run.  Host-side
calls only, so this runs without a GPU."""
import os
import shutil
import subprocess

import pytest

import paper_1412_6862_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs gcc and the ROCm headers")
def test_c_program_compiles_links_and_runs(tmp_path):
    hm.library()     # raises if the library is not built
    exe = str(tmp_path / "abi_consumer")
    libdir = os.path.dirname(hm.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
                           os.path.join(ROOT, "tests", "c_abi_consumer.c"), "-o", exe,
                           "-L" + libdir, "-lhamming", "-Wl,-rpath," + libdir])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "c abi ok" in out.stdout

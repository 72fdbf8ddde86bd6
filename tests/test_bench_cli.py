"""Command-line contract of bench.py that needs no GPU: one GPU only (a
larger --gpus exits with a message and a non-zero status before touching a
device), and the metric and traffic bookkeeping helpers."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_algorithmic_bytes_per_codeword():
    # codeword read (8 or 16 bytes) + k/8 message bytes + one errpos byte
    assert bench.algorithmic_bytes_per_codeword(3) == 8 + 4 / 8 + 1
    assert bench.algorithmic_bytes_per_codeword(6) == 8 + 57 / 8 + 1
    assert bench.algorithmic_bytes_per_codeword(7) == 16 + 120 / 8 + 1


def test_recorded_traffic_follows_the_kernel_sources():
    # the committed counter summary is used only for the kernel it was taken
    # from: a different lane width reads as no record
    d = bench.kernel_source_digest()
    assert len(d) == 16
    assert bench.recorded_traffic("decode_plain_kernel<6,999>") is None

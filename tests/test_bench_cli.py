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


def _fake_full_result():
    """A result dict shaped like a full bench run (every leg, every shape)."""
    per_r = [{"r": r, "n_cw": 1 << 26, "avg_us": 160.0, "p50_us": 160.0, "p99_us": 170.0, "min_us": 150.0,
              "max_us": 180.0, "algorithmic_GBps": 6500.0, "frac_hbm": 0.8125, "payload_Gbps": 20000.0}
             for r in (4, 5, 6)]
    out = {
        "metric": bench.METRIC, "value": 15000.0, "unit": "Gbit/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 0.42, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain decode " + "x" * 200, "n_cw_per_packet": 1 << 26, "r": [4, 5, 6],
                   "p_single": 0.1},
        "roofline": {"kernel": "decode_plain_kernel<6,4>", "bound": "hbm", "achieved": 6500.0, "peak": 8000.0,
                     "unit": "GB/s", "frac": 0.8125, "traffic": 1.09e9, "algorithmic_bytes_per_launch": 1082130432,
                     "avg_launch_us": 166.5, "min_launch_us": 160.0, "max_launch_us": 180.0,
                     "runtime_d2d_copy_GBps": 5200.0},
        "per_r": per_r, "tuned_shapes": {"plain": {r: [4, 0, 1] for r in range(3, 8)}, "batch": [2, 1, 0, 1]},
        "latency_hamming74": {"workload": "w" * 100, "launches": 1000, "p50_us": 6.2, "p99_us": 10.0},
        "size_sweep": {"workload": "w", "rows": [{"r": r, "n_cw": 1 << lg, "us_p50": 1.0} for r in (4, 5, 6)
                                                 for lg in range(10, 29)]},
        "hamming127": {"workload": "w", "us_p50": 170.0, "payload_Gbps": 23000.0, "frac_hbm": 0.79},
        "error_rates": {"workload": "w", "rows": [{"r": 4}] * 18},
        "batched": {"workload": "w" * 300, "packets": 20000, "ms_p50": 6.0, "payload_Gbps": 19000.0,
                    "frac_hbm": 0.72, "batched_over_plain": 0.92, "naive_one_launch_per_packet_ms": 80.0},
        "serving": {"workload": "w" * 300, "plain_mix_Gbps": 19700.0,
                    "points": [{"offered_load": x, "requests": 100000, "p50_us": 123.4, "p99_us": 2345.6,
                                "offered_Gbps": 17000.0, "achieved_Gbps": 16900.0, "served_over_plain": 0.86}
                               for x in bench.SERVE_LOADS],
                    "saturated": {"requests": 110000, "elapsed_ms": 120.0, "achieved_Gbps": 18000.0,
                                  "served_over_plain": 0.91}},
        "host_pipeline": {"sync_ms": 20.0},
        "planes": {"rows": [{"r": r} for r in range(3, 8)]},
        "encode": {"rows": [{"r": r} for r in range(3, 8)]},
        "segmented": {"shapes": [{"M": m, "t": t, "batch_us": 100.0} for m in range(5) for t in range(5)]},
        "cpu_baseline": {"value": 2.5, "unit": "Gbit/s", "cores": 16, "kind": "oracle", "sample": "s" * 150,
                         "single_thread_Gbps_r6": 0.2, "cpu_model": "AMD EPYC 9575F 64-Core Processor",
                         "smt": "on", "cpus_allowed": 16, "host_cpus": 256,
                         "segmented_us_per_packet_1thread": {"%d/%d" % (m, t): 50.0 for m in range(5)
                                                             for t in range(5)},
                         "gpu_over_oracle": {"all_threads": 6000.0, "single_thread_r6": 100000.0}},
    }
    return out


def test_summary_line_is_short_and_carries_the_headline():
    import json

    s = bench.summary_line(_fake_full_result())
    line = json.dumps(s, separators=(",", ":"))
    assert len(line) < bench.SUMMARY_MAX_BYTES
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in s, k
    assert s["config"]["workload"].startswith("plain decode")
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in s["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample", "cpu_model", "smt", "single_thread_Gbps_r6"):
        assert k in s["cpu_baseline"], k
    assert "99x" in s["cpu_baseline"]["paper_speedup_context"]
    assert s["batched"]["batched_over_plain"] == 0.92
    assert s["serving"]["offered_load"] == 0.9 and s["serving"]["p99_us"] == 2345.6
    assert s["serving"]["capacity_over_plain"] == 0.91
    assert len(s["serving"]["points"]) == len(bench.SERVE_LOADS)
    # the per-leg bulk stays off the final line
    assert "segmented_us_per_packet_1thread" not in s["cpu_baseline"]
    assert "size_sweep" not in s and "per_r" not in s


def test_summary_line_without_extra_legs():
    out = _fake_full_result()
    for k in ("batched", "serving", "cpu_baseline", "latency_hamming74", "hamming127"):
        out.pop(k)
    s = bench.summary_line(out)
    assert "batched" not in s and "serving" not in s and s["value"] == 15000.0


def test_host_cpu_info_fields():
    info = bench.host_cpu_info()
    assert info["smt"] in ("on", "off", "unknown")
    assert isinstance(info["cpu_model"], str)

"""Throughput bench of the MI355X Hamming decoder.

One step = the plain decode of one packet of 2^26 codewords for each of
Hamming(15,11), (31,26) and (63,57) (r = 4, 5, 6), 10% single-bit error rate,
inputs resident in HBM.  Prints one JSON line: decoded payload Gbit/s over the
step, the HBM roofline of the dominant kernel (the r = 6 decode) measured with
HIP events on the launch stream, and the CPU oracle timed on the host cores on
a bounded slice of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded payload Gbit/s & %HBM roofline, batched vs plain; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
WORKLOAD_R = (4, 5, 6)
WORKLOAD_LOG2 = 26
P_SINGLE = 0.1
DOMINANT_R = 6
PROFILE_GLOB = os.path.join(ROOT, "profiles", "decode_plain_r6_2p26_traffic.md")
TUNED_SHAPES = os.path.join(ROOT, "paper_1412_6862_amd", "tuned_shapes.json")
SERVE_LOADS = (0.1, 0.3, 0.5, 0.7, 0.8, 0.9)
SERVE_REPORT_LOAD = 0.9
# the last stdout line is the record a reader keeps; it must stay short
SUMMARY_MAX_BYTES = 4096


def algorithmic_bytes_per_codeword(r: int) -> float:
    """Codeword read + dense message write + one errpos byte."""
    k = (1 << r) - 1 - r
    wpc = 2 if r == 7 else 1
    return 8.0 * wpc + k / 8.0 + 1.0


# sources the plain decode kernel and its launch configuration are built from
DOMINANT_SOURCES = ("abi.hip", "decode_plain.hip", "hamming_device.h", "launch.h", "tile.h")


def kernel_source_digest() -> str:
    """Digest of the plain decode kernel's sources and of the plain-decode
    launch shapes the bench loads (the batched lines of the tuning cache do
    not affect this kernel)."""
    h = hashlib.sha256()
    for f in DOMINANT_SOURCES:
        with open(os.path.join(ROOT, "paper_1412_6862_amd", "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    if os.path.exists(TUNED_SHAPES):
        with open(TUNED_SHAPES, "rb") as fh:
            for line in fh:
                if line.startswith(b'{"device"') or line.startswith(b'{"plain"'):
                    h.update(line)
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken from the current kernel sources and the
    same kernel instance (lane width) that this run launches."""
    if not os.path.exists(PROFILE_GLOB):
        return None
    fields = {}
    with open(PROFILE_GLOB) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel source digest") != kernel_source_digest():
        return None
    if fields.get("kernel", "").replace(" ", "").replace("hm::", "") != kernel:
        return None
    try:
        return float(fields["HBM bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


def make_packet(r: int, n_cw: int, p: float, dev):
    """Device-resident received words: random messages encoded on the GPU by
    the library's encoder, then flipped by the seeded channel masks."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm
    import synth

    seed = synth.workload_seed("bench", r, str(p))
    msg = torch.from_numpy(synth.message_stream(seed, n_cw, r).view(np.int64)).to(dev)
    cw = hm.encode(msg, n_cw, r)
    p1, p2 = synth.error_positions(seed, n_cw, r, p_single=p)
    cw ^= torch.from_numpy(synth.flip_masks(p1, p2, r).view(np.int64)).to(dev)
    torch.cuda.synchronize()
    del msg
    return cw


def build_batch(dev, n_packets: int, seed: int):
    """The batched workload: packet sizes log-uniform in [64, 2^20] codewords,
    r uniform in 3..7, per-packet single-error rate uniform in [0, 0.5].
    Messages and flips come from the seeded generator on the device; codewords
    from the library's encoder.  Returns (arena, descs, per-r plain packets)."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm
    import synth

    n_cw, r, p = synth.batch_packets(seed, n_packets)
    wpc = np.where(r == 7, 2, 1)
    words = n_cw * wpc
    in_off = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    descs = np.zeros(n_packets, dtype=hm.packet_dtype())
    descs["in_word_off"] = in_off
    descs["n_cw"] = n_cw
    descs["r"] = r
    hm.hamming_batch_layout(descs)
    arena = torch.empty(int(words.sum()), dtype=torch.int64, device=dev)
    per_r = {}
    for rr in range(3, 8):
        idx = np.flatnonzero(r == rr)
        total = int(n_cw[idx].sum())
        if total == 0:
            continue
        sr = synth.subseed(seed, "r", rr)
        msg = synth.message_stream_torch(sr, total, rr, dev)
        cw = hm.encode(msg, total, rr)
        del msg
        rates = torch.repeat_interleave(torch.from_numpy(p[idx]).to(dev),
                                        torch.from_numpy(n_cw[idx]).to(dev))
        cw ^= synth.flip_masks_torch(sr, total, rr, rates, dev)
        del rates
        w = 2 if rr == 7 else 1
        pos = 0
        for i in idx:
            nw = int(n_cw[i]) * w
            o = int(in_off[i])
            arena[o:o + nw].copy_(cw[pos:pos + nw])
            pos += nw
        per_r[rr] = (cw, total)
        torch.cuda.synchronize()
    return arena, descs, per_r, n_cw, r


def time_events(fn, stream, warmup: int, reps: int):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return sorted(a.elapsed_time(b) for a, b in evs)


def batched_leg(dev, n_packets: int, reps: int):
    """Batched decode of the whole workload in one hamming_decode_batch call,
    beside the plain decode of the same codewords (one call per r)."""
    import torch

    import paper_1412_6862_amd as hm
    import synth

    seed = synth.workload_seed("bench-batch", 0)
    arena, descs, per_r, n_cw, r = build_batch(dev, n_packets, seed)
    bd = hm.BatchDecoder(arena, n_packets)
    bd.set_packets(descs)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        tb = time_events(lambda: bd.decode(stream=stream), stream, 2, reps)
    st = bd.status[:n_packets].cpu()
    if bool((st != 0).any()):
        raise RuntimeError("batched bench: a descriptor was rejected")
    plain_ms = 0.0
    data = torch.empty(max(hm.hamming_data_bytes(t, rr) for rr, (_, t) in per_r.items()), dtype=torch.uint8,
                       device=dev)
    ep = torch.empty(max(t for _, t in per_r.values()), dtype=torch.uint8, device=dev)
    with torch.cuda.stream(stream):
        for rr, (cw, total) in per_r.items():
            tp = time_events(lambda: hm.hamming_decode(cw, total, rr, data, ep, stream), stream, 2, reps)
            plain_ms += tp[len(tp) // 2]
    # the naive alternative: one plain launch per packet, same arenas
    lib = hm.library()
    base_in, base_out, base_ep = arena.data_ptr(), bd.data.data_ptr(), bd.errpos.data_ptr()
    calls = [(base_in + 8 * int(d["in_word_off"]), int(d["n_cw"]), int(d["r"]), base_out + 8 * int(d["data_word_off"]),
              base_ep + int(d["errpos_off"])) for d in descs]
    sh = stream.cuda_stream
    with torch.cuda.stream(stream):
        def naive():
            for c in calls:
                lib.hamming_decode(c[0], c[1], c[2], c[3], c[4], sh)
        t_naive = time_events(naive, stream, 1, 2)
    k = (1 << r) - 1 - r
    bits = float((n_cw * k).sum())
    algo = float(sum(n_cw[r == rr].sum() * algorithmic_bytes_per_codeword(rr) for rr in range(3, 8)))
    med = tb[len(tb) // 2]
    del arena, per_r, bd, data, ep
    torch.cuda.empty_cache()
    return {
        "workload": "%d packets, sizes log-uniform in [64, 2^20] codewords, r uniform in 3..7, per-packet "
                    "single-error rate uniform in [0, 0.5]; one hamming_decode_batch call" % n_packets,
        "packets": n_packets, "codewords": int(n_cw.sum()),
        "algorithmic_bytes": int(algo),
        "ms_p50": round(med, 3), "ms_min": round(tb[0], 3),
        "payload_Gbps": round(bits / med / 1e6, 1),
        "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4),
        "plain_same_mix_ms": round(plain_ms, 3),
        "batched_over_plain": round(plain_ms / med, 4),
        "naive_one_launch_per_packet_ms": round(t_naive[0], 2),
        "schedule": list(hm.hamming_batch_config_get()),
    }


def serving_leg(dev, plain_gBps_per_r: dict, loads, n_requests: int, warm: int, batch_log2: int = 25):
    """Open-loop serving: Poisson arrivals from 256 simulated SDR streams
    (stream s decodes code r = 4 + s % 4), request sizes log-uniform in
    [256, 2^18] codewords, 10% single-bit errors, offered load swept as a
    fraction of the plain decoder's throughput on the same r-mix."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm
    import synth

    rs = (4, 5, 6, 7)
    pool_cw = {4: 1 << 25, 5: 1 << 25, 6: 1 << 25, 7: 1 << 24}
    parts, base = [], {}
    off = 0
    for rr in rs:
        n = pool_cw[rr]
        sr = synth.workload_seed("bench-serve", rr)
        cw = hm.encode(synth.message_stream_torch(sr, n, rr, dev), n, rr)
        cw ^= synth.flip_masks_torch(sr, n, rr, 0.1, dev)
        base[rr] = off
        off += cw.numel()
        parts.append(cw)
    pool = torch.cat(parts)
    del parts
    torch.cuda.synchronize()
    total = n_requests + warm
    rng = np.random.default_rng(synth.workload_seed("bench-serve-trace", 0) & 0xFFFFFFFF)
    stream_id = rng.integers(0, 256, size=total)
    r = (4 + stream_id % 4).astype(np.uint32)
    sizes = np.floor(256 * np.exp2(10 * rng.random(total))).astype(np.uint64)
    wpc = np.where(r == 7, 2, 1).astype(np.uint64)
    offs = np.empty(total, dtype=np.uint64)
    for rr in rs:
        m = r == rr
        span = pool_cw[rr] - sizes[m]
        offs[m] = np.uint64(base[rr]) + (np.floor(rng.random(m.sum()) * span).astype(np.uint64)) * wpc[m]
    k = (1 << r.astype(np.int64)) - 1 - r.astype(np.int64)
    bits = sizes.astype(np.float64) * k
    # plain-decode time of each request from the plain kernels' algorithmic
    # bandwidth on its r; the offered load is rho over the mean of these
    nbytes = np.array([float(n) * algorithmic_bytes_per_codeword(int(x)) for n, x in zip(sizes, r)])
    t_plain = nbytes / np.array([plain_gBps_per_r[int(x)] for x in r]) / 1e9
    # the plain decoder's rate on this mix: every request decoded by a plain call at its r's measured bandwidth
    plain_mix_Gbps = float(bits.sum()) / float(t_plain.sum()) / 1e9
    # at most 2^25 codewords per batch (the default): over caps 2^24, 2^25 and 2^26, each run twice
    # alone and twice after the batched leg, 2^25 had the lowest or equal p50 at 70-80% load and
    # kept 15-16 Tbit/s at 90%; 2^24 fell to 13.7 Tbit/s after the batched leg, 2^26 doubled p50 at 80%
    srv = hm.Server(pool, slots=4, max_batch_packets=4096, max_batch_codewords=1 << batch_log2,
                    output_pool_bytes=32 << 30, auto_release=True)
    out = []
    try:
        for rho in loads:
            gaps = rng.exponential(t_plain.mean() / rho, size=total)
            arrivals = (np.cumsum(gaps) * 1e9).astype(np.uint64)
            lat, elapsed = srv.run_trace(arrivals, offs, sizes, r, timeout_s=120)
            done = arrivals.astype(np.float64) + lat.astype(np.float64)
            # measured window: from the first measured arrival to the last completion
            window_s = (done[warm:].max() - float(arrivals[warm])) / 1e9
            span_s = (float(arrivals[-1]) - float(arrivals[warm])) / 1e9
            lat_us = np.sort(lat[warm:]) / 1e3
            out.append({
                "offered_load": rho,
                "requests": n_requests,
                "p50_us": round(float(lat_us[len(lat_us) // 2]), 1),
                "p99_us": round(float(lat_us[int(0.99 * (len(lat_us) - 1))]), 1),
                "offered_Gbps": round(float(bits[warm:].sum()) / span_s / 1e9, 1),
                "achieved_Gbps": round(float(bits[warm:].sum()) / window_s / 1e9, 1),
                "served_over_plain": round(float(bits[warm:].sum()) / window_s / 1e9 / plain_mix_Gbps, 4),
            })
        # saturation: every request queued at time 0, drained as fast as the server can
        lat, elapsed = srv.run_trace(np.zeros(total, dtype=np.uint64), offs, sizes, r, timeout_s=120)
        sat_Gbps = float(bits.sum()) / (elapsed / 1e9) / 1e9
        saturated = {"requests": total, "elapsed_ms": round(elapsed / 1e6, 2), "achieved_Gbps": round(sat_Gbps, 1),
                     "served_over_plain": round(sat_Gbps / plain_mix_Gbps, 4)}
    finally:
        srv.close()
        del pool
        torch.cuda.empty_cache()
    return {"workload": "256 SDR streams, r = 4 + stream % 4, request sizes log-uniform in [256, 2^18] "
                        "codewords, 10% single-bit errors, Poisson arrivals; 4 batches in flight of at most 2^"
                        + str(batch_log2) + " codewords; output pool (device-memory admission cap) 32 GiB",
            "plain_mix_Gbps": round(plain_mix_Gbps, 1), "points": out, "saturated": saturated}


def latency_leg(dev, reps: int):
    """Hamming(7,4), one packet of 65,536 codewords (p = 0.5): a latency-bound
    launch; p50/p99 of single-launch time over `reps` launches, beside the
    same measurement of a one-element torch kernel (the launch floor)."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm

    r, n = 3, 65536
    cw = make_packet(r, n, 0.5, dev)
    data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, device=dev)
    ep = torch.empty(n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    t = np.array(time_events(lambda: hm.hamming_decode(cw, n, r, data, ep, stream), stream, 20, reps)) * 1e3
    one = torch.zeros(1, dtype=torch.int32, device=dev)
    f = np.array(time_events(lambda: one.add_(1), stream, 20, reps)) * 1e3
    return {"workload": "Hamming(7,4), one packet of 65,536 codewords, 50% single-bit errors",
            "launches": reps, "p50_us": round(float(np.percentile(t, 50)), 2),
            "p99_us": round(float(np.percentile(t, 99)), 2),
            "payload_Gbps_at_p50": round(n * 4 / float(np.percentile(t, 50)) / 1e3, 1),
            "launch_floor_p50_us": round(float(np.percentile(f, 50)), 2)}


def hamming127_leg(dev, reps: int):
    """Hamming(127,120), 2^25 codewords, 70% clean / 25% one flip / 5% two
    flips (the two-flip words are miscorrected by the deterministic rule)."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm
    import synth

    r, n = 7, 1 << 25
    seed = synth.workload_seed("bench-r7", r)
    cw = hm.encode(synth.message_stream_torch(seed, n, r, dev), n, r)
    p1, p2 = synth.error_positions(seed, n, r, p_single=0.25, p_double=0.05)
    cw ^= torch.from_numpy(synth.flip_masks(p1, p2, r).view(np.int64)).to(dev)
    data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, device=dev)
    ep = torch.empty(n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    t = time_events(lambda: hm.hamming_decode(cw, n, r, data, ep, stream), stream, 5, reps)
    med = t[len(t) // 2]
    algo = algorithmic_bytes_per_codeword(r) * n
    return {"workload": "Hamming(127,120), 2^25 codewords, 70% clean / 25% one flip / 5% two flips",
            "us_p50": round(med * 1e3, 2), "payload_Gbps": round(n * 120 / med / 1e6, 1),
            "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4)}


def errors_leg(dev, reps: int):
    """Plain decode of 2^26 codewords of r = 4, 5, 6 at single-bit error
    rates 0, 0.01, 0.1, 0.5 and 1: the correction is branch-free, so the time
    must not depend on the rate.  One encoded packet per r; each rate applies
    its own seeded flips to a copy."""
    import torch

    import paper_1412_6862_amd as hm
    import synth

    stream = torch.cuda.current_stream()
    n, rates, rows = 1 << 26, (0.0, 0.01, 0.1, 0.5, 1.0), []
    for r in WORKLOAD_R:
        seed = synth.workload_seed("bench-errors", r)
        clean = hm.encode(synth.message_stream_torch(seed, n, r, dev), n, r)
        data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, device=dev)
        ep = torch.empty(n, dtype=torch.uint8, device=dev)
        algo = algorithmic_bytes_per_codeword(r) * n
        times = []
        for p in rates:
            cw = clean ^ synth.flip_masks_torch(synth.workload_seed("bench-errors", r, str(p)), n, r, p, dev)
            t = time_events(lambda: hm.hamming_decode(cw, n, r, data, ep, stream), stream, 3, reps)
            med = t[len(t) // 2]
            times.append(med)
            rows.append({"r": r, "p_single": p, "us_p50": round(med * 1e3, 2),
                         "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4)})
            del cw
        rows.append({"r": r, "max_over_min": round(max(times) / min(times), 4)})
        del clean, data, ep
        torch.cuda.empty_cache()
    return {"workload": "plain decode, 2^26 codewords of r = 4, 5, 6 at single-bit error rates 0, 0.01, 0.1, "
                        "0.5 and 1", "rows": rows}


def host_leg(dev, reps: int):
    """Host-resident Hamming(63,57) packet of 2^26 codewords in pinned memory,
    decoded through the copy pipeline: synchronous transfers (copy in,
    decode, copy out, chunk after chunk) against the asynchronous schedule
    over 3 streams, with the speedup Eq. 1 predicts from the measured
    synchronous stage times.  PCIe-inclusive; never the reported value."""
    import time

    import numpy as np
    import torch

    import paper_1412_6862_amd as hm

    r, n, chunk, streams = 6, 1 << 26, 1 << 22, 3
    k = hm.hamming_message_bits(r)
    cw = make_packet(r, n, P_SINGLE, dev).cpu().pin_memory()
    data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, pin_memory=True)
    ep = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    wsb = hm.hamming_host_workspace_bytes(chunk, r, streams)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    n_chunks = n // chunk

    def run(mode, times=False):
        t0 = time.perf_counter()
        if mode == hm.HAMMING_TRANSFER_MAPPED:
            st = hm.hamming_decode_host(cw, n, r, data, ep, chunk, mode, streams, None, 0, times=times)
        else:
            st = hm.hamming_decode_host(cw, n, r, data, ep, chunk, mode, streams, ws, wsb, times=times)
        return time.perf_counter() - t0, st

    run(hm.HAMMING_TRANSFER_SYNC)
    run(hm.HAMMING_TRANSFER_ASYNC)
    run(hm.HAMMING_TRANSFER_MAPPED)
    sync = [run(hm.HAMMING_TRANSFER_SYNC, True) for _ in range(reps)]
    asyn = [run(hm.HAMMING_TRANSFER_ASYNC)[0] for _ in range(reps)]
    mapd = [run(hm.HAMMING_TRANSFER_MAPPED)[0] for _ in range(reps)]
    t_sync = float(np.median([s[0] for s in sync]))
    t_async = float(np.median(asyn))
    t_mapped = float(np.median(mapd))
    ps, dke, pr = (float(np.median([s[1][i] for s in sync])) / n_chunks for i in range(3))
    eq1 = n_chunks * (ps + dke + pr) / (ps + n_chunks * dke + pr)
    stage = max(ps, dke, pr)
    pipe = n_chunks * (ps + dke + pr) / (ps + dke + pr + (n_chunks - 1) * stage)
    return {"workload": "Hamming(63,57), 2^26 codewords (512 MiB) in pinned host memory, %d chunks of 2^22 "
                        "codewords, %d streams, 10%% single-bit errors" % (n_chunks, streams),
            "sync_ms": round(t_sync * 1e3, 2), "async_ms": round(t_async * 1e3, 2),
            "async_speedup": round(t_sync / t_async, 3),
            "mapped_ms": round(t_mapped * 1e3, 2), "mapped_speedup": round(t_sync / t_mapped, 3),
            "mapped_link_GBps": round((n * 8 + n * (k + 8) / 8) / t_mapped / 1e9, 1),
            "chunk_ms": {"h2d": round(ps, 3), "decode": round(dke, 4), "d2h": round(pr, 3)},
            "h2d_GBps": round(chunk * 8 / ps / 1e6, 1),
            "d2h_GBps": round((chunk * (k + 8) / 8) / pr / 1e6, 1),
            "eq1_predicted_speedup": round(eq1, 3), "stage_bound_speedup": round(pipe, 3),
            "payload_Gbps_async": round(n * k / t_async / 1e9, 1),
            "payload_Gbps_mapped": round(n * k / t_mapped / 1e9, 1)}


def sizes_leg(dev):
    """Plain decode over the packet-size sweep 2^10..2^28 codewords of
    Hamming(15,11), (31,26), (63,57): each size decodes a prefix of one
    device-generated 2^28-codeword packet (10% single-bit errors)."""
    import torch

    import paper_1412_6862_amd as hm
    import synth

    stream = torch.cuda.current_stream()
    rows = []
    for r in WORKLOAD_R:
        nmax = 1 << 28
        seed = synth.workload_seed("bench-sizes", r)
        cw = hm.encode(synth.message_stream_torch(seed, nmax, r, dev), nmax, r)
        cw ^= synth.flip_masks_torch(seed, nmax, r, P_SINGLE, dev)
        data = torch.empty(hm.hamming_data_bytes(nmax, r), dtype=torch.uint8, device=dev)
        ep = torch.empty(nmax, dtype=torch.uint8, device=dev)
        k = hm.hamming_message_bits(r)
        for lg in range(10, 29):
            n = 1 << lg
            reps = 200 if lg <= 20 else 20
            t = time_events(lambda: hm.hamming_decode(cw, n, r, data, ep, stream), stream, 3, reps)
            med = t[len(t) // 2]
            algo = algorithmic_bytes_per_codeword(r) * n
            rows.append({"r": r, "n_cw": n, "us_p50": round(med * 1e3, 2),
                         "payload_Gbps": round(n * k / med / 1e6, 1),
                         "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4),
                         "cache_resident": algo < 256e6})
        del cw, data, ep
        torch.cuda.empty_cache()
    return {"workload": "plain decode, packet sizes 2^10..2^28 codewords (every power of two) of r = 4, 5, 6, "
                        "10% single-bit errors", "rows": rows}


def encode_leg(dev, reps: int):
    """The transmitter half: the plain encode of 2^26 messages per r = 3..6
    (2^25 for r = 7) from a device-resident dense message stream, as one
    launch each; algorithmic bytes = message read (k/8 per codeword) +
    codeword write (8 or 16 bytes)."""
    import torch

    import paper_1412_6862_amd as hm
    import synth

    stream = torch.cuda.current_stream()
    rows = []
    for r in (3, 4, 5, 6, 7):
        n = 1 << (25 if r == 7 else 26)
        k = hm.hamming_message_bits(r)
        msg = synth.message_stream_torch(synth.workload_seed("bench-encode", r), n, r, dev)
        out = torch.empty(n * hm.words_per_codeword(r), dtype=torch.int64, device=dev)
        t = time_events(lambda: hm.hamming_encode(msg, n, r, out, stream), stream, 3, reps)
        med = t[len(t) // 2]
        algo = n * (k / 8.0 + 8.0 * hm.words_per_codeword(r))
        rows.append({"r": r, "n_cw": n, "us_p50": round(med * 1e3, 2),
                     "GBps": round(algo / med / 1e6, 1), "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4)})
        del msg, out
    torch.cuda.empty_cache()
    return {"workload": "plain encode, 2^26 codewords per r = 3..6 and 2^25 for r = 7, messages resident in HBM",
            "rows": rows}


def planes_leg(dev, reps: int):
    """Bit-plane input layout against the natural layout on the same received
    words: 2^26 codewords (2^25 for r = 7), 10% single-bit errors."""
    import torch

    import paper_1412_6862_amd as hm

    stream = torch.cuda.current_stream()
    rows = []
    for r in (3, 4, 5, 6, 7):
        n = 1 << (25 if r == 7 else 26)
        k = hm.hamming_message_bits(r)
        cw = make_packet(r, n, P_SINGLE, dev)
        planes, pw = hm.to_planes(cw, r)
        data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, device=dev)
        ep = torch.empty(n, dtype=torch.uint8, device=dev)
        t_nat = time_events(lambda: hm.hamming_decode(cw, n, r, data, ep, stream), stream, 3, reps)
        t_pl = time_events(lambda: hm.hamming_decode_planes(planes, pw, n, r, data, ep, stream), stream, 3, reps)
        nat, pl = t_nat[len(t_nat) // 2], t_pl[len(t_pl) // 2]
        algo = n * (((1 << r) - 1) / 8.0 + k / 8.0 + 1.0)
        rows.append({"r": r, "n_cw": n, "natural_us": round(nat * 1e3, 1), "planes_us": round(pl * 1e3, 1),
                     "speedup": round(nat / pl, 3), "planes_Gcw_per_s": round(n / pl / 1e6, 1),
                     "planes_bytes_per_cw": round(algo / n, 3), "planes_GBps": round(algo / pl / 1e6, 1),
                     "planes_frac_hbm": round(algo / pl / 1e6 / HBM_PEAK_GBPS, 4)})
        del cw, planes, data, ep
        torch.cuda.empty_cache()
    return {"workload": "same received words in the natural layout and in the bit-plane layout; "
                        "2^26 codewords (2^25 for r = 7), 10% single-bit errors", "rows": rows}


SEG_SHAPES = [(m, t) for m in (400, 800, 1200, 1600, 2000) for t in (2, 3, 4, 5, 6)]
SEG_P_SINGLE, SEG_P_DOUBLE = 0.3, 0.05


def segmented_algorithmic_bytes(msg_bytes: int, t: int) -> float:
    """Encoded packet read + descriptor read + message write + syndromes + status."""
    import paper_1412_6862_amd as hm

    _, _, bits = hm.hamming_seg_layout(msg_bytes, t)
    return bits / 8.0 + 32 + msg_bytes + 2 * t + 1


def segmented_encode_bytes(msg_bytes: int, t: int) -> float:
    """Descriptor read + message read + encoded packet write."""
    import paper_1412_6862_amd as hm

    _, _, bits = hm.hamming_seg_layout(msg_bytes, t)
    return 32 + msg_bytes + bits / 8.0


def segmented_leg(dev, n_packets: int, reps: int, lat_reps: int, shapes=None):
    """The paper's packets (Sec. II, Table 1 grid): M bytes in t shortened
    segments.  Per shape: a batch of n_packets packets encoded on the GPU in
    one launch (the transmitter half, timed too), flips from the seeded
    channel, the batch decoded in one launch, and the latency of a one-packet
    decode launch."""
    import numpy as np
    import torch

    import paper_1412_6862_amd as hm
    import synth

    stream = torch.cuda.current_stream()
    rows = []
    for mb, t in (shapes or SEG_SHAPES):
        b = hm.SegmentedBatch(n_packets, mb, t, device=dev)
        seed = synth.workload_seed("bench-seg", mb, t)
        b.msg.copy_(synth.draws_torch(seed, 0, n_packets * b.msg_stride, dev))
        t_enc = time_events(lambda: b.encode(stream), stream, 10, reps)
        enc_med = t_enc[len(t_enc) // 2]
        k, r, _ = hm.hamming_seg_layout(mb, t)
        n = np.asarray(k) + np.asarray(r)
        starts = np.concatenate([[0], np.cumsum(n)[:-1]])
        b1, b2 = synth.segment_flips(seed, n_packets, starts, n, SEG_P_SINGLE, SEG_P_DOUBLE)
        base = (np.arange(n_packets, dtype=np.int64) * b.enc_stride * 64)[:, None]
        bits = torch.from_numpy(np.concatenate([(b1 + base)[b1 >= 0], (b2 + base)[b2 >= 0]])).to(dev)
        one = torch.ones_like(bits)
        b.enc ^= torch.zeros_like(b.enc).scatter_add_(0, bits // 64, torch.bitwise_left_shift(one, bits % 64))
        del bits, one
        t_batch = time_events(lambda: b.decode(stream), stream, 10, reps)
        med = t_batch[len(t_batch) // 2]
        algo = segmented_algorithmic_bytes(mb, t) * n_packets
        lat = np.array(time_events(lambda: hm.hamming_decode_segmented(
            b.enc, b.enc.numel(), b.descs, 1, mb, b.msg, b.msg.numel(), b.syndromes, b.syndromes.numel(),
            b.status, stream), stream, 20, lat_reps)) * 1e3
        st = torch.bincount(b.status.to(torch.int64), minlength=3)[:3].cpu().tolist()
        rows.append({"M": mb, "t": t, "batch_us": round(med * 1e3, 1),
                     "packets_per_s": round(n_packets / med * 1e3, 0),
                     "us_per_packet_batched": round(med * 1e3 / n_packets, 5),
                     "GBps": round(algo / med / 1e6, 1), "frac_hbm": round(algo / med / 1e6 / HBM_PEAK_GBPS, 4),
                     "encode_us": round(enc_med * 1e3, 1),
                     "encode_frac_hbm": round(segmented_encode_bytes(mb, t) * n_packets / enc_med / 1e6 / HBM_PEAK_GBPS, 4),
                     "single_packet_p50_us": round(float(np.percentile(lat, 50)), 2),
                     "single_packet_p99_us": round(float(np.percentile(lat, 99)), 2),
                     "status_clean_corrected_uncorrectable": st})
        del b
        torch.cuda.empty_cache()
    return {"workload": "the paper's packets: M in {400..2000} bytes split into t in {2..6} shortened Hamming "
                        "segments; %d packets per batch, per segment %.0f%% one flip / %.0f%% two flips"
                        % (n_packets, SEG_P_SINGLE * 100, SEG_P_DOUBLE * 100), "shapes": rows}


def cpu_segmented(n_packets: int):
    """The oracle, one thread, per packet of each segmented shape."""
    import numpy as np

    import oracle
    import synth

    out = {}
    for mb, t in SEG_SHAPES:
        seed = synth.workload_seed("bench-seg-cpu", mb, t)
        msgs = synth.packet_bytes(seed, n_packets, mb)
        enc = oracle.seg_encode_many(msgs, t)
        _, _, n, _ = oracle.seg_layout(mb, t)
        starts = np.concatenate([[0], np.cumsum(n)[:-1]])
        b1, b2 = synth.segment_flips(seed, n_packets, starts, n, SEG_P_SINGLE, SEG_P_DOUBLE)
        synth.apply_bit_flips(enc, b1, b2)
        t0 = time.perf_counter()
        oracle.seg_decode_many(enc, mb, t, nthreads=1)
        out["%d/%d" % (mb, t)] = round((time.perf_counter() - t0) / n_packets * 1e6, 2)
    return out


def copy_ceiling(dev) -> float:
    """Device-to-device copy of 1 GiB through the runtime (read + write bytes
    per second), the reference point for a kernel that reads and writes HBM
    once each."""
    import torch

    src = torch.ones(1 << 27, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    t = time_events(lambda: dst.copy_(src), stream, 3, 10)
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * (1 << 30) / t[len(t) // 2] / 1e6, 1)


_CPUID_KEYS = {"cpu family": "cpu_family", "model": "cpu_model_number", "stepping": "cpu_stepping"}


def host_cpu_info() -> dict:
    """CPU model, SMT state and the CPUs this process may run on."""
    info = {"cpu_model": "unknown", "smt": "unknown", "cpus_allowed": None, "host_cpus": os.cpu_count()}
    try:
        siblings = cores = None
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "model name" and info["cpu_model"] == "unknown":
                    info["cpu_model"] = val.strip()
                elif key in _CPUID_KEYS and _CPUID_KEYS[key] not in info:
                    # the numeric identity, for hosts whose model name is generic
                    info[_CPUID_KEYS[key]] = int(val)
                elif key == "siblings" and siblings is None:
                    siblings = int(val)
                elif key == "cpu cores" and cores is None:
                    cores = int(val)
        if siblings and cores:
            info["threads_per_core"] = siblings // cores
    except (OSError, ValueError):
        pass
    try:
        with open("/sys/devices/system/cpu/smt/active") as fh:
            info["smt"] = "on" if fh.read().strip() == "1" else "off"
    except OSError:
        if info.get("threads_per_core"):
            info["smt"] = "on" if info["threads_per_core"] > 1 else "off"
    try:
        info["cpus_allowed"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(log2_sample: int):
    """The oracle on the host cores over a slice of the same workload."""
    import oracle
    import synth

    n = 1 << log2_sample
    threads = oracle.default_threads()
    bits = 0
    elapsed = 0.0
    single = None
    for r in WORKLOAD_R:
        seed = synth.workload_seed("bench", r, str(P_SINGLE))
        stream = synth.message_stream(seed, n, r)
        cw = oracle.encode(stream, n, r, nthreads=threads)
        p1, p2 = synth.error_positions(seed, n, r, p_single=P_SINGLE)
        y = cw ^ synth.flip_masks(p1, p2, r)
        t0 = time.perf_counter()
        oracle.decode(y, r, nthreads=threads)
        elapsed += time.perf_counter() - t0
        bits += n * ((1 << r) - 1 - r)
        if r == WORKLOAD_R[-1]:
            # one thread on a 2^22 slice of the same packet: the analogue of a sequential decoder
            m = min(n, 1 << 22)
            t0 = time.perf_counter()
            oracle.decode(y[:m], r, nthreads=1)
            single = m * ((1 << r) - 1 - r) / (time.perf_counter() - t0) / 1e9
    out = {
        "value": round(bits / elapsed / 1e9, 3),
        "unit": "Gbit/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "2^%d codewords of each of r=4,5,6 (p=%.2f), %d threads, decode only, %.2f s (%.1f thread-s); "
                  "one thread on a 2^22-codeword slice of r=6" % (log2_sample, P_SINGLE, threads, elapsed,
                                                                   elapsed * threads),
        "single_thread_Gbps_r6": round(single, 3),
    }
    out.update(host_cpu_info())
    out["segmented_us_per_packet_1thread"] = cpu_segmented(100)
    return out


PAPER_SPEEDUP_CONTEXT = ("99x: GTX 560 over one core of a 4-core 3.4 GHz Intel (Sec. IV, abstract); other "
                         "hardware and a latency-bound packet size, context only")


def _pick(d: dict, *keys):
    return {k: d[k] for k in keys if k in d}


def summary_line(out: dict) -> dict:
    """The compact final line: the headline keys, the dominant kernel's
    roofline, the CPU baseline and one figure per extra leg.  The per-leg
    detail travels on the earlier lines (and in the --detail file)."""
    s = _pick(out, "metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config")
    s["roofline"] = _pick(out["roofline"], "kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                          "algorithmic_bytes_per_launch", "avg_launch_us", "min_launch_us", "max_launch_us")
    s["plain_frac_hbm"] = {str(x["r"]): x["frac_hbm"] for x in out.get("per_r", [])}
    if "batched" in out:
        b = out["batched"]
        s["batched"] = _pick(b, "ms_p50", "payload_Gbps", "frac_hbm", "batched_over_plain")
    if "serving" in out:
        pts = out["serving"]["points"]
        at = [p for p in pts if p["offered_load"] == SERVE_REPORT_LOAD]
        s["serving"] = {"offered_load": SERVE_REPORT_LOAD}
        if at:
            s["serving"].update(_pick(at[0], "p50_us", "p99_us", "achieved_Gbps", "served_over_plain"))
        sat = out["serving"].get("saturated")
        if sat:
            s["serving"]["capacity_over_plain"] = sat["served_over_plain"]
        s["serving"]["points"] = [[p["offered_load"], p["p50_us"], p["p99_us"], p["achieved_Gbps"]] for p in pts]
    if "hamming127" in out:
        s["hamming127"] = _pick(out["hamming127"], "us_p50", "frac_hbm")
    if "latency_hamming74" in out:
        s["hamming74_launch"] = _pick(out["latency_hamming74"], "p50_us", "p99_us")
    if "cpu_baseline" in out:
        cb = out["cpu_baseline"]
        s["cpu_baseline"] = _pick(cb, "value", "unit", "cores", "kind", "sample", "cpu_model", "cpu_family",
                                  "cpu_model_number", "smt", "cpus_allowed", "single_thread_Gbps_r6",
                                  "gpu_over_oracle")
        s["cpu_baseline"]["paper_speedup_context"] = PAPER_SPEEDUP_CONTEXT
    s["legs"] = sorted(k for k in out if k not in s and k not in ("per_r", "tuned_shapes"))
    # over the limit (never expected): shed the least important fields first
    for path in (("serving", "points"), ("cpu_baseline", "sample"), ("config", "workload"), ("legs",)):
        if len(json.dumps(s, separators=(",", ":"))) <= SUMMARY_MAX_BYTES:
            break
        d = s
        for p in path[:-1]:
            d = d.get(p, {})
        d.pop(path[-1], None)
    return s


def emit(obj: dict) -> None:
    print(json.dumps(obj, separators=(",", ":")), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--log2-cw", type=int, default=WORKLOAD_LOG2)
    # 2^25 codewords of each of the three r: about 20 thread-seconds of oracle work on 16 host threads
    ap.add_argument("--cpu-log2", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--batch-packets", type=int, default=20000)
    ap.add_argument("--serve-requests", type=int, default=100000)
    ap.add_argument("--serve-batch-log2", type=int, default=25, choices=range(16, 31), metavar="L",
                    help="serving leg: at most 2^L codewords per batch")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner before timing instead of loading the committed shapes")
    ap.add_argument("--tune-out", default="", metavar="PATH",
                    help="with --tune: also write the tuned shapes to PATH (the format of tuned_shapes.json)")
    ap.add_argument("--seg-packets", type=int, default=1 << 19)
    ap.add_argument("--seg-shapes", default="",
                    help="segmented leg: comma-separated M/t shapes (e.g. 1200/4); default the Table 1 grid")
    ap.add_argument("--legs", default="latency,sizes,r7,errors,batch,serve,host,seg,planes,encode",
                    help="extra legs after the plain one (which gives the reported value): "
                         "comma-separated subset of latency,sizes,r7,errors,batch,serve,host,seg,planes,encode, or none")
    ap.add_argument("--detail", default="", metavar="PATH", help="also write every leg's full result to PATH (JSON)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this decoder runs on one GPU; --gpus must be 1 (codewords are "
              "independent, so more GPUs would each decode their own share)", file=sys.stderr)
        return 2

    import torch

    import paper_1412_6862_amd as hm

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 8, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 5}), flush=True)
        return 0
    hm.library()
    legs = set(args.legs.split(","))
    if args.tune:
        hm.hamming_tune(args.tune_out or None, 3)
    elif os.path.exists(TUNED_SHAPES):
        try:
            hm.hamming_tune_load(TUNED_SHAPES)
        except hm.HammingError:
            pass    # shapes tuned on another device model: keep the built-in ones
    tuned = {"plain": {r: list(hm.hamming_plain_config_get(r)) for r in range(3, 8)},
             "batch": list(hm.hamming_batch_config_get())}
    n_cw = 1 << args.log2_cw
    packets = {}
    for r in WORKLOAD_R:
        cw = make_packet(r, n_cw, P_SINGLE, dev)
        data = torch.empty(hm.hamming_data_bytes(n_cw, r), dtype=torch.uint8, device=dev)
        ep = torch.empty(n_cw, dtype=torch.uint8, device=dev)
        packets[r] = (cw, data, ep)
    stream = torch.cuda.current_stream()

    def step(events=None):
        for r in WORKLOAD_R:
            cw, data, ep = packets[r]
            if events is not None:
                events[r][0].record(stream)
            hm.hamming_decode(cw, n_cw, r, data, ep, stream)
            if events is not None:
                events[r][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [{r: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for r in WORKLOAD_R} for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t_start.record(stream)
    for i in range(args.steps):
        step(evs[i])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = t_start.elapsed_time(t_end)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps

    per_r = []
    for r in WORKLOAD_R:
        times = sorted(e[r][0].elapsed_time(e[r][1]) for e in evs)
        avg = sum(times) / len(times)
        algo = algorithmic_bytes_per_codeword(r) * n_cw
        k = (1 << r) - 1 - r
        per_r.append({
            "r": r, "n_cw": n_cw, "avg_us": round(avg * 1e3, 2),
            "p50_us": round(times[len(times) // 2] * 1e3, 2),
            "p99_us": round(times[min(len(times) - 1, int(0.99 * len(times)))] * 1e3, 2),
            "min_us": round(times[0] * 1e3, 2), "max_us": round(times[-1] * 1e3, 2),
            "algorithmic_GBps": round(algo / avg / 1e6, 1),
            "frac_hbm": round(algo / avg / 1e6 / HBM_PEAK_GBPS, 4),
            "payload_Gbps": round(n_cw * k / avg / 1e6, 1),
        })
    dom = next(x for x in per_r if x["r"] == DOMINANT_R)
    dominant_kernel = "decode_plain_kernel<6,%d>" % hm.hamming_plain_config_get(DOMINANT_R)[0]
    traffic = recorded_traffic(dominant_kernel)
    bits_per_step = sum(n_cw * ((1 << r) - 1 - r) for r in WORKLOAD_R)
    value = bits_per_step / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "plain decode, one packet of 2^%d codewords each of Hamming(15,11), "
                        "(31,26), (63,57); uniform random messages; %.0f%% single-bit errors at "
                        "uniform positions" % (args.log2_cw, P_SINGLE * 100),
            "n_cw_per_packet": n_cw, "r": list(WORKLOAD_R), "p_single": P_SINGLE,
        },
        "roofline": {
            "kernel": dominant_kernel,
            "bound": "hbm",
            "achieved": dom["algorithmic_GBps"],
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": dom["frac_hbm"],
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(algorithmic_bytes_per_codeword(DOMINANT_R) * n_cw),
            "avg_launch_us": dom["avg_us"],
            "min_launch_us": dom["min_us"],
            "max_launch_us": dom["max_us"],
            "runtime_d2d_copy_GBps": copy_ceiling(dev),
        },
        "per_r": per_r,
        "tuned_shapes": tuned,
    }
    emit({"leg": "plain", "per_r": per_r, "roofline": out["roofline"], "tuned_shapes": tuned})
    del packets
    torch.cuda.empty_cache()

    def run_leg(key, fn, *a):
        t0 = time.perf_counter()
        out[key] = fn(*a)
        emit({"leg": key, "elapsed_s": round(time.perf_counter() - t0, 1), **out[key]})

    if "latency" in legs:
        run_leg("latency_hamming74", latency_leg, dev, 1000)
    if "sizes" in legs:
        run_leg("size_sweep", sizes_leg, dev)
    if "r7" in legs:
        run_leg("hamming127", hamming127_leg, dev, 20)
    if "errors" in legs:
        run_leg("error_rates", errors_leg, dev, 20)
    if "batch" in legs:
        run_leg("batched", batched_leg, dev, args.batch_packets, 5)
    if "serve" in legs:
        gBps = {x["r"]: x["algorithmic_GBps"] for x in per_r}
        if "hamming127" in out:
            gBps[7] = out["hamming127"]["frac_hbm"] * HBM_PEAK_GBPS
        gBps.setdefault(7, gBps[DOMINANT_R])
        run_leg("serving", serving_leg, dev, gBps, SERVE_LOADS, args.serve_requests,
                max(200, args.serve_requests // 10), args.serve_batch_log2)
    if "host" in legs:
        run_leg("host_pipeline", host_leg, dev, 3)
    if "planes" in legs:
        run_leg("planes", planes_leg, dev, 10)
    if "encode" in legs:
        run_leg("encode", encode_leg, dev, 10)
    if "seg" in legs:
        shapes = SEG_SHAPES
        if args.seg_shapes:
            shapes = [tuple(int(v) for v in s.split("/")) for s in args.seg_shapes.split(",")]
        # 20 timed launches after 10 untimed ones per shape: consecutive launches of one shape vary
        # by up to 15%, so a median of 5 moved between runs by as much
        run_leg("segmented", segmented_leg, dev, args.seg_packets, 20, 200, shapes)
    if not args.no_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(args.cpu_log2)
        cb = out["cpu_baseline"]
        cb["gpu_over_oracle"] = {
            "all_threads": round(out["value"] / cb["value"], 0),
            "single_thread_r6": round(dom["payload_Gbps"] / cb["single_thread_Gbps_r6"], 0)}
        if "segmented" in out:
            cpu = out["cpu_baseline"]["segmented_us_per_packet_1thread"]
            for row in out["segmented"]["shapes"]:
                c = cpu.get("%d/%d" % (row["M"], row["t"]))
                if c:
                    row["speedup_vs_oracle_1thread"] = {
                        "single_packet": round(c / row["single_packet_p50_us"], 1),
                        "batched": round(c / row["us_per_packet_batched"], 0)}
        emit({"leg": "cpu_baseline", "elapsed_s": round(time.perf_counter() - t0, 1), **cb})
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(out, fh, indent=1)
    emit(summary_line(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())

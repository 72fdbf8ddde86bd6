"""GPU tests of the serving core: every request's result is the same decoded
alone (plain call), in the mix (continuous batching) and by the oracle;
admission waits for output memory; batches overlap; the open-loop trace
runner completes.  Tolerance: 0 bits."""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words

pytestmark = pytest.mark.gpu


def _pool(seed, sizes, rs):
    chunks, offs, ys = [], [], []
    off = 0
    for i, (n_cw, r) in enumerate(zip(sizes, rs)):
        y = received_words(synth.workload_seed("serve", r, seed * 7919 + i), n_cw, r, p_single=0.1, p_double=0.02)
        offs.append(off)
        chunks.append(y)
        ys.append(y)
        off += y.size
    return np.concatenate(chunks + [np.zeros(2, dtype=np.uint64)]), offs, ys


def _to_dev(a, dev):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)


def _drain(srv, want, limit=200000):
    got = {}
    for _ in range(limit):
        srv.progress()
        for c in srv.poll():
            got[c.request_id] = c
        if len(got) >= want:
            return got
    raise AssertionError("server did not finish: %d of %d" % (len(got), want))


def _check_request(srv, c, y, r, cw_dev, off):
    import torch

    assert c.status == 0
    n_cw = y.size // hm.words_per_codeword(r)
    d, e = srv.result(c, r, n_cw)
    torch.cuda.synchronize()
    d_mix, e_mix = d.cpu().numpy(), e.cpu().numpy()
    d_ref, e_ref = oracle.decode(y, r)
    assert np.array_equal(d_mix, d_ref) and np.array_equal(e_mix, e_ref)
    wpc = hm.words_per_codeword(r)
    d_alone, e_alone = hm.decode(cw_dev[off:off + n_cw * wpc], r)
    torch.cuda.synchronize()
    assert np.array_equal(d_mix, d_alone.cpu().numpy()) and np.array_equal(e_mix, e_alone.cpu().numpy())


def test_serve_results_same_alone_in_mix_and_oracle(gpu_device):
    """Small batches (at most 8 requests): the one-launch form, with empty
    requests and every r among them."""
    rng = np.random.default_rng(5)
    n = 48
    sizes = [int(rng.choice([0, 1, 63, 64, 65, 300, 4097, 20000, 70000])) for _ in range(n)]
    rs = [int(rng.integers(3, 8)) for _ in range(n)]
    pool, offs, ys = _pool(1, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    srv = hm.Server(cw, slots=3, max_batch_packets=8, max_batch_codewords=100000, output_pool_bytes=64 << 20)
    try:
        ids = {}
        for i in range(n):                     # arrivals interleaved with progress: continuous batching
            ids[srv.submit(offs[i], sizes[i], rs[i])] = i
            if i % 5 == 4:
                srv.progress()
        got = _drain(srv, n)
        assert srv.stats()["batches"] >= n // 8
        for rid, c in got.items():
            i = ids[rid]
            if sizes[i]:
                _check_request(srv, c, ys[i], rs[i], cw, offs[i])
            srv.release(rid)
        assert srv.stats()["output_bytes_used"] == 0
    finally:
        srv.close()


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
def test_serve_small_batches_under_every_batch_schedule(gpu_device, schedule):
    """The one-launch small-batch form counts tiles on the host with the lane
    widths of the batch schedule in force; every schedule must give the same
    results."""
    rng = np.random.default_rng(20 + schedule)
    n = 24
    sizes = [int(rng.choice([1, 64, 100, 513, 2048, 9000])) for _ in range(n)]
    rs = [3 + i % 5 for i in range(n)]
    pool, offs, ys = _pool(10 + schedule, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    old = hm.hamming_batch_config_get()
    hm.hamming_batch_config_set(schedule, old[1], old[2], old[3])
    srv = hm.Server(cw, slots=2, max_batch_packets=6, max_batch_codewords=1 << 20, output_pool_bytes=64 << 20)
    try:
        ids = {}
        for i in range(n):
            ids[srv.submit(offs[i], sizes[i], rs[i])] = i
            if i % 3 == 2:
                srv.progress()
        got = _drain(srv, n)
        for rid, c in got.items():
            i = ids[rid]
            _check_request(srv, c, ys[i], rs[i], cw, offs[i])
            srv.release(rid)
    finally:
        srv.close()
        hm.hamming_batch_config_set(*old)


def test_serve_large_batch_through_the_host_plan(gpu_device):
    """Batches above 16 requests are planned on the host (prefix sums and a
    coarse tile map copied with the descriptors, then one decode launch)
    rather than the one-launch small-batch form the other tests exercise;
    the results must be the same."""
    rng = np.random.default_rng(11)
    n = 40
    sizes = [int(rng.choice([0, 1, 63, 64, 65, 300, 4097])) for _ in range(n)]
    rs = [int(rng.integers(3, 8)) for _ in range(n)]
    pool, offs, ys = _pool(4, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    srv = hm.Server(cw, slots=2, max_batch_packets=64, max_batch_codewords=1 << 30, output_pool_bytes=64 << 20)
    try:
        ids = {srv.submit(offs[i], sizes[i], rs[i]): i for i in range(n)}
        got = _drain(srv, n)
        assert srv.stats()["batches"] == 1
        for rid, c in got.items():
            i = ids[rid]
            if sizes[i]:
                _check_request(srv, c, ys[i], rs[i], cw, offs[i])
            srv.release(rid)
    finally:
        srv.close()


def test_serve_batches_overlap_in_flight(gpu_device):
    sizes = [1 << 20] * 6
    rs = [5, 6, 7, 4, 5, 6]
    pool, offs, ys = _pool(2, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    srv = hm.Server(cw, slots=2, max_batch_packets=4, max_batch_codewords=1 << 20, output_pool_bytes=256 << 20)
    try:
        ids = {srv.submit(offs[i], sizes[i], rs[i]): i for i in range(6)}
        srv.progress()
        st = srv.stats()
        # two one-request batches are on the GPU at once; four requests wait
        assert st["inflight"] == 2 and st["queued"] == 4 and st["batches"] == 2
        got = _drain(srv, 6)
        for rid, c in got.items():
            _check_request(srv, c, ys[ids[rid]], rs[ids[rid]], cw, offs[ids[rid]])
            srv.release(rid)
    finally:
        srv.close()


def test_serve_admission_waits_for_output_memory(gpu_device):
    sizes = [50000] * 10
    rs = [7] * 10
    pool, offs, ys = _pool(3, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    one = ((50000 * 120 + 63) // 64) * 8 + 50000
    srv = hm.Server(cw, slots=4, max_batch_packets=16, max_batch_codewords=1 << 30,
                    output_pool_bytes=2 * one + 4096, auto_release=False)
    try:
        ids = {srv.submit(offs[i], sizes[i], rs[i]): i for i in range(10)}
        srv.progress()
        st = srv.stats()
        assert st["inflight"] <= 2 and st["queued"] >= 8       # only two requests' outputs fit
        done = 0
        while done < 10:
            srv.progress()
            for c in srv.poll():
                _check_request(srv, c, ys[ids[c.request_id]], 7, cw, offs[ids[c.request_id]])
                srv.release(c.request_id)                      # frees room for the next ones
                done += 1
    finally:
        srv.close()


def test_serve_submit_validation(gpu_device):
    pool = np.zeros(1000, dtype=np.uint64)
    cw = _to_dev(pool, gpu_device)
    srv = hm.Server(cw, slots=1, max_batch_packets=4, output_pool_bytes=1 << 20, max_queue=8)
    try:
        for args, code in (((0, 10, 8), hm.HAMMING_EINVAL), ((0, 10, 2), hm.HAMMING_EINVAL),
                           ((990, 20, 4), hm.HAMMING_ERANGE), ((0, 501, 7), hm.HAMMING_ERANGE),
                           ((2000, 0, 4), hm.HAMMING_ERANGE)):
            with pytest.raises(hm.HammingError) as e:
                srv.submit(*args)
            assert e.value.status == code
        srv.submit(0, 500, 7)                                   # exactly the whole pool
        srv.submit(1000, 0, 4)                                  # empty request at the end
        got = _drain(srv, 2)
        assert all(c.status == 0 for c in got.values())
    finally:
        srv.close()


def test_serve_queue_limit(gpu_device):
    pool = np.zeros(1000, dtype=np.uint64)
    cw = _to_dev(pool, gpu_device)
    srv = hm.Server(cw, slots=1, max_batch_packets=4, output_pool_bytes=1 << 20, max_queue=2)
    try:
        srv.submit(0, 10, 4)
        srv.submit(10, 10, 4)
        with pytest.raises(hm.HammingError) as e:
            srv.submit(20, 10, 4)
        assert e.value.status == hm.HAMMING_ENOMEM
        _drain(srv, 2)
    finally:
        srv.close()


def test_serve_open_loop_trace(gpu_device):
    rng = np.random.default_rng(9)
    n = 400
    pool_words = 1 << 24
    cw = _to_dev(synth.draws(77, 0, pool_words), gpu_device)
    rs = rng.integers(4, 8, size=n).astype(np.uint32)
    sizes = np.floor(256 * np.exp2(10 * rng.random(n))).astype(np.uint64)
    wpc = np.where(rs == 7, 2, 1).astype(np.uint64)
    offs = (rng.random(n) * (pool_words - sizes * wpc - 1)).astype(np.uint64)
    gaps = rng.exponential(20e3, size=n)                     # mean 20 us between arrivals
    arrivals = np.cumsum(gaps).astype(np.uint64)
    srv = hm.Server(cw, slots=4, max_batch_packets=256, max_batch_codewords=1 << 24,
                    output_pool_bytes=1 << 30, auto_release=True)
    try:
        lat, elapsed = srv.run_trace(arrivals, offs, sizes, rs, timeout_s=60)
        assert (lat > 0).all() and lat.max() < 5e9
        assert elapsed >= int(arrivals[-1])
        assert srv.stats()["output_bytes_used"] == 0
    finally:
        srv.close()


@pytest.fixture(scope="module")
def trace_pool(gpu_device):
    """A codeword pool like the serving trace's, built on the CPU (seeded
    messages, the oracle's encoder, 10% single flips): one segment of 2^21
    codewords per r = 4, 5, 6 and 2^20 for r = 7; plus the plain decoder's
    measured rate on each segment."""
    import torch

    segs, base, off = [], {}, 0
    for r in (4, 5, 6, 7):
        n = 1 << (20 if r == 7 else 21)
        y = received_words(synth.workload_seed("serve-trace", r), n, r, p_single=0.1)
        base[r] = (off, n)
        segs.append(y)
        off += y.size
    host = np.concatenate(segs + [np.zeros(2, dtype=np.uint64)])
    cw = _to_dev(host, gpu_device)
    rate = {}
    for r, (o, n) in base.items():
        wpc = hm.words_per_codeword(r)
        seg = cw[o:o + n * wpc]
        data = torch.empty(hm.hamming_data_bytes(n, r), dtype=torch.uint8, device=gpu_device)
        ep = torch.empty(n, dtype=torch.uint8, device=gpu_device)
        times = []
        for _ in range(6):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            hm.hamming_decode(seg, n, r, data, ep)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) * 1e-3)
        rate[r] = n * hm.hamming_message_bits(r) / sorted(times)[3]      # payload bits per second
    return host, cw, base, rate


@pytest.mark.parametrize("rho", [0.7, 0.9])
def test_serve_trace_scale_results_alone_mix_and_oracle(gpu_device, trace_pool, rho):
    """The serving trace's shape: 256 SDR streams (stream s decodes r = 4 +
    s % 4), request sizes log-uniform in [256, 2^18] codewords, Poisson
    arrivals at 70% and 90% of the plain decoder's measured rate on the mix, 4
    batches in flight of at most 4,096 requests and 2^25 codewords.  Outputs
    stay resident (auto_release off), so every one of the 6,000 requests is
    compared with a plain decode of the same codewords alone, and 400 random
    ones with the oracle."""
    import torch

    host, cw, base, rate = trace_pool
    rng = np.random.default_rng(int(rho * 100))
    n = 6000
    stream_id = rng.integers(0, 256, size=n)
    rs = (4 + stream_id % 4).astype(np.uint32)
    sizes = np.floor(256 * np.exp2(10 * rng.random(n))).astype(np.uint64)
    offs = np.empty(n, dtype=np.uint64)
    for r, (o, seg_n) in base.items():
        m = rs == r
        offs[m] = np.uint64(o) + np.floor(rng.random(m.sum()) * (seg_n - sizes[m])).astype(np.uint64) * \
            np.uint64(hm.words_per_codeword(r))
    t_plain = np.array([float(sz) * hm.hamming_message_bits(int(r)) / rate[int(r)] for sz, r in zip(sizes, rs)])
    arrivals = (np.cumsum(rng.exponential(t_plain.mean() / rho, size=n)) * 1e9).astype(np.uint64)
    out_bytes = sum((((hm.hamming_data_bytes(int(sz), int(r)) + 15) // 16 * 16 + int(sz) + 255) // 256) * 256
                    for sz, r in zip(sizes, rs))
    srv = hm.Server(cw, slots=4, max_batch_packets=4096, max_batch_codewords=1 << 25,
                    output_pool_bytes=out_bytes + (1 << 20), auto_release=False)
    try:
        lat, _ = srv.run_trace(arrivals, offs, sizes, rs, timeout_s=60)
        assert (lat > 0).all()
        got = {}
        for c in srv.poll(max_n=2 * n):
            got[c.request_id] = c
        assert len(got) == n and all(c.status == 0 for c in got.values())
        assert srv.stats()["batches"] < n          # requests were batched together
        ids = sorted(got)
        check = set(rng.choice(n, size=400, replace=False).tolist())
        for i, rid in enumerate(ids):
            r, sz, o = int(rs[i]), int(sizes[i]), int(offs[i])
            wpc = hm.words_per_codeword(r)
            d_mix, e_mix = srv.result(got[rid], r, sz)
            d_alone, e_alone = hm.decode(cw[o:o + sz * wpc], r)
            assert torch.equal(d_mix, d_alone) and torch.equal(e_mix, e_alone), "request %d" % i
            if i in check:
                d_ref, e_ref = oracle.decode(host[o:o + sz * wpc], r)
                assert np.array_equal(d_mix.cpu().numpy(), d_ref), "request %d" % i
                assert np.array_equal(e_mix.cpu().numpy(), e_ref), "request %d" % i
        for rid in ids:
            srv.release(rid)
        assert srv.stats()["output_bytes_used"] == 0
    finally:
        srv.close()


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
@pytest.mark.parametrize("chunk_log2", [0, 3, 5])
def test_serve_host_plan_many_packets_every_schedule(gpu_device, schedule, chunk_log2):
    """Large host-planned batches (hundreds of requests, several with no
    codewords) whose coarse map groups several tiles per entry, under every
    batch schedule and several work chunks (chunks that span many tiny and
    empty requests)."""
    rng = np.random.default_rng(70 + schedule + 10 * chunk_log2)
    n = 600
    sizes = [int(rng.choice([0, 1, 63, 64, 65, 300, 1000, 4097, 30000])) for _ in range(n)]
    rs = [int(rng.integers(3, 8)) for _ in range(n)]
    pool, offs, ys = _pool(30 + schedule + 10 * chunk_log2, sizes, rs)
    cw = _to_dev(pool, gpu_device)
    old = hm.hamming_batch_config_get()
    old_chunk = hm.hamming_batch_chunk_get()
    hm.hamming_batch_config_set(schedule, 8, 0, old[3])
    hm.hamming_batch_chunk_set(chunk_log2)
    srv = hm.Server(cw, slots=2, max_batch_packets=300, max_batch_codewords=1 << 30, output_pool_bytes=1 << 30)
    try:
        ids = {srv.submit(offs[i], sizes[i], rs[i]): i for i in range(n)}
        got = _drain(srv, n)
        assert srv.stats()["batches"] == 2
        for rid, c in got.items():
            i = ids[rid]
            if sizes[i]:
                _check_request(srv, c, ys[i], rs[i], cw, offs[i])
            srv.release(rid)
    finally:
        srv.close()
        hm.hamming_batch_config_set(*old)
        hm.hamming_batch_chunk_set(old_chunk)

"""GPU parity of the batched decode: every packet of a batched launch is
byte-identical to the oracle (and so to a plain call on that packet alone),
output bytes between packets are untouched, invalid descriptors are flagged
and skipped, and graph replays stay correct.  Tolerance: 0 bits."""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000, 4097, 9999]


def _build_batch(seed, n_packets, sizes=None, rs=None, gap_words=True):
    """Host arena of received words and a descriptor array (offsets not laid out)."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = [int(rng.choice(SIZES)) for _ in range(n_packets)]
    if rs is None:
        rs = [int(rng.integers(3, 8)) for _ in range(n_packets)]
    descs = np.zeros(n_packets, dtype=hm.packet_dtype())
    chunks, off = [], 0
    ys = []
    for i, (n_cw, r) in enumerate(zip(sizes, rs)):
        gap = int(rng.integers(0, 3)) if gap_words else 0     # odd gaps give 8-byte-aligned packets
        if gap:
            chunks.append(np.full(gap, 0xDEADBEEF, dtype=np.uint64))
            off += gap
        y = received_words(synth.workload_seed("batch", r, seed * 100003 + i), n_cw, r,
                           p_single=0.3, p_double=0.1) if n_cw else np.zeros(0, dtype=np.uint64)
        descs[i]["in_word_off"] = off
        descs[i]["n_cw"] = n_cw
        descs[i]["r"] = r
        chunks.append(y)
        ys.append(y)
        off += y.size
    arena = np.concatenate(chunks + [np.zeros(2, dtype=np.uint64)])
    return arena, descs, ys


def _expect(ys, descs):
    return [oracle.decode(y, int(d["r"])) for y, d in zip(ys, descs)]


def _to_dev(a, dev):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)


def _check_outputs(bd, descs, expect, data_fill=None, ep_fill=None, skip=()):
    data = bd.data.cpu().numpy().view(np.uint8)
    ep = bd.errpos.cpu().numpy()
    covered_d = np.zeros(data.size, dtype=bool)
    covered_e = np.zeros(ep.size, dtype=bool)
    for i, (d, (dref, eref)) in enumerate(zip(descs, expect)):
        if i in skip:
            continue
        o = int(d["data_word_off"]) * 8
        assert np.array_equal(data[o:o + dref.size], dref), "packet %d data" % i
        covered_d[o:o + dref.size] = True
        if int(d["errpos_off"]) != hm.HAMMING_NO_ERRPOS:
            e = int(d["errpos_off"])
            assert np.array_equal(ep[e:e + eref.size], eref), "packet %d errpos" % i
            covered_e[e:e + eref.size] = True
    if data_fill is not None:
        assert (data[~covered_d] == data_fill).all()
    if ep_fill is not None:
        assert (ep[~covered_e] == ep_fill).all()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batch_matches_oracle_and_leaves_gaps(gpu_device, seed):
    import torch

    arena, descs, ys = _build_batch(seed, 60)
    expect = _expect(ys, descs)
    cw = _to_dev(arena, gpu_device)
    bd = hm.BatchDecoder(cw, 64)
    bd.set_packets(descs)
    bd.data.fill_(0x5A5A5A5A5A5A5A5A)
    bd.errpos.fill_(0xA5)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bd.decode(stream=s)
    torch.cuda.synchronize()
    assert not bd.status[:descs.size].cpu().numpy().any()
    _check_outputs(bd, descs, expect, data_fill=0x5A, ep_fill=0xA5)


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
@pytest.mark.parametrize("xcd_chunk", [1, 3, 64])
@pytest.mark.parametrize("grid_cap", [0, 1, 5])
@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("chunk_log2", [0, 3, 6])
def test_batch_every_schedule_grid_and_launch_mode(gpu_device, schedule, xcd_chunk, grid_cap, use_graph,
                                                    chunk_log2):
    import torch

    old = hm.hamming_batch_config_get()
    old_chunk = hm.hamming_batch_chunk_get()
    arena, descs, ys = _build_batch(7 + grid_cap + 10 * xcd_chunk + 1000 * chunk_log2, 40)
    expect = _expect(ys, descs)
    cw = _to_dev(arena, gpu_device)
    try:
        hm.hamming_batch_config_set(schedule, xcd_chunk, grid_cap, use_graph)
        hm.hamming_batch_chunk_set(chunk_log2)
        bd = hm.BatchDecoder(cw, 40)
        bd.set_packets(descs)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bd.decode(stream=s)
        torch.cuda.synchronize()
        _check_outputs(bd, descs, expect)
    finally:
        hm.hamming_batch_config_set(*old)
        hm.hamming_batch_chunk_set(old_chunk)


def test_batch_on_default_stream(gpu_device):
    import torch

    arena, descs, ys = _build_batch(11, 25)
    expect = _expect(ys, descs)
    bd = hm.BatchDecoder(_to_dev(arena, gpu_device), 25)
    bd.set_packets(descs)
    bd.decode(stream=0)
    torch.cuda.synchronize()
    _check_outputs(bd, descs, expect)


def test_batch_packet_equals_plain_call(gpu_device):
    import torch

    arena, descs, ys = _build_batch(21, 12, sizes=[5000] * 12, rs=[3, 4, 5, 6, 7, 7, 6, 5, 4, 3, 6, 7])
    cw = _to_dev(arena, gpu_device)
    bd = hm.BatchDecoder(cw, 12)
    bd.set_packets(descs)
    bd.decode()
    torch.cuda.synchronize()
    data = bd.data.cpu().numpy().view(np.uint8)
    ep = bd.errpos.cpu().numpy()
    for i, d in enumerate(descs):
        r, n_cw = int(d["r"]), int(d["n_cw"])
        wpc = hm.words_per_codeword(r)
        o = int(d["in_word_off"])
        pd, pe = hm.decode(cw[o:o + n_cw * wpc], r)
        torch.cuda.synchronize()
        pd = pd.cpu().numpy()
        assert np.array_equal(data[int(d["data_word_off"]) * 8:][:pd.size], pd)
        assert np.array_equal(ep[int(d["errpos_off"]):][:n_cw], pe.cpu().numpy())


def test_batch_invalid_descriptors_are_flagged_and_skipped(gpu_device):
    import torch

    arena, descs, ys = _build_batch(31, 10, sizes=[300] * 10, rs=[4, 5, 6, 7, 3, 4, 5, 6, 7, 3])
    expect = _expect(ys, descs)
    hm.hamming_batch_layout(descs)
    dw = int(max(d["data_word_off"] for d in descs)) + 64
    eb = int(max(d["errpos_off"] for d in descs)) + 512
    bad = descs.copy()
    bad[1]["r"] = 9                                   # bad r
    bad[3]["flags"] = 1                               # reserved flags
    bad[5]["in_word_off"] = arena.size                # codewords past the arena
    bad[7]["data_word_off"] = dw                      # message range past the arena
    bad[9]["errpos_off"] = eb - 100                   # errpos range past the arena
    bad[8]["errpos_off"] = hm.HAMMING_NO_ERRPOS       # valid: no errpos wanted
    cw = _to_dev(arena, gpu_device)
    bd = hm.BatchDecoder(cw, 10)
    bd.set_packets(bad, layout=False, data_words=dw, errpos_bytes=eb)
    bd.data.fill_(0x1111111111111111)
    bd.errpos.fill_(0x22)
    bd.decode()
    torch.cuda.synchronize()
    st = bd.status.cpu().numpy()[:10]
    assert list(st) == [0, hm.HAMMING_EINVAL, 0, hm.HAMMING_EINVAL, 0, hm.HAMMING_ERANGE, 0,
                        hm.HAMMING_ERANGE, 0, hm.HAMMING_ERANGE]
    _check_outputs(bd, bad, expect, skip=(1, 3, 5, 7, 9))
    # skipped packets wrote nothing into their laid-out ranges
    data = bd.data.cpu().numpy().view(np.uint8)
    for i in (1, 3, 5):
        o = int(descs[i]["data_word_off"]) * 8
        assert (data[o:o + expect[i][0].size] == 0x11).all()


def test_batch_device_count_below_max_and_graph_replays(gpu_device):
    """One graph serves several batch sizes: the packet count lives on the
    device.  Replays are checked one by one, with eager work in between."""
    import torch

    arena, descs, ys = _build_batch(41, 30)
    expect = _expect(ys, descs)
    cw = _to_dev(arena, gpu_device)
    bd = hm.BatchDecoder(cw, 30)
    bd.set_packets(descs)
    s = torch.cuda.Stream()
    for n in (30, 7, 0, 19, 30, 1):
        bd.data.fill_(0x3333333333333333)
        bd.errpos.fill_(0x44)
        bd.n_dev.fill_(n)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bd.decode(stream=s)
        torch.cuda.synchronize()
        _check_outputs(bd, descs[:n], expect[:n], data_fill=0x33, ep_fill=0x44)


def test_batch_empty_and_all_empty(gpu_device):
    import torch

    arena = np.zeros(4, dtype=np.uint64)
    cw = _to_dev(arena, gpu_device)
    bd = hm.BatchDecoder(cw, 4)
    descs = np.zeros(4, dtype=hm.packet_dtype())
    descs["r"] = [3, 4, 5, 7]
    bd.set_packets(descs)
    bd.decode()
    torch.cuda.synchronize()
    assert not bd.status.cpu().numpy().any()


def test_batch_small_grid_hint_and_coarse_map(gpu_device):
    """A max_codewords hint far below the batch (grid smaller than the tile
    count: waves loop) and a map whose groups span many tiles (more tiles than
    map entries) still decode every packet exactly."""
    import torch

    arena, descs, ys = _build_batch(51, 3, sizes=[300000, 77, 250000], rs=[4, 7, 3])
    expect = _expect(ys, descs)
    bd = hm.BatchDecoder(_to_dev(arena, gpu_device), 3)
    bd.set_packets(descs)
    for hint in (1, 1000, 0):
        bd.data.fill_(0x6666666666666666)
        bd.decode(max_codewords=hint)
        torch.cuda.synchronize()
        _check_outputs(bd, descs, expect)


def _decode_with_workspace(gpu_device, arena, descs, ws_bytes, max_codewords=0):
    import torch

    bd = hm.BatchDecoder(_to_dev(arena, gpu_device), descs.size, workspace_bytes=ws_bytes)
    bd.set_packets(descs)
    bd.data.fill_(0x7777777777777777)
    bd.errpos.fill_(0x88)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bd.decode(stream=s, max_codewords=max_codewords)
    torch.cuda.synchronize()
    return bd


@pytest.mark.parametrize("chunk_log2,fine_log2", [(0, 1), (0, 3), (0, 6), (2, 3), (3, 6), (1, 1)])
@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_grouped_fine_map_probe_path(gpu_device, chunk_log2, fine_log2, schedule, use_graph):
    """A workspace below the recommended size gives a fine map of 2^g tiles
    per entry; when an entry spans more than one chunk, every wave probes the
    prefix sums from its entry's packet.  The map size is chosen from the
    batch's tile count so that g is exactly fine_log2 (never below the chunk
    size; equal to it, the map is exact at every chunk start), and the
    outputs must stay byte-exact."""
    old = hm.hamming_batch_config_get()
    old_chunk = hm.hamming_batch_chunk_get()
    arena, descs, ys = _build_batch(300 + fine_log2 + 7 * schedule + 50 * chunk_log2, 60)
    expect = _expect(ys, descs)
    n = descs.size
    try:
        hm.hamming_batch_config_set(schedule, 1, 0, use_graph)
        hm.hamming_batch_chunk_set(chunk_log2)
        full = _decode_with_workspace(gpu_device, arena, descs, hm.hamming_batch_workspace_bytes(n))
        tiles = full.totals()["tiles"]
        assert full.totals()["fine_log2"] == chunk_log2 and tiles >= 1 << fine_log2
        _check_outputs(full, descs, expect, data_fill=0x77, ep_fill=0x88)
        entries = (tiles >> fine_log2) + 1
        ws = hm.hamming_batch_workspace_min_bytes(n) - 4 + 4 * entries
        bd = _decode_with_workspace(gpu_device, arena, descs, ws)
        assert bd.totals()["fine_log2"] == fine_log2 and bd.totals()["tiles"] == tiles
        _check_outputs(bd, descs, expect, data_fill=0x77, ep_fill=0x88)
    finally:
        hm.hamming_batch_config_set(*old)
        hm.hamming_batch_chunk_set(old_chunk)


@pytest.mark.parametrize("schedule", [0, 2, 3])
@pytest.mark.parametrize("grid_cap", [0, 3])
def test_batch_one_fine_entry_probes_across_many_packets(gpu_device, schedule, grid_cap):
    """The smallest workspace (one fine entry) over 400 tiny and empty packets:
    every wave probes from packet 0, through several 64-entry windows and over
    runs of packets without tiles; with a grid cap the waves also loop."""
    old = hm.hamming_batch_config_get()
    rng = np.random.default_rng(400 + schedule)
    sizes = [int(rng.choice([0, 0, 1, 5, 64, 127, 128, 129, 300])) for _ in range(400)]
    rs = [int(rng.integers(3, 8)) for _ in range(400)]
    arena, descs, ys = _build_batch(500 + schedule, 400, sizes=sizes, rs=rs)
    expect = _expect(ys, descs)
    try:
        hm.hamming_batch_config_set(schedule, 1, grid_cap, 1)
        bd = _decode_with_workspace(gpu_device, arena, descs, hm.hamming_batch_workspace_min_bytes(400))
        t = bd.totals()
        assert t["tiles"] > 64 and (t["tiles"] >> t["fine_log2"]) == 0
        assert not bd.status[:400].cpu().numpy().any()
        _check_outputs(bd, descs, expect, data_fill=0x77, ep_fill=0x88)
    finally:
        hm.hamming_batch_config_set(*old)


def test_batch_workspace_below_minimum_is_rejected(gpu_device):
    import torch

    arena, descs, _ = _build_batch(600, 4)
    cw = _to_dev(arena, gpu_device)
    small = hm.hamming_batch_workspace_min_bytes(4) - 1
    with pytest.raises(hm.HammingError) as e:
        bd = hm.BatchDecoder(cw, 4, workspace_bytes=small)
        bd.set_packets(descs)
        bd.decode()
    assert e.value.status == hm.HAMMING_ENOMEM
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def full_batch(gpu_device):
    """The bench's batched workload at full size (20,000 packets, ~2.2e9
    codewords: messages and flips drawn on the device by the seeded
    generator, codewords from the library's encoder), decoded by one
    hamming_decode_batch call in the bench's launch configuration; the outputs
    come back to the host (about 17 GB)."""
    import os
    import sys

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench

    n_packets = 20000
    seed = synth.workload_seed("bench-batch", 0)
    arena, descs, per_r, n_cw, r = bench.build_batch(gpu_device, n_packets, seed)
    del per_r
    torch.cuda.empty_cache()
    if os.path.exists(bench.TUNED_SHAPES):
        try:
            hm.hamming_tune_load(bench.TUNED_SHAPES)
        except hm.HammingError:
            pass
    bd = hm.BatchDecoder(arena, n_packets)
    bd.set_packets(descs)
    bd.decode()
    torch.cuda.synchronize()
    status = bd.status[:n_packets].cpu().numpy()
    data = bd.data.view(torch.uint8).cpu().numpy()
    ep = bd.errpos.cpu().numpy()
    del bd, arena
    torch.cuda.empty_cache()
    _, _, p = synth.batch_packets(seed, n_packets)
    # first codeword of each packet inside its r's generated stream
    pos = np.zeros(n_packets, dtype=np.int64)
    for rr in range(3, 8):
        idx = np.flatnonzero(r == rr)
        pos[idx] = np.concatenate([[0], np.cumsum(n_cw[idx])[:-1]])
    return {"seed": seed, "descs": descs, "n_cw": n_cw, "r": r, "p": p, "pos": pos, "status": status,
            "data": data, "errpos": ep}


@pytest.mark.parametrize("rr", [3, 4, 5, 6, 7])
def test_batch_full_size_every_packet_recovers_its_message(full_batch, rr):
    """Every packet of code r of the full-size batch: each received word
    carries at most one flip, so the exact decode is fixed without running a
    decoder (a single-error-correcting code returns the sent message and names
    the flipped position): the payload must equal the generator's message
    stream for those codewords and errpos its flip positions (0 where none),
    byte for byte.  Together with the oracle comparison below and the
    encoder's own parity tests, this covers all 20,000 packets."""
    fb = full_batch
    assert not fb["status"].any()
    sr = synth.subseed(fb["seed"], "r", rr)
    for i in np.flatnonzero(fb["r"] == rr):
        n, first = int(fb["n_cw"][i]), int(fb["pos"][i])
        msg = synth.message_stream_slice(sr, first, n, rr).view(np.uint8)
        p1, p2 = synth.error_positions(sr, n, rr, p_single=float(fb["p"][i]), start=first)
        assert not p2.any()
        o, e = int(fb["descs"][i]["data_word_off"]) * 8, int(fb["descs"][i]["errpos_off"])
        assert np.array_equal(fb["data"][o:o + msg.size], msg), "packet %d (r=%d, n=%d)" % (i, rr, n)
        assert np.array_equal(fb["errpos"][e:e + n], p1), "packet %d (r=%d, n=%d)" % (i, rr, n)


def test_batch_full_size_oracle_on_small_and_sampled_packets(full_batch):
    """The oracle on the full-size batch: every packet of at most 2^14
    codewords (more than half of the 20,000) and 60 random larger ones plus
    the largest and smallest of each r, regenerated on the CPU from the same
    seeded streams, encoded by the oracle's encoder, decoded by the oracle and
    compared with the batch output byte for byte."""
    fb = full_batch
    n_cw, r = fb["n_cw"], fb["r"]
    rng = np.random.default_rng(3)
    large = np.flatnonzero(n_cw > (1 << 14))
    sample = set(np.flatnonzero(n_cw <= (1 << 14)).tolist())
    sample |= set(rng.choice(large, size=60, replace=False).tolist())
    for rr in range(3, 8):
        idx = np.flatnonzero(r == rr)
        sample.add(int(idx[np.argmax(n_cw[idx])]))
        sample.add(int(idx[np.argmin(n_cw[idx])]))
    assert len(sample) > 10000
    for i in sorted(sample):
        rr, n, first = int(r[i]), int(n_cw[i]), int(fb["pos"][i])
        sr = synth.subseed(fb["seed"], "r", rr)
        msg = synth.message_stream_slice(sr, first, n, rr)
        cw = oracle.encode(msg, n, rr)
        p1, p2 = synth.error_positions(sr, n, rr, p_single=float(fb["p"][i]), start=first)
        d_ref, e_ref = oracle.decode(cw ^ synth.flip_masks(p1, p2, rr), rr)
        o, e = int(fb["descs"][i]["data_word_off"]) * 8, int(fb["descs"][i]["errpos_off"])
        assert np.array_equal(fb["data"][o:o + d_ref.size], d_ref), "packet %d (r=%d, n=%d)" % (i, rr, n)
        assert np.array_equal(fb["errpos"][e:e + n], e_ref), "packet %d (r=%d, n=%d)" % (i, rr, n)

"""GPU parity of the plain decode (and the encoder) against the CPU oracle.

Tolerance: 0 bits.  The arithmetic is integer GF(2) and the decoder is a
total function with exactly one correct output per input, so the data stream
and the error positions must be byte-identical to the oracle's.
"""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words, to_device, to_host_u8

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4097, 20000]


def _check(y, r, device, stream=None):
    import torch

    d_ref, e_ref = oracle.decode(y, r)
    data, ep = hm.decode(to_device(y, device), r, stream=stream)
    torch.cuda.synchronize()
    assert np.array_equal(to_host_u8(data), d_ref)
    assert np.array_equal(to_host_u8(ep), e_ref)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("n_cw", SIZES)
def test_plain_parity_ragged_sizes(gpu_device, r, n_cw):
    y = received_words(synth.workload_seed("gpu-ragged", r, n_cw), n_cw, r, p_single=0.3, p_double=0.1)
    _check(y, r, gpu_device)


@pytest.mark.parametrize("r", [4, 5, 6])
@pytest.mark.parametrize("p", synth.PLAIN_ERROR_RATES)
def test_plain_parity_error_rates(gpu_device, r, p):
    n_cw = 50000
    y = received_words(synth.workload_seed("gpu-rates", r, str(p)), n_cw, r, p_single=p)
    _check(y, r, gpu_device)


def test_plain_parity_hamming127_error_mix(gpu_device):
    # 70% clean, 25% one flip, 5% two flips (deterministic miscorrection)
    r, n_cw = 7, 30000
    y = received_words(synth.workload_seed("gpu-mix", r), n_cw, r, p_single=0.25, p_double=0.05)
    _check(y, r, gpu_device)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_plain_every_lane_shape_and_grid_cap(gpu_device, r):
    old = hm.hamming_plain_config_get(r)
    n_cw = 9000
    y = received_words(synth.workload_seed("gpu-shapes", r), n_cw, r, p_single=0.4, p_double=0.1)
    try:
        for u in (2, 4, 8, 16):
            if u * hm.hamming_message_bits(r) < 32:
                continue
            for cap, chunk in ((0, 1), (1, 1), (3, 2), (64, 4), (0, 3), (0, 64)):
                hm.hamming_plain_config_set(r, u, cap, chunk)
                _check(y, r, gpu_device)
    finally:
        hm.hamming_plain_config_set(r, *old)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_plain_looping_grid_large_ragged(gpu_device, r):
    # grids far smaller than the packet: every wave decodes many full tiles
    # with the next tile's loads in flight, then one wave takes the ragged tail
    old = hm.hamming_plain_config_get(r)
    n_cw = 300_013
    y = received_words(synth.workload_seed("gpu-loop", r), n_cw, r, p_single=0.3, p_double=0.05)
    try:
        for cap, chunk in ((5, 1), (37, 2), (256, 8), (2048, 32)):
            hm.hamming_plain_config_set(r, hm.hamming_plain_config_get(r)[0], cap, chunk)
            _check(y, r, gpu_device)
    finally:
        hm.hamming_plain_config_set(r, *old)


@pytest.mark.parametrize("r", [3, 6, 7])
def test_plain_unaligned_input_and_errpos(gpu_device, r):
    import torch

    n_cw = 3000
    wpc = hm.words_per_codeword(r)
    y = received_words(synth.workload_seed("gpu-unaligned", r), n_cw, r, p_single=0.5)
    d_ref, e_ref = oracle.decode(y, r)
    big = torch.zeros(y.size + 1, dtype=torch.int64, device=gpu_device)
    big[1:] = to_device(y, gpu_device)
    cw = big[1:]                                   # 8-byte but not 16-byte aligned
    assert cw.data_ptr() % 16 == 8
    nbytes = hm.hamming_data_bytes(n_cw, r)
    dbuf = torch.zeros(nbytes + 16, dtype=torch.uint8, device=gpu_device)
    data = dbuf[8:8 + nbytes]                      # 8-byte but not 16-byte aligned
    assert data.data_ptr() % 16 == 8
    epbuf = torch.zeros(n_cw + 3, dtype=torch.uint8, device=gpu_device)
    hm.hamming_decode(cw, n_cw, r, data, epbuf[1:])
    torch.cuda.synchronize()
    assert np.array_equal(to_host_u8(data), d_ref)
    db = to_host_u8(dbuf)
    assert not db[:8].any() and not db[8 + nbytes:].any()
    ep = to_host_u8(epbuf)
    assert np.array_equal(ep[1:n_cw + 1], e_ref)
    assert ep[0] == 0 and not ep[n_cw + 1:].any()
    assert wpc in (1, 2)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_plain_writes_nothing_outside_outputs_and_keeps_input(gpu_device, r):
    import torch

    n_cw = 4099
    y = received_words(synth.workload_seed("gpu-canary", r), n_cw, r, p_single=0.5)
    d_ref, e_ref = oracle.decode(y, r)
    nbytes = hm.hamming_data_bytes(n_cw, r)
    canary = 4096
    data = torch.full((nbytes + canary,), 0xA5, dtype=torch.uint8, device=gpu_device)
    ep = torch.full((n_cw + canary,), 0x5A, dtype=torch.uint8, device=gpu_device)
    cw = to_device(y, gpu_device)
    before = cw.clone()
    hm.hamming_decode(cw, n_cw, r, data, ep)
    torch.cuda.synchronize()
    d = to_host_u8(data)
    e = to_host_u8(ep)
    assert np.array_equal(d[:nbytes], d_ref) and (d[nbytes:] == 0xA5).all()
    assert np.array_equal(e[:n_cw], e_ref) and (e[n_cw:] == 0x5A).all()
    assert torch.equal(cw, before)


def test_plain_empty_packet_writes_nothing(gpu_device):
    import torch

    data = torch.full((64,), 7, dtype=torch.uint8, device=gpu_device)
    cw = torch.zeros(8, dtype=torch.int64, device=gpu_device)
    for r in range(3, 8):
        hm.hamming_decode(cw, 0, r, data, None)
    torch.cuda.synchronize()
    assert (data.cpu() == 7).all()


def test_plain_errpos_optional(gpu_device):
    import torch

    r, n_cw = 5, 7000
    y = received_words(synth.workload_seed("gpu-noep", r), n_cw, r, p_single=0.5)
    d_ref, _ = oracle.decode(y, r)
    data, ep = hm.decode(to_device(y, gpu_device), r, errpos=False)
    torch.cuda.synchronize()
    assert ep is None and np.array_equal(to_host_u8(data), d_ref)


def test_plain_on_side_stream(gpu_device):
    import torch

    r, n_cw = 6, 12345
    y = received_words(synth.workload_seed("gpu-stream", r), n_cw, r, p_single=0.5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _check(y, r, gpu_device, stream=s)


# ---- full workload sizes (the bench's launch configuration) ------------------

FULL = [
    (3, 65536, 0.5, 0.0),
    (4, 1 << 26, 0.1, 0.0),
    (5, 1 << 26, 0.1, 0.0),
    (6, 1 << 26, 0.1, 0.0),
    (7, 1 << 25, 0.25, 0.05),
]


@pytest.mark.parametrize("r,n_cw,p1,p2", FULL)
def test_plain_parity_full_size(gpu_device, r, n_cw, p1, p2):
    y = received_words(synth.workload_seed("gpu-full", r), n_cw, r, p_single=p1, p_double=p2)
    _check(y, r, gpu_device)


# ---- encoder -------------------------------------------------------------------

@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("n_cw", [1, 63, 64, 65, 511, 512, 513, 1000, 1023, 1024, 1025, 65537])
def test_encode_parity(gpu_device, r, n_cw):
    import torch

    stream = synth.message_stream(synth.workload_seed("gpu-enc", r, n_cw), n_cw, r)
    ref = oracle.encode(stream, n_cw, r)
    out = hm.encode(to_device(stream, gpu_device), n_cw, r)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref)


@pytest.mark.parametrize("r", [3, 6, 7])
@pytest.mark.parametrize("n_cw", [1, 2, 65, 4097])
def test_encode_parity_unaligned_output(gpu_device, r, n_cw):
    """Output 8-byte but not 16-byte aligned: the encoder takes its 64-bit
    store form; the words around the output stay untouched."""
    import torch

    wpc = hm.words_per_codeword(r)
    stream = synth.message_stream(synth.workload_seed("gpu-enc-unaligned", r, n_cw), n_cw, r)
    ref = oracle.encode(stream, n_cw, r)
    buf = torch.full((n_cw * wpc + 2,), 0x5A5A5A5A5A5A5A5A, dtype=torch.int64, device=gpu_device)
    out = buf[1:1 + n_cw * wpc]
    assert out.data_ptr() % 16 == 8
    hm.hamming_encode(to_device(stream, gpu_device), n_cw, r, out)
    torch.cuda.synchronize()
    host = buf.cpu().numpy().view(np.uint64)
    assert np.array_equal(host[1:1 + n_cw * wpc], ref)
    assert host[0] == 0x5A5A5A5A5A5A5A5A and host[-1] == 0x5A5A5A5A5A5A5A5A


# 2^15 workgroups of 1,024 (r = 6) or 512 (r = 7) codewords, plus a few more
# tiles: the first workgroups loop, prefetching a second tile, the last of
# them ragged.
@pytest.mark.parametrize("r,n_cw", [(6, (1 << 25) + 3 * 1024 + 29), (7, (1 << 24) + 2 * 512 + 3)])
def test_encode_parity_grid_loop_sampled(gpu_device, r, n_cw):
    """Long-message encodes with more LDS-staged tiles than workgroups and a
    ragged last tile; slices of the output against the oracle, the input
    regenerated on the CPU from the same stream."""
    import torch

    seed = synth.workload_seed("gpu-enc-loop", r)
    cw = hm.encode(synth.message_stream_torch(seed, n_cw, r, gpu_device), n_cw, r)
    torch.cuda.synchronize()
    host = cw.cpu().numpy().view(np.uint64)
    wpc = hm.words_per_codeword(r)
    n = 3000
    rng = np.random.default_rng(n_cw)
    firsts = [0, 1021, n_cw // 2 + 3, n_cw - n - 7, n_cw - n] + [int(x) for x in rng.integers(0, n_cw - n, 4)]
    # the tiles the first workgroups take second
    tile = 1024 if r == 6 else 512
    firsts += [min(f, n_cw - n) for f in ((1 << 15) * tile - 17, (1 << 15) * tile + 100)]
    for first in firsts:
        ref = oracle.encode(synth.message_stream_slice(seed, first, n, r), n, r)
        assert np.array_equal(host[first * wpc:(first + n) * wpc], ref), first


def test_tuner_applies_and_persists_valid_shapes(gpu_device, tmp_path):
    import torch

    old_plain = {r: hm.hamming_plain_config_get(r) for r in range(3, 8)}
    old_batch = hm.hamming_batch_config_get()
    path = str(tmp_path / "tune.json")
    try:
        hm.hamming_tune(path, 3)
        torch.cuda.synchronize()
        text = open(path).read()
        assert '"device"' in text and text.count('"plain"') == 5 and '"batch"' in text
        tuned = {r: hm.hamming_plain_config_get(r) for r in range(3, 8)}
        for r in range(3, 8):
            hm.hamming_plain_config_set(r, *old_plain[r])
        hm.hamming_tune_load(path)
        assert {r: hm.hamming_plain_config_get(r) for r in range(3, 8)} == tuned
        # decoding with the tuned shapes is still exact
        for r in (3, 6, 7):
            y = received_words(synth.workload_seed("gpu-tuned", r), 5000, r, p_single=0.5)
            _check(y, r, gpu_device)
    finally:
        for r in range(3, 8):
            hm.hamming_plain_config_set(r, *old_plain[r])
        hm.hamming_batch_config_set(*old_batch)


def test_tuner_batch_only_keeps_the_loaded_plain_lines(gpu_device, tmp_path):
    """A run that tunes only the batched decode writes the plain shapes back as
    the cache it loaded held them, times included (the bench's traffic record
    is keyed on those lines), and a batch shape the library accepts."""
    import json
    import os

    import torch

    shipped = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                           "paper_1412_6862_amd", "tuned_shapes.json")
    old_plain = {r: hm.hamming_plain_config_get(r) for r in range(3, 8)}
    old_batch = hm.hamming_batch_config_get()
    old_chunk = hm.hamming_batch_chunk_get()
    path = str(tmp_path / "batch_only.json")
    try:
        hm.hamming_tune_load(shipped)
        hm.hamming_tune(path, 2)
        torch.cuda.synchronize()
        want = [ln for ln in open(shipped).read().splitlines() if ln.startswith(('{"device"', '{"plain"'))]
        got = open(path).read().splitlines()
        assert [ln for ln in got if ln.startswith(('{"device"', '{"plain"'))] == want
        batch = [json.loads(ln) for ln in got if ln.startswith('{"batch"')]
        assert len(batch) == 1 and batch[0]["batch"] in (0, 1, 2, 3) and batch[0]["ms"] > 0
        assert batch[0]["xcd_chunk"] in (1, 8, 16, 32, 64, 128)
        assert hm.hamming_batch_config_get()[:2] == (batch[0]["batch"], batch[0]["xcd_chunk"])
    finally:
        for r in range(3, 8):
            hm.hamming_plain_config_set(r, *old_plain[r])
        hm.hamming_batch_config_set(*old_batch)
        hm.hamming_batch_chunk_set(old_chunk)


@pytest.mark.parametrize("r", [4, 6])
def test_plain_parity_2p28_sampled(gpu_device, r):
    """The largest packet of the size sweep, 2^28 codewords, generated and
    encoded on the device; slices are regenerated on the CPU from the same
    counter-based streams and checked against the oracle one by one."""
    import torch

    n_cw, p = 1 << 28, 0.1
    seed = synth.workload_seed("gpu-2p28", r)
    cw = hm.encode(synth.message_stream_torch(seed, n_cw, r, gpu_device), n_cw, r)
    cw ^= synth.flip_masks_torch(seed, n_cw, r, p, gpu_device)
    data, ep = hm.decode(cw, r)
    torch.cuda.synchronize()
    del cw
    k = hm.hamming_message_bits(r)
    rng = np.random.default_rng(r)
    firsts = [0, n_cw // 2, n_cw - 4096] + [int(x) // 64 * 64 for x in rng.integers(0, n_cw - 4096, 5)]
    for first in firsts:
        n = 4096
        y = oracle.encode(synth.message_stream_slice(seed, first, n, r), n, r)
        p1, p2 = synth.error_positions(seed, n, r, p_single=p, start=first)
        y ^= synth.flip_masks(p1, p2, r)
        d_ref, e_ref = oracle.decode(y, r)
        b0 = first * k // 8
        assert np.array_equal(data[b0:b0 + d_ref.size].cpu().numpy(), d_ref), first
        assert np.array_equal(ep[first:first + n].cpu().numpy(), e_ref), first
    assert data.numel() == hm.hamming_data_bytes(n_cw, r)

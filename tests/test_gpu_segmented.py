"""GPU parity of the segmented-packet decode and encode (the paper's
t-segment packets, Sec. II, Fig. 1) against the CPU oracle.

Tolerance: 0 bits.  Messages, per-segment syndromes and packet status must
be identical to the oracle's; message bytes past M in the last word are 0.
"""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth

pytestmark = pytest.mark.gpu

MODES = [8, 16, 32, 64, 256]   # threads per packet


@pytest.fixture
def seg_mode(request):
    old = hm.hamming_seg_config_get()
    hm.hamming_seg_config_set(request.param)
    yield request.param
    hm.hamming_seg_config_set(old)


def _received(seed, P, msg_bytes, t, row_bytes, p_single, p_double):
    """Oracle-encoded random packets with per-segment channel flips."""
    msgs = synth.packet_bytes(seed, P, msg_bytes)
    enc = oracle.seg_encode_many(msgs, t, row_bytes=row_bytes)
    _, _, n, _ = oracle.seg_layout(msg_bytes, t)
    starts = np.concatenate([[0], np.cumsum(n)[:-1]])
    b1, b2 = synth.segment_flips(seed, P, starts, n, p_single, p_double)
    synth.apply_bit_flips(enc, b1, b2)
    return enc


def _check_batch(device, P, msg_bytes, t, p_single=0.4, p_double=0.2, garbage=True):
    import torch

    b = hm.SegmentedBatch(P, msg_bytes, t, device=device)
    seed = synth.workload_seed("gpu-seg", msg_bytes, t)
    enc = _received(seed, P, msg_bytes, t, b.enc_stride * 8, p_single, p_double)
    if garbage:   # bits after the last segment of each packet are ignored
        _, _, _, bits = oracle.seg_layout(msg_bytes, t)
        tail = np.unpackbits(enc, axis=1, bitorder="little")
        rnd = np.unpackbits(synth.packet_bytes(seed + 1, P, enc.shape[1]), axis=1, bitorder="little")
        tail[:, bits:] = rnd[:, bits:]
        enc = np.packbits(tail, axis=1, bitorder="little")
    b.enc.copy_(torch.from_numpy(enc.reshape(-1).view(np.int64)))
    b.msg.fill_(-1)
    b.decode()
    torch.cuda.synchronize()
    m_ref, s_ref, st_ref = oracle.seg_decode_many(enc, msg_bytes, t)
    got = b.msg.cpu().numpy().view(np.uint8).reshape(P, b.msg_stride * 8)
    assert np.array_equal(got[:, :msg_bytes], m_ref)
    assert not got[:, msg_bytes:].any()
    assert np.array_equal(b.syndromes.cpu().numpy().view(np.uint16).reshape(P, t), s_ref)
    assert np.array_equal(b.status.cpu().numpy(), st_ref)
    return st_ref


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
@pytest.mark.parametrize("msg_bytes", synth.PAPER_PACKET_BYTES)
@pytest.mark.parametrize("t", synth.PAPER_SEGMENTS)
def test_segmented_parity_papers_packet_shapes(gpu_device, seg_mode, msg_bytes, t):
    st = _check_batch(gpu_device, 301, msg_bytes, t)
    assert (st == 1).any() and (st == 2).any()       # clean packets: see the error-extremes test


@pytest.mark.parametrize("msg_bytes,t", [(1, 1), (1, 3), (1, 8), (7, 8), (13, 5), (3, 24), (57, 8), (15, 1),
                                         (4096, 1), (4096, 32), (1000, 32), (8, 1), (9, 1), (255, 7)])
@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
def test_segmented_parity_edge_shapes(gpu_device, seg_mode, msg_bytes, t):
    _check_batch(gpu_device, 130, msg_bytes, t)


@pytest.mark.parametrize("p_single,p_double", [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)])
@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
def test_segmented_parity_error_extremes(gpu_device, seg_mode, p_single, p_double):
    st = _check_batch(gpu_device, 200, 1200, 4, p_single, p_double)
    if p_single == 0 and p_double == 0:
        assert not st.any()
    if p_single == 1:
        assert (st == 1).all()


@pytest.mark.parametrize("seg_mode", MODES + [0], indirect=True)
@pytest.mark.parametrize("msg_bytes,t", [(400, 2), (2000, 6), (1, 1), (13, 5), (4096, 1), (4096, 32), (255, 7)])
def test_segmented_encoder_parity(gpu_device, seg_mode, msg_bytes, t):
    import torch

    P = 157
    b = hm.SegmentedBatch(P, msg_bytes, t, device=gpu_device)
    msgs = synth.packet_bytes(synth.workload_seed("gpu-seg-enc", msg_bytes, t), P, msg_bytes)
    rows = np.full((P, b.msg_stride * 8), 0xA5, dtype=np.uint8)    # bytes past M are ignored
    rows[:, :msg_bytes] = msgs
    b.msg.copy_(torch.from_numpy(rows.reshape(-1).view(np.int64)))
    b.enc.fill_(-1)
    b.encode()
    torch.cuda.synchronize()
    want = oracle.seg_encode_many(msgs, t, row_bytes=b.enc_stride * 8)
    assert np.array_equal(b.enc.cpu().numpy().view(np.uint8).reshape(P, -1), want)
    # and the decoder takes the encoder's output back to the messages
    b.msg.zero_()
    b.decode()
    torch.cuda.synchronize()
    got = b.msg.cpu().numpy().view(np.uint8).reshape(P, -1)[:, :msg_bytes]
    assert np.array_equal(got, msgs) and not b.status.cpu().numpy().any()


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
def test_segmented_mixed_shapes_offsets_and_invalid_descriptors(gpu_device, seg_mode):
    import torch

    rng = np.random.default_rng(7)
    P = 400
    shapes = [(int(rng.integers(1, 2100)), int(rng.integers(1, 9))) for _ in range(P)]
    shapes = [(mb, min(t, 8 * mb)) for mb, t in shapes]
    d = np.zeros(P, dtype=hm.seg_packet_dtype())
    enc_off = msg_off = seg_off = 0
    rows, refs = [], []
    for q, (mb, t) in enumerate(shapes):
        enc = _received(synth.workload_seed("gpu-seg-mix", q), 1, mb, t, None, 0.5, 0.25)[0]
        ew = (enc.size + 7) // 8
        d[q] = (enc_off, msg_off, mb, t, seg_off)
        rows.append((enc_off, enc))
        refs.append(oracle.seg_decode(enc, mb, t))
        enc_off += ew + int(rng.integers(0, 3))             # gaps between packets
        msg_off += (mb + 7) // 8 + int(rng.integers(0, 2))
        seg_off += t + int(rng.integers(0, 2))
    bad = {5: dict(t=0), 17: dict(t=33), 29: dict(msg_bytes=0), 41: dict(msg_bytes=2101),
           53: dict(enc_word_off=enc_off + 10), 65: dict(msg_word_off=msg_off), 77: dict(seg_off=seg_off),
           89: dict(t=9, msg_bytes=1)}
    for q, kv in bad.items():
        for f, v in kv.items():
            d[q][f] = v
    arena = np.zeros(enc_off + 1, dtype=np.uint64)
    for off, enc in rows:
        w = np.zeros((enc.size + 7) // 8 * 8, dtype=np.uint8)
        w[:enc.size] = enc
        arena[off:off + w.size // 8] = w.view(np.uint64)
    dev = gpu_device
    enc_t = torch.from_numpy(arena.view(np.int64)).to(dev)
    msg_t = torch.full((msg_off,), 0x3C3C3C3C3C3C3C3C, dtype=torch.int64, device=dev)
    syn_t = torch.full((seg_off,), 0x7777, dtype=torch.int16, device=dev)
    st_t = torch.zeros(P, dtype=torch.uint8, device=dev)
    desc_t = torch.from_numpy(d.view(np.uint8)).to(dev)
    hm.hamming_decode_segmented(enc_t, enc_t.numel(), desc_t, P, 2100, msg_t, msg_t.numel(), syn_t, syn_t.numel(),
                                st_t)
    torch.cuda.synchronize()
    msg = msg_t.cpu().numpy().view(np.uint8)
    syn = syn_t.cpu().numpy().view(np.uint16)
    st = st_t.cpu().numpy()
    written_msg = np.zeros(msg.size, dtype=bool)
    written_syn = np.zeros(syn.size, dtype=bool)
    for q, (mb, t) in enumerate(shapes):
        mo, so = int(d[q]["msg_word_off"]) * 8, int(d[q]["seg_off"])
        if q in bad:
            assert st[q] == hm.HAMMING_SEG_INVALID
            continue
        m_ref, s_ref, st_ref = refs[q]
        assert np.array_equal(msg[mo:mo + mb], m_ref), q
        assert not msg[mo + mb:mo + (mb + 7) // 8 * 8].any()
        assert np.array_equal(syn[so:so + t], s_ref) and st[q] == st_ref
        written_msg[mo:mo + (mb + 7) // 8 * 8] = True
        written_syn[so:so + t] = True
    assert (msg[~written_msg] == 0x3C).all()          # gaps and rejected packets untouched
    assert (syn[~written_syn] == 0x7777).all()


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
def test_segmented_encoder_mixed_shapes_offsets_and_invalid_descriptors(gpu_device, seg_mode):
    """The encoder on packets of mixed shapes at scattered offsets: each valid
    packet's encoded words equal the oracle's (tail bits 0), and the words
    between packets and those of rejected descriptors are left as they were."""
    import torch

    rng = np.random.default_rng(8)
    P = 300
    shapes = [(int(rng.integers(1, 2100)), int(rng.integers(1, 9))) for _ in range(P)]
    shapes = [(mb, min(t, 8 * mb)) for mb, t in shapes]
    d = np.zeros(P, dtype=hm.seg_packet_dtype())
    enc_off = msg_off = 0
    msgs = []
    for q, (mb, t) in enumerate(shapes):
        ew = (oracle.seg_layout(mb, t)[3] + 63) // 64
        d[q] = (enc_off, msg_off, mb, t, 0)
        msgs.append(synth.packet_bytes(synth.workload_seed("gpu-seg-enc-mix", q), 1, mb)[0])
        enc_off += ew + int(rng.integers(0, 3))
        msg_off += (mb + 7) // 8 + int(rng.integers(0, 2))
    bad = {3: dict(t=0), 11: dict(t=33), 19: dict(msg_bytes=0), 27: dict(msg_bytes=2101),
           35: dict(enc_word_off=enc_off + 10), 43: dict(msg_word_off=msg_off), 51: dict(t=9, msg_bytes=1)}
    for q, kv in bad.items():
        for f, v in kv.items():
            d[q][f] = v
    marena = np.frombuffer(rng.integers(0, 256, msg_off * 8, dtype=np.uint8).tobytes(), dtype=np.uint8).copy()
    for q, (mb, t) in enumerate(shapes):
        if q not in bad:
            mo = int(d[q]["msg_word_off"]) * 8
            marena[mo:mo + mb] = msgs[q]                    # bytes past M stay random: they are ignored
    dev = gpu_device
    msg_t = torch.from_numpy(marena.view(np.int64).copy()).to(dev)
    enc_t = torch.full((enc_off,), 0x5A5A5A5A5A5A5A5A, dtype=torch.int64, device=dev)
    desc_t = torch.from_numpy(d.view(np.uint8)).to(dev)
    hm.hamming_encode_segmented(msg_t, msg_t.numel(), desc_t, P, 2100, enc_t, enc_t.numel())
    torch.cuda.synchronize()
    enc = enc_t.cpu().numpy().view(np.uint8)
    written = np.zeros(enc.size, dtype=bool)
    for q, (mb, t) in enumerate(shapes):
        if q in bad:
            continue
        eo = int(d[q]["enc_word_off"]) * 8
        nbytes = (oracle.seg_layout(mb, t)[3] + 63) // 64 * 8
        want = np.zeros(nbytes, dtype=np.uint8)
        ref = oracle.seg_encode(msgs[q], t)
        want[:ref.size] = ref
        assert np.array_equal(enc[eo:eo + nbytes], want), q
        written[eo:eo + nbytes] = True
    assert (enc[~written] == 0x5A).all()


# segments that end at each boundary of a 128-position window (n mod 128 = 62, 63, 127, 1, 64, 126):
# the masks of a window's upper and lower halves switch there
WINDOW_EDGE_SHAPES = [(56, 8), (57, 8), (120, 8), (121, 8), (184, 8), (123, 4)]


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
@pytest.mark.parametrize("msg_bytes,t", WINDOW_EDGE_SHAPES)
def test_segmented_segments_ending_at_window_boundaries(gpu_device, seg_mode, msg_bytes, t):
    import torch

    P = 700
    n = oracle.seg_layout(msg_bytes, t)[2]
    assert len({x % 128 for x in n}) == 1
    b = hm.SegmentedBatch(P, msg_bytes, t, device=gpu_device)
    seed = synth.workload_seed("gpu-seg-edge", msg_bytes, t)
    msgs = synth.packet_bytes(seed, P, msg_bytes)
    clean = oracle.seg_encode_many(msgs, t, row_bytes=b.enc_stride * 8)
    enc = _received(seed, P, msg_bytes, t, b.enc_stride * 8, 0.4, 0.2)
    b.enc.copy_(torch.from_numpy(np.ascontiguousarray(enc).reshape(-1).view(np.int64)).to(gpu_device))
    b.decode()
    torch.cuda.synchronize()
    m_ref, s_ref, st_ref = oracle.seg_decode_many(enc, msg_bytes, t)
    got = b.msg.cpu().numpy().view(np.uint8).reshape(P, -1)[:, :msg_bytes]
    assert np.array_equal(got, m_ref)
    assert np.array_equal(b.syndromes.cpu().numpy().view(np.uint16).reshape(P, t), s_ref)
    assert np.array_equal(b.status.cpu().numpy(), st_ref)
    rows = np.zeros((P, b.msg_stride * 8), dtype=np.uint8)
    rows[:, :msg_bytes] = msgs
    b.msg.copy_(torch.from_numpy(rows.reshape(-1).view(np.int64)).to(gpu_device))
    b.encode()
    torch.cuda.synchronize()
    assert np.array_equal(b.enc.cpu().numpy().view(np.uint8).reshape(P, -1), clean)


def _long_segment_edge_shapes():
    """(M, t) shapes whose segments all have at least 256 positions and end
    at given places of their last 128-position window: n mod 128 = 0 (a last
    window of one position), 1, 2, 63, 64, 65, 126, 127; first found, M in
    32..800."""
    found = {}
    for M in range(32, 801):
        for t in range(1, 7):
            if 8 * M < t:
                continue
            n = oracle.seg_layout(M, t)[2]
            if min(n) < 256:
                continue
            for x in n:
                if x % 128 in (0, 1, 2, 63, 64, 65, 126, 127) and x % 128 not in found:
                    found[x % 128] = (M, t)
    assert len(found) == 8, found
    return sorted(set(found.values()))


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
@pytest.mark.parametrize("msg_bytes,t", _long_segment_edge_shapes())
def test_segmented_long_segments_ending_at_window_boundaries(gpu_device, seg_mode, msg_bytes, t):
    # a short last window of a long segment, followed by the next segment's
    # window 0, in every group size
    _check_batch(gpu_device, 257, msg_bytes, t, p_single=0.5, p_double=0.2)


def _message_boundary_shapes():
    """(M, t) shapes whose segments carry at least 128 message bits, chosen
    so that the segment boundaries K_j mod 64 (where a segment's message run
    starts in the merged message words) and the packet end 8M mod 64 take the
    values 0 (a word start), 1, 7, 8, 56, 57 (the 57 head bits end on a word
    boundary) and 63; plus 128-bit segments (also with t = 32), 127-bit ones
    and single-segment packets."""
    want = {0, 1, 7, 8, 56, 57, 63}
    found_k, found_end = {}, {}
    for M in range(16, 700):
        for t in range(2, 7):
            k = oracle.seg_layout(M, t)[0]
            if min(k) < 128:
                continue
            K = np.cumsum(k)[:-1]
            for x in K % 64:
                if x in want and x not in found_k:
                    found_k[int(x)] = (M, t)
            e = (8 * M) % 64
            if e in want and e not in found_end:
                found_end[e] = (M, t)
    assert set(found_k) == want and set(found_end) == {0, 8, 56}, (found_k, found_end)
    extra = [(512, 32), (16, 1), (400, 1), (4096, 32), (508, 32), (160, 10), (159, 10)]
    return sorted(set(found_k.values()) | set(found_end.values()) | set(extra))


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
@pytest.mark.parametrize("msg_bytes,t", _message_boundary_shapes())
def test_segmented_segment_boundaries_at_every_word_offset(gpu_device, seg_mode, msg_bytes, t):
    _check_batch(gpu_device, 131, msg_bytes, t, p_single=0.5, p_double=0.2)


@pytest.mark.parametrize("seg_mode", [8, 16, 256], indirect=True)
@pytest.mark.parametrize("msg_bytes,t", [(200, 3), (40, 2), (33, 2)])
def test_segmented_every_single_error_position(gpu_device, seg_mode, msg_bytes, t):
    """Packet i carries one flip at stream bit i, for every bit of the packet:
    each position of each segment (checksum positions, head positions, the
    last position) is corrected or reported exactly as the oracle does."""
    import torch

    _, _, n, bits = oracle.seg_layout(msg_bytes, t)
    P = int(bits)
    b = hm.SegmentedBatch(P, msg_bytes, t, device=gpu_device)
    seed = synth.workload_seed("gpu-seg-every-position", msg_bytes, t)
    msgs = synth.packet_bytes(seed, P, msg_bytes)
    enc = oracle.seg_encode_many(msgs, t, row_bytes=b.enc_stride * 8)
    rows = np.arange(P)
    enc[rows, rows // 8] ^= (1 << (rows % 8)).astype(np.uint8)
    b.enc.copy_(torch.from_numpy(np.ascontiguousarray(enc).reshape(-1).view(np.int64)).to(gpu_device))
    b.decode()
    torch.cuda.synchronize()
    m_ref, s_ref, st_ref = oracle.seg_decode_many(enc, msg_bytes, t)
    assert np.array_equal(m_ref, msgs)          # every single flip is corrected
    got = b.msg.cpu().numpy().view(np.uint8).reshape(P, -1)[:, :msg_bytes]
    assert np.array_equal(got, m_ref)
    assert np.array_equal(b.syndromes.cpu().numpy().view(np.uint16).reshape(P, t), s_ref)
    assert np.array_equal(b.status.cpu().numpy(), st_ref)


@pytest.mark.parametrize("seg_mode", MODES, indirect=True)
def test_segmented_max_msg_bytes_bound_rejects_longer_packets(gpu_device, seg_mode):
    import torch

    b = hm.SegmentedBatch(8, 800, 3, device=gpu_device)
    b.status.zero_()
    hm.hamming_decode_segmented(b.enc, b.enc.numel(), b.descs, 8, 799, b.msg, b.msg.numel(), b.syndromes,
                                b.syndromes.numel(), b.status)
    torch.cuda.synchronize()
    assert (b.status.cpu().numpy() == hm.HAMMING_SEG_INVALID).all()


@pytest.mark.parametrize("P,mb,t", [(1 << 20, 1500, 4), (1 << 19, 400, 6), (1 << 19, 800, 3), (1 << 19, 1200, 4),
                                    (1 << 19, 2000, 6)])
def test_segmented_full_size_sampled(gpu_device, P, mb, t):
    """Full-size batches in the library's own launch choice (the Table 1 grid
    is decoded with 2^19 packets per shape: 400 and 800 bytes take 8 threads
    per packet, 1200 and 2000 bytes 16, with two or four windows loaded ahead),
    encoded on the GPU; a sample of packets is checked against the oracle one
    by one."""
    import torch

    assert hm.hamming_seg_config_get() == 0
    b = hm.SegmentedBatch(P, mb, t, device=gpu_device)
    seed = synth.workload_seed("gpu-seg-full", mb, t)
    w = synth.draws_torch(seed, 0, P * b.msg_stride, gpu_device)
    b.msg.copy_(w)
    b.encode()
    enc_clean = b.enc.clone()
    _, _, n, _ = oracle.seg_layout(mb, t)
    starts = np.concatenate([[0], np.cumsum(n)[:-1]])
    b1, b2 = synth.segment_flips(seed, P, starts, n, 0.3, 0.1)
    base = (np.arange(P, dtype=np.int64) * b.enc_stride * 64)[:, None]
    flips = np.concatenate([(b1 + base)[b1 >= 0], (b2 + base)[b2 >= 0]])
    bits = torch.from_numpy(flips).to(gpu_device)
    mask = torch.zeros_like(b.enc).scatter_add_(0, bits // 64, torch.bitwise_left_shift(torch.ones_like(bits),
                                                                                          bits % 64))
    b.enc ^= mask
    b.decode()
    torch.cuda.synchronize()
    sample = np.unique(np.concatenate([np.arange(0, P, 9973), [P - 1]]))
    enc = b.enc.view(P, b.enc_stride)[sample].cpu().numpy().view(np.uint8)
    msg = b.msg.view(P, b.msg_stride)[sample].cpu().numpy().view(np.uint8)
    syn = b.syndromes.view(P, t)[sample].cpu().numpy().view(np.uint16)
    st = b.status[sample].cpu().numpy()
    clean = enc_clean.view(P, b.enc_stride)[sample].cpu().numpy().view(np.uint8)
    sent = w.view(P, b.msg_stride)[sample].cpu().numpy().view(np.uint8)[:, :mb]
    assert np.array_equal(oracle.seg_encode_many(sent, t, row_bytes=b.enc_stride * 8), clean)
    m_ref, s_ref, st_ref = oracle.seg_decode_many(enc, mb, t)
    assert np.array_equal(msg[:, :mb], m_ref) and np.array_equal(syn, s_ref) and np.array_equal(st, st_ref)
    # single-flip packets decode to what was sent
    one = (st_ref == 1) & ((b2[sample] < 0).all(axis=1))
    assert one.any() and np.array_equal(msg[one, :mb], sent[one])

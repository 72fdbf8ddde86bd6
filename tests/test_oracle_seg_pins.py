"""Pins of the segmented-packet oracle (the paper's t-segment workload,
Sec. II, Fig. 1; shortened segments as in the worked example of Sec. III.A).

The oracle is checked against things it does not compute itself:
  * the paper's worked example: an 11-bit segment carries 4 checksum bits
    and the index sets the paper prints;
  * the code's definition and bounded-distance decoding by brute force: for
    small segments the whole codebook is enumerated from the parity-check
    matrix (column p = binary expansion of p) and every received word is
    decoded by searching for a codeword within Hamming distance 1;
  * reduction to the plain decoder: when every segment is a perfect code
    the packet decode equals the (separately pinned) plain oracle;
  * closed forms: one flip is corrected with syndrome = its position, two
    flips at a and b give syndrome a XOR b.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bits(v: int, n: int) -> list[int]:
    return [(v >> q) & 1 for q in range(n)]


def _syndrome_by_definition(word_bits) -> int:
    """H y over GF(2) with column p of H equal to the binary expansion of p."""
    s = 0
    for q, b in enumerate(word_bits):
        if b:
            s ^= q + 1
    return s


def _codebook(n: int) -> np.ndarray:
    """All n-bit words (bit p-1 = position p) in the null space of H."""
    words = np.arange(1 << n, dtype=np.int64)
    syn = np.zeros_like(words)
    for q in range(n):
        syn ^= np.where((words >> q) & 1, q + 1, 0)
    return words[syn == 0]


def _message_of(word: int, n: int) -> list[int]:
    return [(word >> (p - 1)) & 1 for p in range(1, n + 1) if p & (p - 1)]


def _bounded_distance(y: int, book: np.ndarray, n: int):
    """(corrected word, status) by exhaustive search of the codebook."""
    d = np.array([bin(int(c) ^ y).count("1") for c in book])
    near = book[d <= 1]
    assert near.size <= 1            # minimum distance 3: at most one codeword within distance 1
    if near.size == 0:
        return y, 2
    return int(near[0]), int(d[d <= 1][0])


def test_layout_of_the_papers_example_segment():
    k, r, n, total = oracle.seg_layout(7, 8)
    assert n == [11] * 8 and r == [4] * 8 and k == [7] * 8 and total == 88
    rows = [[int(v) for v in l.split()] for l in open(os.path.join(GOLDEN, "paper_index_sets.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for nn, j, *pos in rows:
        assert nn == 11 and oracle.index_set(11, j) == pos


@pytest.mark.parametrize("msg_bytes", [1, 2, 3, 50, 400, 777, 2000, 8000])
@pytest.mark.parametrize("t", [1, 2, 3, 5, 6, 7, 32])
def test_layout_rule(msg_bytes, t):
    if 8 * msg_bytes < t or (8 * msg_bytes + t - 1) // t > 65519:
        with pytest.raises(ValueError):
            oracle.seg_layout(msg_bytes, t)
        return
    k, r, n, total = oracle.seg_layout(msg_bytes, t)
    assert sum(k) == 8 * msg_bytes
    assert max(k) - min(k) <= 1 and k == sorted(k, reverse=True)
    for ki, ri, ni in zip(k, r, n):
        assert ni == ki + ri and ri >= 2
        assert (1 << ri) - 1 - ri >= ki                      # enough checksum bits
        assert ri == 2 or (1 << (ri - 1)) - ri < ki           # and no more than needed
    assert total == sum(n)


def test_layout_rejects_unsupported_shapes():
    for mb, t in ((0, 1), (1, 9), (1, 0), (10, 33), (8190, 1)):
        with pytest.raises(ValueError):
            oracle.seg_layout(mb, t)


@pytest.mark.parametrize("n", [3, 5, 6, 7, 11, 12])
def test_codebook_dimension_and_distance(n):
    book = _codebook(n)
    r = max(j for j in range(1, 6) if (1 << j) <= n) + 1
    assert book.size == 1 << (n - r)
    nz = book[book != 0]
    assert min(bin(int(c)).count("1") for c in nz) == 3


@pytest.mark.parametrize("msg_bytes,t", [(1, 1), (1, 2), (1, 3)])
def test_every_received_packet_against_brute_force(msg_bytes, t):
    """Every possible received packet of a short shape: each segment decoded
    to the unique codeword within distance 1, else detected-uncorrectable."""
    k, r, n, total = oracle.seg_layout(msg_bytes, t)
    books = {ni: _codebook(ni) for ni in set(n)}
    count = 1 << total
    rows = np.zeros((count, (total + 7) // 8), dtype=np.uint8)
    for b in range((total + 7) // 8):
        rows[:, b] = (np.arange(count) >> (8 * b)) & 0xFF
    msg, syn, st = oracle.seg_decode_many(rows, msg_bytes, t)
    # exhaustive per-segment answer: one table per segment length
    table = {}
    for ni, book in books.items():
        corr = np.zeros(1 << ni, dtype=np.int64)
        stat = np.zeros(1 << ni, dtype=np.int64)
        for y in range(1 << ni):
            corr[y], stat[y] = _bounded_distance(y, book, ni)
        table[ni] = (corr, stat)
    idx = np.arange(count)
    off = 0
    K = 0
    msg_bits = np.unpackbits(msg, axis=1, bitorder="little")
    status = np.zeros(count, dtype=np.int64)
    for i in range(t):
        y = (idx >> off) & ((1 << n[i]) - 1)
        corr, stat = table[n[i]]
        want = corr[y]
        status = np.maximum(status, stat[y])
        # message bits of the corrected (or, if uncorrectable, received) word
        mpos = [p for p in range(1, n[i] + 1) if p & (p - 1)]
        for m, p in enumerate(mpos):
            assert np.array_equal(msg_bits[:, K + m], (want >> (p - 1)) & 1)
        # syndrome: 0 for codewords, the flipped position for distance 1
        flipped = want ^ y
        pos = np.where(flipped > 0, np.log2(np.maximum(flipped, 1)).astype(np.int64) + 1, 0)
        ok = stat[y] < 2
        assert np.array_equal(syn[ok, i], pos[ok])
        assert (syn[~ok, i] > n[i]).all()
        off += n[i]
        K += k[i]
    assert np.array_equal(st, status)


def test_papers_eleven_bit_segments_against_brute_force():
    """Eight (11,7) segments (the worked example's code), 0..3 flips each."""
    msg_bytes, t = 7, 8
    k, r, n, total = oracle.seg_layout(msg_bytes, t)
    book = _codebook(11)
    P = 3000
    rng = np.random.default_rng(11)
    msgs = rng.integers(0, 256, (P, msg_bytes), dtype=np.uint8)
    enc = oracle.seg_encode_many(msgs, t)
    flips = np.zeros((P, t), dtype=np.int64)
    for q in range(P):
        for i in range(t):
            cnt = rng.integers(0, 4)
            for p in rng.choice(11, cnt, replace=False):
                flips[q, i] |= 1 << int(p)
    ybits = np.unpackbits(enc, axis=1, bitorder="little")[:, :total].copy()
    for i in range(t):
        for q in range(11):
            ybits[:, 11 * i + q] ^= ((flips[:, i] >> q) & 1).astype(np.uint8)
    y = np.packbits(ybits, axis=1, bitorder="little")
    msg, syn, st = oracle.seg_decode_many(y, msg_bytes, t)
    mbits = np.unpackbits(msg, axis=1, bitorder="little")
    for q in range(0, P, 7):
        worst = 0
        for i in range(t):
            yi = int(sum(int(ybits[q, 11 * i + b]) << b for b in range(11)))
            c, s = _bounded_distance(yi, book, 11)
            worst = max(worst, s)
            assert list(mbits[q, 7 * i:7 * i + 7]) == _message_of(c, 11)
            if s < 2:
                assert syn[q, i] == (0 if c == yi else (c ^ yi).bit_length())
            else:
                assert syn[q, i] > 11
        assert st[q] == worst


def test_encoder_output_is_in_the_code_and_carries_the_message():
    rng = np.random.default_rng(5)
    for msg_bytes, t in ((1, 3), (7, 8), (400, 6), (2000, 2), (13, 1)):
        msg = rng.integers(0, 256, msg_bytes, dtype=np.uint8)
        enc = oracle.seg_encode(msg, t)
        k, r, n, total = oracle.seg_layout(msg_bytes, t)
        bits = np.unpackbits(enc, bitorder="little")
        assert not bits[total:].any()
        mbits = np.unpackbits(msg, bitorder="little")
        off = K = 0
        for i in range(t):
            seg = [int(b) for b in bits[off:off + n[i]]]
            assert _syndrome_by_definition(seg) == 0
            data = [seg[p - 1] for p in range(1, n[i] + 1) if p & (p - 1)]
            assert data == list(mbits[K:K + k[i]])
            off += n[i]
            K += k[i]


# shapes whose segments are all perfect codes: (msg_bytes, t, r)
PERFECT = [(1, 2, 3), (11, 8, 4), (13, 4, 5), (57, 8, 6), (15, 1, 7), (120, 8, 7)]


@pytest.mark.parametrize("msg_bytes,t,r", PERFECT)
def test_perfect_code_shapes_equal_the_plain_decoder(msg_bytes, t, r):
    n_code = (1 << r) - 1
    k, rr, n, total = oracle.seg_layout(msg_bytes, t)
    assert rr == [r] * t and n == [n_code] * t
    P = 500
    seed = synth.workload_seed("seg-perfect", r, t)
    msgs = synth.packet_bytes(seed, P, msg_bytes)
    enc = oracle.seg_encode_many(msgs, t)
    ranges = [(i * n_code, n_code) for i in range(t)]
    b1, b2 = synth.segment_flips(seed, P, [a for a, _ in ranges], [b for _, b in ranges], 0.4, 0.2)
    synth.apply_bit_flips(enc, b1, b2)
    msg, syn, st = oracle.seg_decode_many(enc, msg_bytes, t)
    # the same received words in the plain decoder's storage layout
    bits = np.unpackbits(enc, axis=1, bitorder="little")[:, :total].reshape(P * t, n_code)
    wpc = 2 if r == 7 else 1
    store = np.zeros((P * t, 64 * wpc), dtype=np.uint8)
    store[:, :n_code] = bits
    words = np.packbits(store, axis=1, bitorder="little").view(np.uint64).reshape(-1)
    data, errpos = oracle.decode(words, r)
    plain_bits = np.unpackbits(data, bitorder="little")[:P * t * k[0]].reshape(P, 8 * msg_bytes)
    assert np.array_equal(np.unpackbits(msg, axis=1, bitorder="little"), plain_bits)
    assert np.array_equal(syn.reshape(-1), errpos.astype(np.uint16))
    assert np.array_equal(st, np.where((errpos.reshape(P, t) > 0).any(axis=1), 1, 0))


@pytest.mark.parametrize("msg_bytes", synth.PAPER_PACKET_BYTES)
@pytest.mark.parametrize("t", synth.PAPER_SEGMENTS)
def test_round_trips_at_the_papers_packet_sizes(msg_bytes, t):
    k, r, n, total = oracle.seg_layout(msg_bytes, t)
    starts = np.concatenate([[0], np.cumsum(n)[:-1]])
    P = 40
    seed = synth.workload_seed("seg-roundtrip", msg_bytes, t)
    msgs = synth.packet_bytes(seed, P, msg_bytes)
    enc = oracle.seg_encode_many(msgs, t)
    msg, syn, st = oracle.seg_decode_many(enc, msg_bytes, t)
    assert np.array_equal(msg, msgs) and not syn.any() and not st.any()
    # one flip per segment: corrected, syndrome = position
    b1, _ = synth.segment_flips(seed, P, starts, n, 1.0)
    one = enc.copy()
    synth.apply_bit_flips(one, b1)
    msg, syn, st = oracle.seg_decode_many(one, msg_bytes, t)
    assert np.array_equal(msg, msgs) and (st == 1).all()
    assert np.array_equal(syn, (b1 - starts + 1).astype(np.uint16))
    # two flips per segment: syndrome = a XOR b, uncorrectable iff beyond n_i
    b1, b2 = synth.segment_flips(seed + 1, P, starts, n, 0.0, 1.0)
    two = enc.copy()
    synth.apply_bit_flips(two, b1, b2)
    msg, syn, st = oracle.seg_decode_many(two, msg_bytes, t)
    s_expect = (b1 - starts + 1) ^ (b2 - starts + 1)
    assert np.array_equal(syn, s_expect.astype(np.uint16))
    beyond = s_expect > np.asarray(n)
    assert np.array_equal(st, np.where(beyond.any(axis=1), 2, 1))

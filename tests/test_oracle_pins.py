"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or the mathematics
fixes: the index sets printed in Sec. III.A, a Hamming(7,4) codeword worked by
hand from Hamming's construction, brute-force nearest-codeword decoding over
every received word of the (7,4) and (15,11) codes (codewords enumerated from
the parity-check definition, not from the oracle), the sphere invariant of a
perfect code, linearity of the checksum, the closed form of a two-bit
miscorrection and the layout of the merged message stream.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _unpack_stream(stream: np.ndarray, n_cw: int, k: int) -> np.ndarray:
    """Messages (n_cw, k) of bits from a dense LSB-first stream."""
    bits = np.unpackbits(stream.view(np.uint8), bitorder="little")
    return bits[: n_cw * k].reshape(n_cw, k)


def _positions_bits(words: np.ndarray, r: int) -> np.ndarray:
    """(n_cw, n) array of bits at positions 1..n from storage words."""
    n, _, wpc = synth.code_sizes(r)
    w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, wpc)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(w.shape[0], 64 * wpc)
    return bits[:, :n]


def _message_positions(n):
    return [p for p in range(1, n + 1) if p & (p - 1)]


# --- the paper's printed index sets --------------------------------------

def test_index_sets_match_paper():
    rows = _read_golden("paper_index_sets.txt")
    assert len(rows) == 4
    for row in rows:
        n, j, *pos = (int(v) for v in row)
        assert oracle.index_set(n, j) == pos


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_index_set_sizes_closed_form(r):
    # every index set of a (2^r - 1)-bit word holds 2^(r-1) positions, and
    # position p lies in exactly popcount(p) of the sets
    n = (1 << r) - 1
    sets = [oracle.index_set(n, j) for j in range(r)]
    assert all(len(s) == 1 << (r - 1) for s in sets)
    for p in range(1, n + 1):
        assert sum(p in s for s in sets) == bin(p).count("1")


# --- textbook Hamming(7,4) -------------------------------------------------

def test_textbook_hamming74():
    for kind, r, msg, word, *rest in _read_golden("hamming74_textbook.txt"):
        r, msg, word = int(r), int(msg, 16), int(word, 16)
        if kind == "encode":
            cw = oracle.encode(np.array([msg], dtype=np.uint8), 1, r)
            assert int(cw[0]) == word
        else:
            data, errpos = oracle.decode(np.array([word], dtype=np.uint64), r)
            assert int(data[0]) == msg and int(errpos[0]) == int(rest[0])
            assert data.size == 8 and not data[1:].any()


# --- encoder against the parity-check definition ----------------------------

def _check_codeword_definition(cw_words, stream, n_cw, r):
    n, k, wpc = synth.code_sizes(r)
    bits = _positions_bits(cw_words, r)
    pos = np.arange(1, n + 1, dtype=np.int64)
    # H has binary(p) as column p: a codeword's set positions XOR to zero
    xor = np.bitwise_xor.reduce(np.where(bits.astype(bool), pos, 0), axis=1)
    assert not xor.any()
    # message bits sit at the non-power-of-two positions, in order
    msg = _unpack_stream(stream, n_cw, k)
    mp = np.array(_message_positions(n)) - 1
    assert np.array_equal(bits[:, mp], msg)
    # storage padding stays clear
    full = np.unpackbits(np.ascontiguousarray(cw_words).view(np.uint8), bitorder="little")
    assert not full.reshape(n_cw, 64 * wpc)[:, n:].any()


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_encoder_satisfies_parity_check_definition(r):
    n_cw = 3000
    stream = synth.message_stream(synth.workload_seed("enc-pin", r), n_cw, r)
    cw = oracle.encode(stream, n_cw, r)
    _check_codeword_definition(cw, stream, n_cw, r)


# --- brute-force maximum-likelihood decoding --------------------------------

def _all_codewords_by_definition(r):
    """All words of length n whose set positions XOR to zero."""
    n = (1 << r) - 1
    words = np.arange(1 << n, dtype=np.int64)
    xor = np.zeros_like(words)
    for p in range(1, n + 1):
        xor ^= np.where((words >> (p - 1)) & 1, p, 0)
    return words[xor == 0]


@pytest.mark.parametrize("r", [3, 4])
def test_bruteforce_nearest_codeword_all_received_words(r):
    n, k, _ = synth.code_sizes(r)
    code = _all_codewords_by_definition(r)
    assert code.size == 1 << k
    received = np.arange(1 << n, dtype=np.int64)
    dist = np.bitwise_count((received[:, None] ^ code[None, :]).astype(np.uint64))
    best = np.argmin(dist, axis=1)
    dmin = dist[np.arange(received.size), best]
    assert dmin.max() <= 1
    assert ((dist == dmin[:, None]).sum(axis=1) == 1).all()   # unique (perfect code)
    nearest = code[best]
    diff = received ^ nearest
    exp_errpos = np.where(diff == 0, 0, np.log2(np.maximum(diff, 1)).astype(np.int64) + 1)
    mp = np.array(_message_positions(n)) - 1
    exp_msg = (nearest[:, None] >> mp[None, :]) & 1

    data, errpos = oracle.decode(received.astype(np.uint64), r)
    assert np.array_equal(errpos.astype(np.int64), exp_errpos)
    assert np.array_equal(_unpack_stream(data, received.size, k), exp_msg)


@pytest.mark.parametrize("r", [3, 4])
def test_every_single_error_every_message(r):
    n, k, _ = synth.code_sizes(r)
    msgs = np.arange(1 << k, dtype=np.uint64)
    stream = np.packbits(((msgs[:, None] >> np.arange(k, dtype=np.uint64)) & np.uint64(1))
                         .astype(np.uint8).reshape(-1), bitorder="little")
    cw = oracle.encode(stream, msgs.size, r)
    for p in range(0, n + 1):
        y = cw ^ (np.uint64(1 << (p - 1)) if p else np.uint64(0))
        data, errpos = oracle.decode(y, r)
        assert (errpos == p).all()
        assert np.array_equal(_unpack_stream(data, msgs.size, k),
                              _unpack_stream(stream, msgs.size, k))


@pytest.mark.parametrize("r", [3, 4])
def test_zero_checksum_every_codeword(r):
    code = _all_codewords_by_definition(r).astype(np.uint64)
    _, errpos = oracle.decode(code, r)
    assert not errpos.any()


def test_zero_checksum_random_codewords_r5_r6_r7():
    for r in (5, 6, 7):
        n_cw = 1 << 16
        stream = synth.message_stream(synth.workload_seed("zero-syn", r), n_cw, r)
        cw = oracle.encode(stream, n_cw, r)
        data, errpos = oracle.decode(cw, r)
        assert not errpos.any()
        assert np.array_equal(data[: stream.nbytes], stream.view(np.uint8))


# --- invariants at every r ---------------------------------------------------

@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_sphere_invariant_random_received_words(r):
    """For a perfect code the decoded message is the one whose codeword lies
    within distance 1 of the received word, and errpos names the differing
    position: both follow from the encoder (pinned above) alone."""
    n, k, wpc = synth.code_sizes(r)
    n_cw = 4096
    seed = synth.workload_seed("sphere", r)
    y = synth.draws(seed, 0, n_cw * wpc)          # arbitrary received words, garbage padding
    data, errpos = oracle.decode(y, r)
    re = oracle.encode(data, n_cw, r)
    yb = _positions_bits(y, r)
    cb = _positions_bits(re, r)
    diff = yb ^ cb
    assert (diff.sum(axis=1) <= 1).all()
    where = np.where(diff.any(axis=1), diff.argmax(axis=1) + 1, 0)
    assert np.array_equal(where, errpos.astype(np.int64))


@pytest.mark.parametrize("r", [5, 6, 7])
def test_checksum_is_linear(r):
    n, _, wpc = synth.code_sizes(r)
    n_cw = 2048
    a = synth.draws(synth.workload_seed("lin-a", r), 0, n_cw * wpc)
    b = synth.draws(synth.workload_seed("lin-b", r), 0, n_cw * wpc)
    _, sa = oracle.decode(a, r)
    _, sb = oracle.decode(b, r)
    _, sab = oracle.decode(a ^ b, r)
    assert np.array_equal(sab, sa ^ sb)


@pytest.mark.parametrize("r", [4, 5, 6, 7])
def test_double_error_closed_form(r):
    """Two flips at a != b give checksum a xor b; the decoder then flips
    position a xor b as well, landing on another codeword."""
    n, k, wpc = synth.code_sizes(r)
    n_cw = 2048
    seed = synth.workload_seed("double", r)
    stream = synth.message_stream(seed, n_cw, r)
    cw = oracle.encode(stream, n_cw, r)
    p1, p2 = synth.error_positions(seed, n_cw, r, p_single=0.0, p_double=1.0)
    assert (p1 > 0).all() and (p2 > 0).all() and (p1 != p2).all()
    y = cw ^ synth.flip_masks(p1, p2, r)
    data, errpos = oracle.decode(y, r)
    s = p1.astype(np.int64) ^ p2.astype(np.int64)
    assert np.array_equal(errpos.astype(np.int64), s)
    # expected output: the message bits of y with position s flipped as well
    bits = _positions_bits(y, r).copy()
    bits[np.arange(n_cw), s - 1] ^= 1
    mp = np.array(_message_positions(n)) - 1
    assert np.array_equal(_unpack_stream(data, n_cw, k), bits[:, mp])


# --- the merged stream --------------------------------------------------------

@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("n_cw", [1, 5, 63, 64, 65, 129])
def test_merge_layout_and_zero_tail(r, n_cw):
    n, k, wpc = synth.code_sizes(r)
    seed = synth.workload_seed("merge", r, n_cw)
    y = synth.draws(seed, 0, n_cw * wpc)
    data, errpos = oracle.decode(y, r)
    assert data.size == ((n_cw * k + 63) // 64) * 8
    bits = np.unpackbits(data, bitorder="little")
    assert not bits[n_cw * k:].any()
    for i in range(n_cw):
        d1, e1 = oracle.decode(y[i * wpc:(i + 1) * wpc], r)
        assert np.array_equal(bits[i * k:(i + 1) * k], np.unpackbits(d1, bitorder="little")[:k])
        assert e1[0] == errpos[i]


@pytest.mark.parametrize("r", [3, 5, 6, 7])
def test_padding_bits_are_ignored(r):
    n, _, wpc = synth.code_sizes(r)
    n_cw = 1000
    seed = synth.workload_seed("pad", r)
    y = synth.draws(seed, 0, n_cw * wpc)
    valid = [(1 << min(64, max(0, n - 64 * w))) - 1 for w in range(wpc)]
    clean = y.reshape(n_cw, wpc).copy()
    for w in range(wpc):
        clean[:, w] &= np.uint64(valid[w])
    assert np.array_equal(oracle.decode(y, r)[0], oracle.decode(clean.reshape(-1), r)[0])
    assert np.array_equal(oracle.decode(y, r)[1], oracle.decode(clean.reshape(-1), r)[1])


def test_empty_packet():
    for r in range(3, 8):
        data, errpos = oracle.decode(np.zeros(0, dtype=np.uint64), r)
        assert data.size == 0 and errpos.size == 0


def test_thread_count_does_not_change_results():
    r = 6
    y = synth.draws(synth.workload_seed("threads", r), 0, 10000)
    a = oracle.decode(y, r, nthreads=1)
    b = oracle.decode(y, r, nthreads=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.decode(np.zeros(4, dtype=np.uint64), 8)
    with pytest.raises(ValueError):
        oracle.decode(np.zeros(3, dtype=np.uint64), 7)

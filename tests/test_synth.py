"""The seeded input generator: published SplitMix64 outputs, determinism and
slice independence, and the channel statistics it promises."""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if l.strip() and not l.startswith("#")]
    seed = int(rows[0][1])
    expect = [int(r[0]) for r in rows[1:]]
    assert [int(v) for v in synth.draws(seed, 0, len(expect))] == expect
    assert [synth.mix64_int(seed + (i + 1) * 0x9E3779B97F4A7C15) for i in range(len(expect))] == expect


def test_slices_are_independent_of_chunking():
    full = synth.draws(99, 0, 5000)
    parts = np.concatenate([synth.draws(99, a, 1000) for a in range(0, 5000, 1000)])
    assert np.array_equal(full, parts)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_message_stream_shape_and_tail(r):
    _, k, _ = synth.code_sizes(r)
    for n_cw in (1, 63, 64, 1000):
        s = synth.message_stream(7, n_cw, r)
        assert s.size == (n_cw * k + 63) // 64
        bits = np.unpackbits(s.view(np.uint8), bitorder="little")
        assert not bits[n_cw * k:].any()
    s = synth.message_stream(7, 100000, r)
    frac = np.unpackbits(s.view(np.uint8)).mean()
    assert abs(frac - 0.5) < 0.01


@pytest.mark.parametrize("r", [3, 6, 7])
def test_error_positions_statistics(r):
    n, _, _ = synth.code_sizes(r)
    n_cw = 200000
    p1, p2 = synth.error_positions(11, n_cw, r, p_single=0.25, p_double=0.05)
    single = (p1 > 0) & (p2 == 0)
    double = p2 > 0
    assert abs(single.mean() - 0.25) < 0.01
    assert abs(double.mean() - 0.05) < 0.005
    assert (p1[double] != p2[double]).all()
    assert p1.max() <= n and p2.max() <= n
    used = p1[p1 > 0]
    counts = np.bincount(used, minlength=n + 1)[1:]
    assert counts.min() > 0.7 * used.size / n


def test_error_rate_extremes():
    p1, p2 = synth.error_positions(3, 5000, 4, p_single=0.0)
    assert not p1.any() and not p2.any()
    p1, p2 = synth.error_positions(3, 5000, 4, p_single=1.0)
    assert (p1 > 0).all() and not p2.any()


def test_flip_masks_and_garbage_layout():
    p1 = np.array([1, 64, 65, 127, 0], dtype=np.uint8)
    p2 = np.array([0, 0, 0, 1, 0], dtype=np.uint8)
    m = synth.flip_masks(p1, p2, 7).reshape(-1, 2)
    assert [int(v) for v in m[:, 0]] == [1, 1 << 63, 0, 1, 0]
    assert [int(v) for v in m[:, 1]] == [0, 0, 1, 1 << 62, 0]
    g = synth.padding_garbage(5, 100, 6)
    assert not (g & np.uint64((1 << 63) - 1)).any()
    g7 = synth.padding_garbage(5, 100, 7).reshape(-1, 2)
    assert not g7[:, 0].any() and not (g7[:, 1] & np.uint64((1 << 63) - 1)).any()


def test_batch_packets_recipe():
    n_cw, r, p = synth.batch_packets(1, 20000)
    assert n_cw.min() >= 64 and n_cw.max() <= 64 << 14
    assert set(np.unique(r)) == {3, 4, 5, 6, 7}
    assert p.min() >= 0 and p.max() <= 0.5
    med = np.median(np.log2(n_cw))
    assert abs(med - 13) < 0.2


def test_torch_generator_matches_numpy_bit_for_bit():
    import torch

    for seed in (1, 1234567, synth.BASE_SEED):
        a = synth.draws(seed, 5, 3000)
        b = synth.draws_torch(seed, 5, 3000, torch.device("cpu")).numpy().view(np.uint64)
        assert np.array_equal(a, b)
    for r in (3, 6, 7):
        s1 = synth.message_stream(9, 777, r)
        s2 = synth.message_stream_torch(9, 777, r, torch.device("cpu")).numpy().view(np.uint64)
        assert np.array_equal(s1, s2)
        p1, p2 = synth.error_positions(4, 5000, r, p_single=0.3)
        m1 = synth.flip_masks(p1, p2, r)
        m2 = synth.flip_masks_torch(4, 5000, r, 0.3, torch.device("cpu")).numpy().view(np.uint64)
        assert np.array_equal(m1, m2)
        rates = torch.full((5000,), 0.3, dtype=torch.float64)
        m3 = synth.flip_masks_torch(4, 5000, r, rates, torch.device("cpu")).numpy().view(np.uint64)
        assert np.array_equal(m1, m3)


@pytest.mark.parametrize("r", [3, 5, 7])
def test_slices_regenerate_the_same_stream(r):
    _, k, _ = synth.code_sizes(r)
    full = synth.message_stream(31, 1000, r)
    bits = np.unpackbits(full.view(np.uint8), bitorder="little")
    for first, n in ((0, 1000), (1, 5), (17, 300), (999, 1), (64, 64)):
        sl = synth.message_stream_slice(31, first, n, r)
        sb = np.unpackbits(sl.view(np.uint8), bitorder="little")
        assert np.array_equal(sb[:n * k], bits[first * k:(first + n) * k])
        assert not sb[n * k:].any()
    p1, p2 = synth.error_positions(8, 1000, r, p_single=0.3, p_double=0.1)
    q1, q2 = synth.error_positions(8, 200, r, p_single=0.3, p_double=0.1, start=400)
    assert np.array_equal(p1[400:600], q1) and np.array_equal(p2[400:600], q2)


def test_segmented_packet_generators():
    b = synth.packet_bytes(3, 1000, 13)
    assert b.shape == (1000, 13) and abs(b.mean() - 127.5) < 2
    assert np.array_equal(synth.packet_bytes(3, 10, 13), b[:10])
    starts, lens = [0, 11, 22], [11, 11, 5]
    b1, b2 = synth.segment_flips(5, 100000, starts, lens, 0.3, 0.1)
    assert abs((b1 >= 0).mean() - 0.4) < 0.01 and abs((b2 >= 0).mean() - 0.1) < 0.005
    for i, (a, n) in enumerate(zip(starts, lens)):
        hit = b1[:, i][b1[:, i] >= 0]
        assert hit.min() == a and hit.max() == a + n - 1
        both = b2[:, i] >= 0
        assert (b2[both, i] != b1[both, i]).all()
        assert (b2[both, i] >= a).all() and (b2[both, i] < a + n).all()
    rows = np.zeros((2, 4), dtype=np.uint8)
    synth.apply_bit_flips(rows, np.array([[0, 9], [31, -1]]), np.array([[1, -1], [-1, -1]]))
    assert rows.tolist() == [[3, 2, 0, 0], [0, 0, 0, 128]]

"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and shapes them into the channel model
of a decode workload: random message bits, and per-codeword error positions
turned into flip masks.  It contains none of the decoder's arithmetic (no
parity, syndrome, correction or extraction).  Turning messages into codewords
is left to an encoder: the CPU oracle in the tests, the library's own encoder
where the bench prepares device-resident inputs.

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style: draw ``c``
of a stream seeded with ``s`` is ``mix64(s + (c + 1) * GAMMA)``, which is the
c-th output of SplitMix64 started from state ``s``.  Any slice of a stream can
be produced independently, so results do not depend on chunking or threads.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1
BASE_SEED = 0x14126862
_CHUNK = 1 << 22


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(total: int, fn) -> None:
    """Run fn(a, b) over [0, total) in chunks, on a thread pool (numpy
    releases the GIL inside its loops).  Results must not depend on order."""
    spans = [(a, min(total, a + _CHUNK)) for a in range(0, total, _CHUNK)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(lambda ab: fn(*ab), spans))


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(z: int) -> int:
    """Scalar SplitMix64 output function on a Python int (mod 2^64)."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def subseed(base: int, *tags: int | str) -> int:
    """Derive an independent stream seed from a base seed and tags."""
    s = base & _MASK64
    for t in tags:
        if isinstance(t, str):
            v = 0
            for ch in t.encode():
                v = (v * 131 + ch) & _MASK64
            t = v
        s = mix64_int(s ^ mix64_int((int(t) + 0x632BE59BD9B4E019) & _MASK64))
    return s


def draws(seed: int, start: int, count: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the stream seeded with ``seed``."""
    ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _MASK64) + ctr * GAMMA
    return mix64(state)


def code_sizes(r: int) -> tuple[int, int, int]:
    """(n, k, storage words per codeword) of the (2^r-1, 2^r-1-r) code."""
    if not 3 <= r <= 7:
        raise ValueError("r must be in [3, 7]")
    n = (1 << r) - 1
    return n, n - r, (2 if r == 7 else 1)


def message_stream(seed: int, n_cw: int, r: int) -> np.ndarray:
    """Uniform random message bits for n_cw codewords as a dense stream.

    Returns uint64 words, ceil(n_cw*k/64) of them; the bits after n_cw*k are 0.
    Every message bit is an independent fair coin, i.e. data i.i.d.
    Bernoulli(0.5).
    """
    _, k, _ = code_sizes(r)
    bits = n_cw * k
    nwords = (bits + 63) // 64
    out = np.empty(nwords, dtype=np.uint64)

    def fill(a, b):
        out[a:b] = draws(seed, a, b - a)

    _chunked(nwords, fill)
    tail = bits % 64
    if nwords and tail:
        out[-1] &= np.uint64((1 << tail) - 1)
    return out


def message_stream_slice(seed: int, first_cw: int, n_cw: int, r: int) -> np.ndarray:
    """The message bits of codewords [first_cw, first_cw + n_cw) of the stream
    ``message_stream(seed, ., r)`` describes, realigned to start at bit 0 and
    with the bits after n_cw*k cleared (a slice of the same random stream)."""
    _, k, _ = code_sizes(r)
    b0 = first_cw * k
    b1 = b0 + n_cw * k
    w0, w1 = b0 // 64, (b1 + 63) // 64
    a = np.concatenate([draws(seed, w0, w1 - w0), np.zeros(1, dtype=np.uint64)])
    sh = np.uint64(b0 % 64)
    if sh:
        out = (a[:-1] >> sh) | (a[1:] << np.uint64(64 - int(sh)))
    else:
        out = a[:-1].copy()
    nwords = (n_cw * k + 63) // 64
    out = out[:nwords]
    tail = (n_cw * k) % 64
    if nwords and tail:
        out[-1] &= np.uint64((1 << tail) - 1)
    return out


def _threshold(prob: float) -> int:
    """Integer threshold t such that a 53-bit uniform u is below t with
    probability ``prob`` (exact for prob = 0 and prob = 1)."""
    if not 0.0 <= prob <= 1.0:
        raise ValueError("probability out of range")
    return int(math.floor(prob * (1 << 53)))


def _first_position(u: np.ndarray, n: int) -> np.ndarray:
    return np.uint64(1) + (((u >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32))


def _second_position(u: np.ndarray, first: np.ndarray, n: int) -> np.ndarray:
    step = np.uint64(1) + (((u & np.uint64(0xFFFFFFFF)) * np.uint64(n - 1)) >> np.uint64(32))
    return np.uint64(1) + ((first - np.uint64(1) + step) % np.uint64(n))


def error_positions(seed: int, n_cw: int, r: int, p_single: float = 0.0,
                    p_double: float = 0.0, start: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Per-codeword channel errors.

    Each codeword independently gets one flipped bit with probability
    ``p_single``, two distinct flipped bits with probability ``p_double`` and
    none otherwise.  Positions are uniform over all n positions (parity
    positions included); the two positions of a double error are a uniform
    unordered pair.  Returns (pos1, pos2) uint8 arrays, 0 meaning "no flip".
    Codeword i uses draw ``start + i`` of the streams, so a slice of a longer
    packet can be regenerated on its own.
    """
    n, _, _ = code_sizes(r)
    t1 = _threshold(p_single)
    t2 = _threshold(min(1.0, p_single + p_double))
    s_kind = subseed(seed, "kind")
    s_pos = subseed(seed, "pos")
    pos1 = np.zeros(n_cw, dtype=np.uint8)
    pos2 = np.zeros(n_cw, dtype=np.uint8)

    def fill(a, b):
        u = draws(s_kind, start + a, b - a) >> np.uint64(11)
        one = u < np.uint64(t1)
        if t2 == 0:
            return
        v = draws(s_pos, start + a, b - a)
        first = _first_position(v, n)
        pos1[a:b] = np.where(u < np.uint64(t2), first, 0).astype(np.uint8)
        if t2 > t1:
            two = (~one) & (u < np.uint64(t2))
            second = _second_position(v, first, n)
            pos2[a:b] = np.where(two, second, 0).astype(np.uint8)

    _chunked(n_cw, fill)
    return pos1, pos2


def flip_masks(pos1: np.ndarray, pos2: np.ndarray, r: int) -> np.ndarray:
    """Storage-layout flip masks (bit p-1 for position p) for the positions."""
    _, _, wpc = code_sizes(r)
    n_cw = pos1.size
    masks = np.zeros(n_cw * wpc, dtype=np.uint64)
    for pos in (pos1, pos2):
        idx = np.flatnonzero(pos)
        bit = pos[idx].astype(np.uint64) - np.uint64(1)
        word = idx.astype(np.int64) * wpc + (bit >> np.uint64(6)).astype(np.int64)
        masks[word] ^= np.left_shift(np.uint64(1), bit & np.uint64(63))
    return masks


def padding_garbage(seed: int, n_cw: int, r: int) -> np.ndarray:
    """Random bits in the storage padding (bits at or above n) of each
    codeword, zero elsewhere.  A decoder must ignore them."""
    n, _, wpc = code_sizes(r)
    g = np.empty(n_cw * wpc, dtype=np.uint64)
    gseed = subseed(seed, "garbage")

    def fill(a, b):
        g[a:b] = draws(gseed, a, b - a)

    _chunked(g.size, fill)
    g = g.reshape(n_cw, wpc)
    valid = [(1 << min(64, max(0, n - 64 * w))) - 1 for w in range(wpc)]
    for w in range(wpc):
        g[:, w] &= np.uint64(~valid[w] & _MASK64)
    return g.reshape(-1)


# --- the same generator on torch tensors (CPU or GPU) --------------------------
#
# Identical bits to the numpy functions above: int64 arithmetic wraps modulo
# 2^64 exactly like uint64, and logical right shifts are masked arithmetic
# shifts.  Used to synthesise workloads too large to build on the host.

def _to_i64(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(x, s: int):
    import torch

    return torch.bitwise_and(torch.bitwise_right_shift(x, s), _to_i64((1 << (64 - s)) - 1))


def mix64_torch(z):
    z = torch_mul(torch_xor(z, _srl(z, 30)), 0xBF58476D1CE4E5B9)
    z = torch_mul(torch_xor(z, _srl(z, 27)), 0x94D049BB133111EB)
    return torch_xor(z, _srl(z, 31))


def torch_xor(a, b):
    import torch

    return torch.bitwise_xor(a, b)


def torch_mul(a, c: int):
    return a * _to_i64(c)


def draws_torch(seed: int, start: int, count: int, device):
    """Draws start .. start+count-1 of the stream seeded with ``seed`` as an
    int64 tensor on ``device`` (bit-identical to ``draws``)."""
    import torch

    ctr = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    state = ctr * _to_i64(0x9E3779B97F4A7C15) + _to_i64(seed)
    return mix64_torch(state)


def message_stream_torch(seed: int, n_cw: int, r: int, device):
    """``message_stream`` as an int64 tensor on ``device``."""
    _, k, _ = code_sizes(r)
    bits = n_cw * k
    nwords = (bits + 63) // 64
    out = draws_torch(seed, 0, nwords, device)
    tail = bits % 64
    if nwords and tail:
        out[-1] &= _to_i64((1 << tail) - 1)
    return out


def flip_masks_torch(seed: int, n_cw: int, r: int, p_single, device):
    """Single-flip masks (storage layout, int64, n_cw*WPC words) with the same
    draws as ``error_positions(seed, n_cw, r, p_single)``; ``p_single`` may be a
    per-codeword float64 tensor (a packet-wise rate) or a number."""
    import torch

    n, _, wpc = code_sizes(r)
    u = _srl(draws_torch(subseed(seed, "kind"), 0, n_cw, device), 11)
    if isinstance(p_single, (int, float)):
        thr = torch.full((n_cw,), _threshold(float(p_single)), dtype=torch.int64, device=device)
    else:
        thr = torch.floor(p_single.to(torch.float64) * float(1 << 53)).to(torch.int64)
    hit = u < thr
    v = draws_torch(subseed(seed, "pos"), 0, n_cw, device)
    pos = 1 + torch.bitwise_right_shift(_srl(v, 32) * n, 32)          # (v >> 32) * n < 2^39
    bit = pos - 1
    masks = torch.zeros((n_cw, wpc), dtype=torch.int64, device=device)
    one = torch.ones_like(bit)
    for w in range(wpc):
        in_w = hit & (torch.div(bit, 64, rounding_mode="floor") == w)
        val = torch.bitwise_left_shift(one, torch.remainder(bit, 64))
        masks[:, w] = torch.where(in_w, val, torch.zeros_like(val))
    return masks.reshape(-1)


# --- segmented packets ------------------------------------------------------

def packet_bytes(seed: int, n_packets: int, msg_bytes: int) -> np.ndarray:
    """[n_packets, msg_bytes] uniformly random message bytes; packet q is
    drawn from counters [q * W, (q + 1) * W), W = ceil(msg_bytes / 8)."""
    w = (msg_bytes + 7) // 8
    out = np.empty(n_packets * w, dtype=np.uint64)

    def fill(a, b):
        out[a:b] = draws(subseed(seed, "bytes"), a, b - a)

    _chunked(n_packets * w, fill)
    return out.view(np.uint8).reshape(n_packets, w * 8)[:, :msg_bytes].copy()


def segment_flips(seed: int, n_packets: int, seg_start, seg_len, p_single: float,
                  p_double: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Channel errors of packets made of bit ranges: in every packet, each
    range [seg_start[i], seg_start[i] + seg_len[i]) independently gets no
    flip, one flip (probability p_single) or two distinct flips (p_double) at
    uniform positions in the range.  Returns (bit1, bit2), int64 arrays of
    shape [n_packets, len(seg_start)] holding the flipped bit indices within
    the packet, -1 for none.  Range i of packet q uses counter q*T + i."""
    start = np.asarray(seg_start, dtype=np.int64)
    length = np.asarray(seg_len, dtype=np.int64)
    T = start.size
    total = n_packets * T
    t1 = _threshold(p_single)
    t2 = _threshold(min(1.0, p_single + p_double))
    u = draws(subseed(seed, "seg-kind"), 0, total).reshape(n_packets, T) >> np.uint64(11)
    v = draws(subseed(seed, "seg-pos"), 0, total).reshape(n_packets, T)
    n = np.broadcast_to(length.astype(np.uint64), (n_packets, T))
    first = np.uint64(1) + (((v >> np.uint64(32)) * n) >> np.uint64(32))
    step = np.uint64(1) + (((v & np.uint64(0xFFFFFFFF)) * np.maximum(n - np.uint64(1), np.uint64(1)))
                           >> np.uint64(32))
    second = np.uint64(1) + ((first - np.uint64(1) + step) % n)
    hit = u < np.uint64(t2)
    two = (u >= np.uint64(t1)) & hit & (n > np.uint64(1))
    bit1 = np.where(hit, first.astype(np.int64) - 1 + start, -1)
    bit2 = np.where(two, second.astype(np.int64) - 1 + start, -1)
    return bit1, bit2


def apply_bit_flips(rows: np.ndarray, *bits: np.ndarray) -> None:
    """XOR the given bit indices (LSB-first within each row, -1 = none) into
    a [P, row_bytes] uint8 array in place."""
    P, row = rows.shape
    flat = rows.reshape(-1)
    for b in bits:
        q, _ = np.nonzero(b >= 0)
        idx = b[b >= 0]
        np.bitwise_xor.at(flat, q * row + idx // 8, (1 << (idx % 8)).astype(np.uint8))


# --- workload recipes ------------------------------------------------------

PLAIN_ERROR_RATES = (0.0, 0.01, 0.1, 0.5, 1.0)


PAPER_PACKET_BYTES = (400, 800, 1200, 1600, 2000)
PAPER_SEGMENTS = (2, 3, 4, 5, 6)


def workload_seed(tag: str, r: int, extra: int | str = 0) -> int:
    return subseed(BASE_SEED, tag, r, extra)


def batch_packets(seed: int, n_packets: int, min_cw: int = 64, max_log2_span: int = 14,
                  r_values=(3, 4, 5, 6, 7), max_p: float = 0.5):
    """Packet list of a batched workload: sizes log-uniform in
    [min_cw, min_cw * 2^max_log2_span], r uniform over ``r_values``, per-packet
    single-error rate uniform in [0, max_p].  Returns (n_cw, r, p) arrays."""
    u = draws(subseed(seed, "sizes"), 0, n_packets)
    ur = draws(subseed(seed, "rs"), 0, n_packets)
    up = draws(subseed(seed, "ps"), 0, n_packets)
    f_u = (u >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    f_r = (ur >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    f_p = (up >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    n_cw = np.floor(min_cw * np.exp2(max_log2_span * f_u)).astype(np.int64)
    rv = np.asarray(r_values, dtype=np.int64)
    r = rv[np.minimum((f_r * len(rv)).astype(np.int64), len(rv) - 1)]
    p = max_p * f_p
    return n_cw, r, p

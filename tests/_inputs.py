"""Received-word construction for the parity tests: seeded messages and
channel errors from ``synth``, codewords from the CPU oracle's encoder.  No
input here ever comes from the HIP library."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def received_words(seed: int, n_cw: int, r: int, p_single: float = 0.0, p_double: float = 0.0,
                   garbage: bool = True) -> np.ndarray:
    """uint64 received words (n_cw*WPC) of a packet: encoded random messages,
    per-codeword flips at uniform positions, random padding bits."""
    stream = synth.message_stream(seed, n_cw, r)
    cw = oracle.encode(stream, n_cw, r)
    p1, p2 = synth.error_positions(seed, n_cw, r, p_single=p_single, p_double=p_double)
    y = cw ^ synth.flip_masks(p1, p2, r)
    if garbage:
        y ^= synth.padding_garbage(seed, n_cw, r)
    return y


def to_device(a: np.ndarray, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


def to_host_u8(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint8)


def to_planes(words: np.ndarray, n_cw: int, r: int, plane_words: int | None = None) -> np.ndarray:
    """Plane layout of received words (a pure re-arrangement of bits):
    plane p-1 holds position p of every codeword, codeword i at bit i%64 of
    word i/64.  Returns uint64 [n, plane_words]."""
    n = (1 << r) - 1
    wpc = 2 if r == 7 else 1
    pw = plane_words or (n_cw + 63) // 64
    w = np.ascontiguousarray(words, dtype=np.uint64).reshape(n_cw, wpc)
    bits = np.unpackbits(w.view(np.uint8).reshape(n_cw, 8 * wpc), axis=1, bitorder="little")[:, :n]
    planes = np.zeros((n, pw * 64), dtype=np.uint8)
    planes[:, :n_cw] = bits.T
    return np.packbits(planes, axis=1, bitorder="little").view(np.uint64)

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

"""Python binding of libhamming.so, the MI355X Hamming decoder.

Argument marshalling only: every step of the decode runs in the library's HIP
kernels.  torch provides device memory and streams.  The C entry points of
``include/hamming.h`` are exposed under the same names; ``decode`` and
``encode`` are conveniences that allocate outputs with torch and call them.

The library must be built (``python -m paper_1412_6862_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises, and no
operation has a CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhamming.so")

HAMMING_OK = 0
HAMMING_EINVAL = -1
HAMMING_EALIGN = -2
HAMMING_ERANGE = -3
HAMMING_ENOMEM = -4
HAMMING_EDEVICE = -5
HAMMING_MAX_CODEWORDS = 1 << 40


class HammingError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, strerror(status), status))


_lock = threading.Lock()
_lib = None

# name -> (argtypes, restype); mirrors include/hamming.h
_u64, _i32, _vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
_SIGNATURES = {
    "hamming_message_bits": ([_i32], _i32),
    "hamming_data_bytes": ([_u64, _i32], _u64),
    "hamming_decode": ([_vp, _u64, _i32, _vp, _vp, _vp], _i32),
    "hamming_encode": ([_vp, _u64, _i32, _vp, _vp], _i32),
    "hamming_plain_config_set": ([_i32, _i32, _u64], _i32),
    "hamming_plain_config_get": ([_i32, ctypes.POINTER(_i32), ctypes.POINTER(_u64)], _i32),
    "hamming_strerror": ([_i32], ctypes.c_char_p),
}


def library() -> ctypes.CDLL:
    """Load libhamming.so from the package directory (raises if missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libhamming.so is not built (run paper_1412_6862_amd/build.py); "
                                  "there is no fallback decoder")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGNATURES.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = res
            _lib = lib
    return _lib


def hamming_strerror(status: int) -> str:
    return library().hamming_strerror(status).decode()


strerror = hamming_strerror


def _check(status: int, where: str) -> None:
    if status != HAMMING_OK:
        raise HammingError(status, where)


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- C entry points, same names ------------------------------------------------

def hamming_message_bits(r: int) -> int:
    return library().hamming_message_bits(r)


def hamming_data_bytes(n_cw: int, r: int) -> int:
    return int(library().hamming_data_bytes(n_cw, r))


def hamming_decode(codewords, n_cw: int, r: int, data_out, errpos_out=None, stream=None) -> None:
    """Enqueue ``hamming_decode`` on ``stream`` (default: torch's current stream)."""
    _check(library().hamming_decode(_ptr(codewords), n_cw, r, _ptr(data_out), _ptr(errpos_out),
                                    _stream(stream)), "hamming_decode")


def hamming_encode(data_in, n_cw: int, r: int, codewords_out, stream=None) -> None:
    _check(library().hamming_encode(_ptr(data_in), n_cw, r, _ptr(codewords_out), _stream(stream)),
           "hamming_encode")


def hamming_plain_config_set(r: int, lane_codewords: int, max_blocks: int = 0) -> None:
    _check(library().hamming_plain_config_set(r, lane_codewords, max_blocks), "hamming_plain_config_set")


def hamming_plain_config_get(r: int) -> tuple[int, int]:
    u = ctypes.c_int()
    mb = ctypes.c_uint64()
    _check(library().hamming_plain_config_get(r, ctypes.byref(u), ctypes.byref(mb)), "hamming_plain_config_get")
    return u.value, mb.value


# ---- conveniences over torch tensors --------------------------------------------

def words_per_codeword(r: int) -> int:
    return 2 if r == 7 else 1


def decode(codewords, r: int, errpos: bool = True, stream=None):
    """Decode a device tensor of codewords (int64/uint64, n_cw or n_cw*2 words).

    Returns (data, errpos): data is a uint8 tensor of hamming_data_bytes(n_cw, r)
    bytes holding the dense message stream, errpos a uint8 tensor of n_cw bytes
    (or None).
    """
    import torch

    if codewords.device.type != "cuda":
        raise ValueError("codewords must be a device tensor")
    cw = codewords.contiguous().view(-1)
    wpc = words_per_codeword(r)
    if cw.numel() % wpc:
        raise ValueError("codeword tensor length is not a multiple of the words per codeword")
    n_cw = cw.numel() // wpc
    nbytes = hamming_data_bytes(n_cw, r)
    data = torch.empty(nbytes, dtype=torch.uint8, device=cw.device)
    ep = torch.empty(n_cw, dtype=torch.uint8, device=cw.device) if errpos else None
    hamming_decode(cw, n_cw, r, data, ep, stream)
    return data, ep


def encode(messages, n_cw: int, r: int, stream=None):
    """Encode n_cw messages from a device tensor holding the dense message
    stream (at least ceil(n_cw*k/64)*8 bytes); returns int64 codewords."""
    import torch

    if messages.device.type != "cuda":
        raise ValueError("messages must be a device tensor")
    out = torch.empty(n_cw * words_per_codeword(r), dtype=torch.int64, device=messages.device)
    hamming_encode(messages.contiguous(), n_cw, r, out, stream)
    return out

"""Hamming decoder oracle: TEST INFRASTRUCTURE ONLY.

A plain CPU implementation (``hamming_oracle.c``, bit-by-bit loops, no masks or
popcounts) of what the decode path computes, following the paper's
decomposition: error detection by a modulo-2 checksum over each index set
(Sec. III.C, Algorithm 1), correction of the bit the checksum names, removal of
the redundancy bits and merging of the messages (Sec. II, Fig. 1).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product decode library never loads
it and shares no code with it.

Every function here is pinned by ``tests/test_oracle_pins.py`` against the
paper's printed index sets, a textbook Hamming(7,4) codeword, brute-force
nearest-codeword decoding and closed-form invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hamming_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
            lib.oracle_code_n.argtypes = [i32]
            lib.oracle_code_n.restype = i32
            lib.oracle_code_k.argtypes = [i32]
            lib.oracle_code_k.restype = i32
            lib.oracle_data_bytes.argtypes = [u64, i32]
            lib.oracle_data_bytes.restype = u64
            lib.oracle_index_set.argtypes = [i32, i32, vp]
            lib.oracle_index_set.restype = i32
            lib.oracle_decode.argtypes = [vp, u64, i32, vp, u64, vp, i32]
            lib.oracle_decode.restype = i32
            lib.oracle_encode.argtypes = [vp, u64, i32, vp, i32]
            lib.oracle_encode.restype = i32
            _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def code_n(r: int) -> int:
    return _load().oracle_code_n(r)


def code_k(r: int) -> int:
    return _load().oracle_code_k(r)


def words_per_codeword(r: int) -> int:
    return 2 if r == 7 else 1


def data_bytes(n_cw: int, r: int) -> int:
    return int(_load().oracle_data_bytes(n_cw, r))


def index_set(n: int, j: int) -> list[int]:
    """Positions of index set I_j of an n-bit segment (Sec. III.A)."""
    buf = np.zeros(max(n, 1), dtype=np.int32)
    cnt = _load().oracle_index_set(n, j, buf.ctypes.data)
    if cnt < 0:
        raise ValueError("bad index set arguments")
    return [int(v) for v in buf[:cnt]]


def decode(codewords: np.ndarray, r: int, nthreads: int | None = None):
    """Decode a packet; returns (data stream as uint8 array, errpos uint8 array).

    ``codewords`` is a uint64 array of n_cw words (r <= 6) or 2*n_cw words
    (r = 7, or shape (n_cw, 2)).
    """
    cw = np.ascontiguousarray(codewords, dtype=np.uint64).reshape(-1)
    wpc = words_per_codeword(r)
    if cw.size % wpc:
        raise ValueError("codeword array length is not a multiple of the words per codeword")
    n_cw = cw.size // wpc
    nbytes = data_bytes(n_cw, r)
    data = np.zeros(nbytes, dtype=np.uint8)
    errpos = np.zeros(n_cw, dtype=np.uint8)
    rc = _load().oracle_decode(cw.ctypes.data, n_cw, r, data.ctypes.data, nbytes,
                               errpos.ctypes.data, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_decode rejected its arguments")
    return data, errpos


def encode(stream: np.ndarray, n_cw: int, r: int, nthreads: int | None = None) -> np.ndarray:
    """Encode n_cw messages taken from a dense LSB-first stream (bytes or words)."""
    s = np.ascontiguousarray(stream).view(np.uint8).reshape(-1)
    need = (n_cw * code_k(r) + 7) // 8
    if s.size < need:
        raise ValueError("message stream too short")
    out = np.zeros(n_cw * words_per_codeword(r), dtype=np.uint64)
    rc = _load().oracle_encode(s.ctypes.data, n_cw, r, out.ctypes.data,
                               nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_encode rejected its arguments")
    return out

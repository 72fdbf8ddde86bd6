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
_SRCS = [os.path.join(_HERE, "hamming_oracle.c"), os.path.join(_HERE, "segmented_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(s) for s in _SRCS)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-Wall", "-Wextra", "-o", tmp] + _SRCS
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            # ORACLE_LIB names another build of the same sources (the
            # sanitizer build of the CPU test suite)
            path = os.environ.get("ORACLE_LIB") or build()
            lib = ctypes.CDLL(path)
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
            u32p = ctypes.POINTER(ctypes.c_uint32)
            lib.oracle_seg_layout.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p]
            lib.oracle_seg_layout.restype = ctypes.c_int64
            lib.oracle_seg_decode.argtypes = [vp, u64, ctypes.c_uint32, ctypes.c_uint32, vp, vp, vp]
            lib.oracle_seg_decode.restype = i32
            lib.oracle_seg_encode.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp, u64]
            lib.oracle_seg_encode.restype = i32
            lib.oracle_seg_many.argtypes = [i32, vp, u64, u64, ctypes.c_uint32, ctypes.c_uint32, vp, u64, vp, vp,
                                            i32]
            lib.oracle_seg_many.restype = i32
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


# ---- segmented packets (the paper's t-segment workload) ---------------------

def seg_layout(msg_bytes: int, t: int):
    """(k, r, n, encoded_bits) of a packet of msg_bytes bytes in t segments:
    message bits, checksum bits and positions of every segment."""
    k = (ctypes.c_uint32 * max(t, 1))()
    r = (ctypes.c_uint32 * max(t, 1))()
    n = (ctypes.c_uint32 * max(t, 1))()
    tot = _load().oracle_seg_layout(msg_bytes, t, k, r, n)
    if tot < 0:
        raise ValueError("unsupported packet shape")
    return list(k)[:t], list(r)[:t], list(n)[:t], int(tot)


def seg_encoded_bytes(msg_bytes: int, t: int) -> int:
    return (seg_layout(msg_bytes, t)[3] + 7) // 8


def seg_decode(enc: np.ndarray, msg_bytes: int, t: int):
    """Decode one encoded packet (bytes or words); returns (message bytes,
    per-segment syndromes as uint16, packet status 0/1/2)."""
    e = np.ascontiguousarray(enc).view(np.uint8).reshape(-1)
    msg = np.zeros(msg_bytes, dtype=np.uint8)
    syn = np.zeros(t, dtype=np.uint16)
    st = np.zeros(1, dtype=np.uint8)
    if _load().oracle_seg_decode(e.ctypes.data, e.size, msg_bytes, t, msg.ctypes.data, syn.ctypes.data,
                                 st.ctypes.data) != 0:
        raise ValueError("oracle_seg_decode rejected its arguments")
    return msg, syn, int(st[0])


def seg_encode(msg: np.ndarray, t: int) -> np.ndarray:
    """Encode one packet (bytes); returns the encoded bit string as bytes
    (ceil(encoded_bits / 8))."""
    m = np.ascontiguousarray(msg, dtype=np.uint8).reshape(-1)
    out = np.zeros(seg_encoded_bytes(m.size, t), dtype=np.uint8)
    if _load().oracle_seg_encode(m.ctypes.data, m.size, t, out.ctypes.data, out.size) != 0:
        raise ValueError("oracle_seg_encode rejected its arguments")
    return out


def seg_decode_many(enc: np.ndarray, msg_bytes: int, t: int, nthreads: int | None = None):
    """Decode packets of one shape stored as rows of a 2-D byte array (row
    length >= the encoded bytes); returns (messages [P, msg_bytes],
    syndromes [P, t], status [P])."""
    e = np.ascontiguousarray(enc, dtype=np.uint8)
    P = e.shape[0]
    msg = np.zeros((P, msg_bytes), dtype=np.uint8)
    syn = np.zeros((P, t), dtype=np.uint16)
    st = np.zeros(P, dtype=np.uint8)
    if _load().oracle_seg_many(0, e.ctypes.data, e.shape[1], P, msg_bytes, t, msg.ctypes.data, msg_bytes,
                               syn.ctypes.data, st.ctypes.data, nthreads or default_threads()) != 0:
        raise ValueError("oracle_seg_many rejected its arguments")
    return msg, syn, st


def seg_encode_many(msg: np.ndarray, t: int, row_bytes: int | None = None, nthreads: int | None = None):
    """Encode rows of a [P, msg_bytes] byte array; returns [P, row_bytes]
    encoded rows (row_bytes >= the encoded bytes, default exactly that)."""
    m = np.ascontiguousarray(msg, dtype=np.uint8)
    P, mb = m.shape
    eb = seg_encoded_bytes(mb, t)
    row = row_bytes or eb
    out = np.zeros((P, row), dtype=np.uint8)
    if _load().oracle_seg_many(1, m.ctypes.data, mb, P, mb, t, out.ctypes.data, row, None, None,
                               nthreads or default_threads()) != 0:
        raise ValueError("oracle_seg_many rejected its arguments")
    return out

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
    "hamming_plain_config_set": ([_i32, _i32, _u64, ctypes.c_uint32], _i32),
    "hamming_plain_config_get": ([_i32, ctypes.POINTER(_i32), ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_uint32)],
                                 _i32),
    "hamming_strerror": ([_i32], ctypes.c_char_p),
    "hamming_batch_layout": ([_vp, ctypes.c_uint32, ctypes.POINTER(_u64), ctypes.POINTER(_u64)], _i32),
    "hamming_batch_workspace_bytes": ([ctypes.c_uint32], _u64),
    "hamming_batch_workspace_min_bytes": ([ctypes.c_uint32], _u64),
    "hamming_decode_grid": ([_u64, _i32], _u64),
    "hamming_decode_batch_grid": ([_u64, ctypes.c_uint32, _u64], _u64),
    "hamming_batch_release_graphs": ([], _i32),
    "hamming_decode_batch": ([_vp, _u64, _vp, _vp, ctypes.c_uint32, _u64, _vp, _u64, _vp, _u64, _vp, _vp, _u64,
                              _vp], _i32),
    "hamming_decode_batch_noalloc": ([_vp, _u64, _vp, _vp, ctypes.c_uint32, _u64, _vp, _u64, _vp, _u64, _vp,
                                      _vp], _i32),
    "hamming_batch_chunk_set": ([ctypes.c_uint32], _i32),
    "hamming_batch_chunk_get": ([ctypes.POINTER(ctypes.c_uint32)], _i32),
    "hamming_batch_config_set": ([_i32, ctypes.c_uint32, ctypes.c_uint32, _i32], _i32),
    "hamming_batch_config_get": ([ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_i32)], _i32),
}

class hamming_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("max_batch_packets", ctypes.c_uint32),
                ("max_batch_codewords", ctypes.c_uint64), ("max_queue", ctypes.c_uint32),
                ("auto_release", ctypes.c_uint32)]


class hamming_completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("data_offset", ctypes.c_uint64),
                ("errpos_offset", ctypes.c_uint64), ("submit_ns", ctypes.c_uint64),
                ("complete_ns", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


_SIGNATURES.update({
    "hamming_tune": ([ctypes.c_char_p, ctypes.c_uint32, _vp], _i32),
    "hamming_tune_load": ([ctypes.c_char_p], _i32),
    "hamming_server_now_ns": ([], _u64),
    "hamming_server_create": ([ctypes.POINTER(hamming_server_config), _vp, _u64, _vp, _u64, ctypes.POINTER(_vp)],
                              _i32),
    "hamming_server_destroy": ([_vp], _i32),
    "hamming_server_submit": ([_vp, _u64, _u64, ctypes.c_uint32, _u64, ctypes.POINTER(_u64)], _i32),
    "hamming_server_progress": ([_vp], _i32),
    "hamming_server_poll": ([_vp, ctypes.POINTER(hamming_completion), ctypes.c_uint32,
                             ctypes.POINTER(ctypes.c_uint32)], _i32),
    "hamming_server_release": ([_vp, _u64], _i32),
    "hamming_server_output_pool": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_u64)], _i32),
    "hamming_server_stats": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                              ctypes.POINTER(_u64)], _i32),
    "hamming_server_run_trace": ([_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _u64, _vp, ctypes.POINTER(_u64)],
                                 _i32),
    "hamming_host_workspace_bytes": ([_u64, _i32, ctypes.c_uint32], _u64),
    "hamming_decode_host": ([_vp, _u64, _i32, _vp, _vp, _u64, _i32, ctypes.c_uint32, _vp, _u64,
                             ctypes.POINTER(ctypes.c_double)], _i32),
})

_SIGNATURES.update({
    "hamming_seg_layout": ([ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int64),
    "hamming_decode_segmented": ([_vp, _u64, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _u64, _vp, _u64, _vp,
                                  _vp], _i32),
    "hamming_encode_segmented": ([_vp, _u64, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _u64, _vp], _i32),
    "hamming_seg_config_set": ([ctypes.c_uint32], _i32),
    "hamming_seg_config_get": ([ctypes.POINTER(ctypes.c_uint32)], _i32),
})

_SIGNATURES.update({
    "hamming_planes_words": ([_u64, _i32], _u64),
    "hamming_decode_planes": ([_vp, _u64, _u64, _i32, _vp, _vp, _vp], _i32),
    "hamming_to_planes": ([_vp, _u64, _i32, _vp, _u64, _vp], _i32),
})

HAMMING_SEG_MAX_T = 32
HAMMING_SEG_MAX_K = 65519
HAMMING_SEG_MAX_BYTES = 4096
HAMMING_SEG_INVALID = 0xFF

HAMMING_TRANSFER_SYNC = 0
HAMMING_TRANSFER_ASYNC = 1
HAMMING_TRANSFER_MAPPED = 2

HAMMING_NO_ERRPOS = (1 << 64) - 1
HAMMING_MAX_BATCH = 1 << 24


def packet_dtype():
    """numpy dtype of ``hamming_packet`` (40 bytes, the C struct's layout)."""
    import numpy as np

    return np.dtype([("in_word_off", "<u8"), ("n_cw", "<u8"), ("r", "<u4"), ("flags", "<u4"),
                     ("data_word_off", "<u8"), ("errpos_off", "<u8")])


def library() -> ctypes.CDLL:
    """Load libhamming.so from the package directory (raises if missing).
    HAMMING_LIB may name another build of the same sources (the sanitizer
    build of the CPU test suite)."""
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("HAMMING_LIB") or LIB_PATH
            if not os.path.exists(path):
                raise ImportError("%s is not built (run paper_1412_6862_amd/build.py); "
                                  "there is no fallback decoder" % path)
            lib = ctypes.CDLL(path)
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


def hamming_plain_config_set(r: int, lane_codewords: int, max_blocks: int = 0, xcd_chunk: int = 1) -> None:
    _check(library().hamming_plain_config_set(r, lane_codewords, max_blocks, xcd_chunk), "hamming_plain_config_set")


def hamming_plain_config_get(r: int) -> tuple[int, int, int]:
    u = ctypes.c_int()
    mb = ctypes.c_uint64()
    xc = ctypes.c_uint32()
    _check(library().hamming_plain_config_get(r, ctypes.byref(u), ctypes.byref(mb), ctypes.byref(xc)),
           "hamming_plain_config_get")
    return u.value, mb.value, xc.value


def hamming_batch_layout(descs) -> tuple[int, int]:
    """Fill data_word_off / errpos_off of a host numpy array of packets in place;
    returns (data_words, errpos_bytes)."""
    import numpy as np

    if descs.dtype != packet_dtype() or not descs.flags["C_CONTIGUOUS"]:
        raise ValueError("descs must be a contiguous array of packet_dtype()")
    dw = ctypes.c_uint64()
    eb = ctypes.c_uint64()
    _check(library().hamming_batch_layout(descs.ctypes.data if descs.size else None, descs.size,
                                          ctypes.byref(dw), ctypes.byref(eb)), "hamming_batch_layout")
    assert isinstance(descs, np.ndarray)
    return dw.value, eb.value


def hamming_batch_workspace_bytes(max_packets: int) -> int:
    return int(library().hamming_batch_workspace_bytes(max_packets))


def hamming_batch_workspace_min_bytes(max_packets: int) -> int:
    return int(library().hamming_batch_workspace_min_bytes(max_packets))


def hamming_decode_grid(n_cw: int, r: int) -> int:
    return int(library().hamming_decode_grid(n_cw, r))


def hamming_decode_batch_grid(cw_words: int, max_packets: int, max_codewords: int = 0) -> int:
    return int(library().hamming_decode_batch_grid(cw_words, max_packets, max_codewords))


def hamming_batch_release_graphs() -> None:
    _check(library().hamming_batch_release_graphs(), "hamming_batch_release_graphs")


def hamming_decode_batch(cw_arena, cw_words: int, descs, n_packets_dev, max_packets: int, max_codewords: int,
                         data_arena, data_words: int, errpos_arena, errpos_bytes: int, status_out, workspace,
                         workspace_bytes: int, stream=None) -> None:
    """Enqueue ``hamming_decode_batch`` (device tensors or raw pointers)."""
    _check(library().hamming_decode_batch(_ptr(cw_arena), cw_words, _ptr(descs), _ptr(n_packets_dev),
                                          max_packets, max_codewords, _ptr(data_arena), data_words,
                                          _ptr(errpos_arena),
                                          errpos_bytes, _ptr(status_out), _ptr(workspace), workspace_bytes,
                                          _stream(stream)), "hamming_decode_batch")


def hamming_decode_batch_noalloc(cw_arena, cw_words: int, descs, n_packets_dev, max_packets: int,
                                 max_codewords: int, data_arena, data_words: int, errpos_arena, errpos_bytes: int,
                                 status_out, stream=None) -> None:
    """Enqueue ``hamming_decode_batch_noalloc`` (device tensors or raw pointers)."""
    _check(library().hamming_decode_batch_noalloc(_ptr(cw_arena), cw_words, _ptr(descs), _ptr(n_packets_dev),
                                                  max_packets, max_codewords, _ptr(data_arena), data_words,
                                                  _ptr(errpos_arena), errpos_bytes, _ptr(status_out),
                                                  _stream(stream)), "hamming_decode_batch_noalloc")


HAMMING_NOALLOC_MAX_PACKETS = 65536
HAMMING_NOALLOC_SCRATCH_BYTES = 4 << 20


def hamming_batch_chunk_set(tiles_log2: int) -> None:
    _check(library().hamming_batch_chunk_set(tiles_log2), "hamming_batch_chunk_set")


def hamming_batch_chunk_get() -> int:
    v = ctypes.c_uint32()
    _check(library().hamming_batch_chunk_get(ctypes.byref(v)), "hamming_batch_chunk_get")
    return v.value


def hamming_batch_config_set(schedule: int, xcd_chunk: int = 1, grid_cap_blocks: int = 0,
                             use_graph: int = 1) -> None:
    _check(library().hamming_batch_config_set(schedule, xcd_chunk, grid_cap_blocks, use_graph),
           "hamming_batch_config_set")


def hamming_batch_config_get() -> tuple[int, int, int, int]:
    s, rt, b, g = ctypes.c_int(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
    _check(library().hamming_batch_config_get(ctypes.byref(s), ctypes.byref(rt), ctypes.byref(b), ctypes.byref(g)),
           "hamming_batch_config_get")
    return s.value, rt.value, b.value, g.value


def hamming_planes_words(n_cw: int, r: int) -> int:
    return int(library().hamming_planes_words(n_cw, r))


def hamming_decode_planes(planes, plane_words: int, n_cw: int, r: int, data_out, errpos_out=None,
                          stream=None) -> None:
    _check(library().hamming_decode_planes(_ptr(planes), plane_words, n_cw, r, _ptr(data_out), _ptr(errpos_out),
                                           _stream(stream)), "hamming_decode_planes")


def hamming_to_planes(codewords, n_cw: int, r: int, planes, plane_words: int, stream=None) -> None:
    _check(library().hamming_to_planes(_ptr(codewords), n_cw, r, _ptr(planes), plane_words, _stream(stream)),
           "hamming_to_planes")


def to_planes(codewords, r: int, stream=None):
    """Plane layout of a device tensor of codewords; returns (planes tensor,
    plane_words)."""
    import torch

    cw = codewords.contiguous().view(-1)
    n_cw = cw.numel() // words_per_codeword(r)
    pw = (n_cw + 63) // 64
    planes = torch.zeros(((1 << r) - 1) * pw, dtype=torch.int64, device=cw.device)
    hamming_to_planes(cw, n_cw, r, planes, pw, stream)
    return planes, pw


def decode_planes(planes, plane_words: int, n_cw: int, r: int, errpos: bool = True, stream=None):
    """Decode a device tensor in the plane layout; returns (data, errpos)."""
    import torch

    data = torch.empty(hamming_data_bytes(n_cw, r), dtype=torch.uint8, device=planes.device)
    ep = torch.empty(n_cw, dtype=torch.uint8, device=planes.device) if errpos else None
    hamming_decode_planes(planes, plane_words, n_cw, r, data, ep, stream)
    return data, ep


def seg_packet_dtype():
    """numpy dtype of ``hamming_seg_packet`` (32 bytes, the C struct's layout)."""
    import numpy as np

    return np.dtype([("enc_word_off", "<u8"), ("msg_word_off", "<u8"), ("msg_bytes", "<u4"), ("t", "<u4"),
                     ("seg_off", "<u8")])


def hamming_seg_layout(msg_bytes: int, t: int):
    """(k, r, encoded_bits) of a segmented packet; raises for a shape the
    decoder does not take."""
    k = (ctypes.c_uint32 * max(t, 1))()
    r = (ctypes.c_uint32 * max(t, 1))()
    tot = library().hamming_seg_layout(msg_bytes, t, k, r) if 1 <= t <= HAMMING_SEG_MAX_T else -1
    if tot < 0:
        raise HammingError(HAMMING_EINVAL, "hamming_seg_layout")
    return list(k)[:t], list(r)[:t], int(tot)


def hamming_decode_segmented(enc_arena, enc_words: int, descs, n_packets: int, max_msg_bytes: int, msg_arena,
                             msg_words: int, syndromes=None, syndrome_count: int = 0, status=None,
                             stream=None) -> None:
    _check(library().hamming_decode_segmented(_ptr(enc_arena), enc_words, _ptr(descs), n_packets, max_msg_bytes,
                                              _ptr(msg_arena), msg_words, _ptr(syndromes), syndrome_count,
                                              _ptr(status), _stream(stream)), "hamming_decode_segmented")


def hamming_seg_config_set(threads_per_packet: int) -> None:
    _check(library().hamming_seg_config_set(threads_per_packet), "hamming_seg_config_set")


def hamming_seg_config_get() -> int:
    m = ctypes.c_uint32()
    _check(library().hamming_seg_config_get(ctypes.byref(m)), "hamming_seg_config_get")
    return m.value


def hamming_encode_segmented(msg_arena, msg_words: int, descs, n_packets: int, max_msg_bytes: int, enc_arena,
                             enc_words: int, stream=None) -> None:
    _check(library().hamming_encode_segmented(_ptr(msg_arena), msg_words, _ptr(descs), n_packets, max_msg_bytes,
                                              _ptr(enc_arena), enc_words, _stream(stream)),
           "hamming_encode_segmented")


def hamming_host_workspace_bytes(chunk_cw: int, r: int, streams: int) -> int:
    return int(library().hamming_host_workspace_bytes(chunk_cw, r, streams))


def hamming_decode_host(host_cw, n_cw: int, r: int, host_data_out, host_errpos_out, chunk_cw: int, mode: int,
                        streams: int, workspace, workspace_bytes: int, times: bool = False):
    """Decode a host-resident packet through the copy pipeline; returns the
    summed (h2d, decode, d2h) milliseconds when ``times`` is set."""
    t = (ctypes.c_double * 3)() if times else None
    _check(library().hamming_decode_host(_ptr(host_cw), n_cw, r, _ptr(host_data_out), _ptr(host_errpos_out),
                                         chunk_cw, mode, streams, _ptr(workspace), workspace_bytes, t),
           "hamming_decode_host")
    return tuple(t) if times else None


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


def decode_host(codewords, r: int, chunk_cw: int = 1 << 22, mode: int = HAMMING_TRANSFER_ASYNC,
                streams: int = 3, errpos: bool = True, device=None):
    """Decode a host tensor of codewords (pin it for overlapping copies; the
    mapped mode requires it); returns host (data, errpos) tensors, pinned when
    the input is."""
    import torch

    if codewords.device.type != "cpu":
        raise ValueError("codewords must be a host tensor")
    cw = codewords.contiguous().view(-1)
    n_cw = cw.numel() // words_per_codeword(r)
    pin = cw.is_pinned()
    data = torch.empty(hamming_data_bytes(n_cw, r), dtype=torch.uint8, pin_memory=pin)
    ep = torch.empty(n_cw, dtype=torch.uint8, pin_memory=pin) if errpos else None
    if mode == HAMMING_TRANSFER_MAPPED:
        ws, wsb = None, 0
    else:
        wsb = hamming_host_workspace_bytes(chunk_cw, r, streams)
        if wsb == 0:
            raise HammingError(HAMMING_EINVAL, "hamming_host_workspace_bytes")
        ws = torch.empty(wsb, dtype=torch.uint8, device=device or torch.device("cuda"))
    hamming_decode_host(cw, n_cw, r, data, ep, chunk_cw, mode, streams, ws, wsb)
    return data, ep


class SegmentedBatch:
    """Device arenas for ``n_packets`` segmented packets of one shape
    (msg_bytes, t), packed back to back: encoded packet q at word
    q * enc_stride, message q at word q * msg_stride, syndromes q*t..q*t+t-1."""

    def __init__(self, n_packets: int, msg_bytes: int, t: int, device=None):
        import numpy as np
        import torch

        dev = device or torch.device("cuda")
        _, _, bits = hamming_seg_layout(msg_bytes, t)
        self.n_packets, self.msg_bytes, self.t = n_packets, msg_bytes, t
        self.enc_stride = (bits + 63) // 64
        self.msg_stride = (msg_bytes + 7) // 8
        d = np.zeros(n_packets, dtype=seg_packet_dtype())
        q = np.arange(n_packets, dtype=np.uint64)
        d["enc_word_off"] = q * np.uint64(self.enc_stride)
        d["msg_word_off"] = q * np.uint64(self.msg_stride)
        d["msg_bytes"] = msg_bytes
        d["t"] = t
        d["seg_off"] = q * np.uint64(t)
        self.descs = torch.from_numpy(d.view(np.uint8)).to(dev)
        self.enc = torch.zeros(n_packets * self.enc_stride, dtype=torch.int64, device=dev)
        self.msg = torch.zeros(n_packets * self.msg_stride, dtype=torch.int64, device=dev)
        self.syndromes = torch.zeros(n_packets * t, dtype=torch.int16, device=dev)
        self.status = torch.zeros(n_packets, dtype=torch.uint8, device=dev)

    def decode(self, stream=None) -> None:
        hamming_decode_segmented(self.enc, self.enc.numel(), self.descs, self.n_packets, self.msg_bytes, self.msg,
                                 self.msg.numel(), self.syndromes, self.syndromes.numel(), self.status, stream)

    def encode(self, stream=None) -> None:
        hamming_encode_segmented(self.msg, self.msg.numel(), self.descs, self.n_packets, self.msg_bytes, self.enc,
                                 self.enc.numel(), stream)


class BatchDecoder:
    """Device-resident batch: descriptor array, packet count, outputs and
    workspace for up to ``max_packets`` packets over one codeword arena.

    ``set_packets`` lays out a host descriptor array, uploads it and sizes the
    output arenas; ``decode`` enqueues one ``hamming_decode_batch``.
    """

    def __init__(self, cw_arena, max_packets: int, device=None, workspace_bytes: int | None = None):
        import torch

        self.device = device or cw_arena.device
        self.cw_arena = cw_arena
        self.max_packets = max_packets
        self.ws_bytes = workspace_bytes or hamming_batch_workspace_bytes(max_packets)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.descs_dev = torch.zeros(max_packets * 40, dtype=torch.uint8, device=self.device)
        self.n_dev = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(max_packets, dtype=torch.int32, device=self.device)
        self.data = None
        self.errpos = None
        self.descs = None

    def set_packets(self, descs, layout: bool = True, data_words=None, errpos_bytes=None):
        import numpy as np
        import torch

        if descs.size > self.max_packets:
            raise ValueError("more packets than max_packets")
        if layout:
            data_words, errpos_bytes = hamming_batch_layout(descs)
        self.descs = descs
        raw = torch.from_numpy(np.ascontiguousarray(descs).view(np.uint8).copy())
        self.descs_dev[: raw.numel()].copy_(raw.to(self.device))
        self.n_dev.fill_(int(descs.size))
        if self.data is None or self.data.numel() < max(1, data_words):
            self.data = torch.empty(max(1, data_words), dtype=torch.int64, device=self.device)
        if self.errpos is None or self.errpos.numel() < max(1, errpos_bytes):
            self.errpos = torch.empty(max(1, errpos_bytes), dtype=torch.uint8, device=self.device)
        self.data_words = data_words
        self.errpos_bytes = errpos_bytes

    def totals(self) -> dict:
        """Batch totals the last decode left in the workspace header."""
        import numpy as np

        h = self.workspace[:32].cpu().numpy()
        q = h[:16].view(np.uint64)
        g = h[16:24].view(np.uint32)
        return {"tiles": int(q[0]), "packets": int(q[1]), "coarse_log2": int(g[0]), "fine_log2": int(g[1])}

    def decode(self, stream=None, max_codewords: int = 0):
        hamming_decode_batch(self.cw_arena, self.cw_arena.numel(), self.descs_dev, self.n_dev, self.max_packets,
                             max_codewords, self.data, self.data.numel(), self.errpos, self.errpos.numel(), self.status,
                             self.workspace, self.ws_bytes, stream)


# ---- autotuning ----------------------------------------------------------------

def hamming_tune(cache_path: str | None = None, flags: int = 3, stream=None) -> None:
    _check(library().hamming_tune(cache_path.encode() if cache_path else None, flags, _stream(stream)),
           "hamming_tune")


def hamming_tune_load(cache_path: str) -> None:
    _check(library().hamming_tune_load(cache_path.encode()), "hamming_tune_load")


# ---- serving -------------------------------------------------------------------

def hamming_server_now_ns() -> int:
    return int(library().hamming_server_now_ns())


def hamming_server_create(config: hamming_server_config, cw_pool, cw_pool_words: int, output_pool,
                          output_pool_bytes: int) -> int:
    h = ctypes.c_void_p()
    _check(library().hamming_server_create(ctypes.byref(config), _ptr(cw_pool), cw_pool_words, _ptr(output_pool),
                                           output_pool_bytes, ctypes.byref(h)), "hamming_server_create")
    return h.value


def hamming_server_destroy(server: int) -> None:
    _check(library().hamming_server_destroy(server), "hamming_server_destroy")


def hamming_server_submit(server: int, in_word_off: int, n_cw: int, r: int, arrival_ns: int) -> int:
    rid = ctypes.c_uint64()
    _check(library().hamming_server_submit(server, in_word_off, n_cw, r, arrival_ns, ctypes.byref(rid)),
           "hamming_server_submit")
    return rid.value


def hamming_server_progress(server: int) -> None:
    _check(library().hamming_server_progress(server), "hamming_server_progress")


def hamming_server_poll(server: int, max_n: int = 1024) -> list:
    buf = (hamming_completion * max_n)()
    n = ctypes.c_uint32()
    _check(library().hamming_server_poll(server, buf, max_n, ctypes.byref(n)), "hamming_server_poll")
    return [buf[i] for i in range(n.value)]


def hamming_server_release(server: int, request_id: int) -> None:
    _check(library().hamming_server_release(server, request_id), "hamming_server_release")


def hamming_server_output_pool(server: int) -> tuple[int, int]:
    base = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    _check(library().hamming_server_output_pool(server, ctypes.byref(base), ctypes.byref(nbytes)),
           "hamming_server_output_pool")
    return base.value, nbytes.value


def hamming_server_stats(server: int) -> dict:
    q, f, u, b = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(library().hamming_server_stats(server, ctypes.byref(q), ctypes.byref(f), ctypes.byref(u), ctypes.byref(b)),
           "hamming_server_stats")
    return {"queued": q.value, "inflight": f.value, "output_bytes_used": u.value, "batches": b.value}


def hamming_server_run_trace(server: int, arrival_ns, in_word_off, n_cw, r, timeout_ns: int):
    """Run an open-loop trace (numpy arrays); returns (latency_ns array, elapsed_ns)."""
    import numpy as np

    a = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
    o = np.ascontiguousarray(in_word_off, dtype=np.uint64)
    c = np.ascontiguousarray(n_cw, dtype=np.uint64)
    rr = np.ascontiguousarray(r, dtype=np.uint32)
    lat = np.zeros(a.size, dtype=np.uint64)
    el = ctypes.c_uint64()
    _check(library().hamming_server_run_trace(server, a.size, a.ctypes.data, o.ctypes.data, c.ctypes.data,
                                              rr.ctypes.data, timeout_ns, lat.ctypes.data, ctypes.byref(el)),
           "hamming_server_run_trace")
    return lat, el.value


class Server:
    """Continuous-batching decode server over a device codeword pool."""

    def __init__(self, cw_pool, slots: int = 4, max_batch_packets: int = 1024,
                 max_batch_codewords: int = 1 << 24, output_pool_bytes: int = 1 << 30,
                 max_queue: int = 1 << 20, auto_release: bool = False):
        import torch

        self.handle = None
        self.pool = cw_pool
        self.output = torch.empty(max(256, output_pool_bytes // 256 * 256), dtype=torch.uint8,
                                  device=cw_pool.device)
        cfg = hamming_server_config(slots, max_batch_packets, max_batch_codewords, max_queue,
                                    1 if auto_release else 0)
        torch.cuda.synchronize()
        self.handle = hamming_server_create(cfg, cw_pool, cw_pool.numel(), self.output, self.output.numel())

    def result(self, completion, r: int, n_cw: int):
        """(data, errpos) device views of a completed request's outputs."""
        nbytes = hamming_data_bytes(n_cw, r)
        return (self.output[completion.data_offset:completion.data_offset + nbytes],
                self.output[completion.errpos_offset:completion.errpos_offset + n_cw])

    def submit(self, in_word_off: int, n_cw: int, r: int, arrival_ns: int | None = None) -> int:
        return hamming_server_submit(self.handle, in_word_off, n_cw, r,
                                     hamming_server_now_ns() if arrival_ns is None else arrival_ns)

    def progress(self) -> None:
        hamming_server_progress(self.handle)

    def poll(self, max_n: int = 1024) -> list:
        return hamming_server_poll(self.handle, max_n)

    def release(self, request_id: int) -> None:
        hamming_server_release(self.handle, request_id)

    def output_pool(self) -> tuple[int, int]:
        return hamming_server_output_pool(self.handle)

    def stats(self) -> dict:
        return hamming_server_stats(self.handle)

    def run_trace(self, arrival_ns, in_word_off, n_cw, r, timeout_s: float = 60.0):
        return hamming_server_run_trace(self.handle, arrival_ns, in_word_off, n_cw, r, int(timeout_s * 1e9))

    def close(self) -> None:
        if self.handle:
            hamming_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

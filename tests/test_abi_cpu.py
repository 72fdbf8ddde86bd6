"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/hamming.h declares, and validates arguments on the host before any
launch (every call below returns before touching the HIP runtime)."""
import ctypes
import os
import re

import pytest

import paper_1412_6862_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(hamming_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = hm.library()
    names = _declared_functions()
    assert "hamming_decode" in names and "hamming_encode" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    for n in _declared_functions():
        assert hasattr(hm, n), n


def test_message_bits_and_data_bytes():
    assert [hm.hamming_message_bits(r) for r in range(3, 8)] == [4, 11, 26, 57, 120]
    assert hm.hamming_message_bits(2) == -1 and hm.hamming_message_bits(8) == -1
    for r, k in zip(range(3, 8), [4, 11, 26, 57, 120]):
        for n in (0, 1, 63, 64, 65, 1 << 26):
            assert hm.hamming_data_bytes(n, r) == ((n * k + 63) // 64) * 8
    assert hm.hamming_data_bytes(10, 9) == 0
    assert hm.hamming_data_bytes(hm.HAMMING_MAX_CODEWORDS + 1, 4) == 0


def _raw_decode(cw, n, r, data, ep):
    return hm.library().hamming_decode(cw, n, r, data, ep, 0)


def test_decode_validation_codes():
    A = 1 << 20   # aligned fake addresses; never dereferenced
    assert _raw_decode(A, 10, 2, A, A) == hm.HAMMING_EINVAL
    assert _raw_decode(A, 10, 8, A, A) == hm.HAMMING_EINVAL
    assert _raw_decode(0, 10, 4, A, A) == hm.HAMMING_EINVAL
    assert _raw_decode(A, 10, 4, 0, A) == hm.HAMMING_EINVAL
    assert _raw_decode(A + 4, 10, 4, A, A) == hm.HAMMING_EALIGN
    assert _raw_decode(A, 10, 4, A + 2, A) == hm.HAMMING_EALIGN
    assert _raw_decode(A, hm.HAMMING_MAX_CODEWORDS + 1, 4, A, A) == hm.HAMMING_ERANGE
    # an empty packet is valid and enqueues nothing, even with NULL pointers
    assert _raw_decode(0, 0, 5, 0, 0) == hm.HAMMING_OK


def test_encode_validation_codes():
    lib = hm.library()
    A = 1 << 20
    assert lib.hamming_encode(A, 4, 1, A, 0) == hm.HAMMING_EINVAL
    assert lib.hamming_encode(0, 4, 3, A, 0) == hm.HAMMING_EINVAL
    assert lib.hamming_encode(A + 1, 4, 3, A, 0) == hm.HAMMING_EALIGN
    assert lib.hamming_encode(A, hm.HAMMING_MAX_CODEWORDS + 1, 3, A, 0) == hm.HAMMING_ERANGE
    assert lib.hamming_encode(0, 0, 3, 0, 0) == hm.HAMMING_OK


def test_plain_config_roundtrip_and_validation():
    old = {r: hm.hamming_plain_config_get(r) for r in range(3, 8)}
    try:
        hm.hamming_plain_config_set(6, 8, 1024, 16)
        assert hm.hamming_plain_config_get(6) == (8, 1024, 16)
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(6, 8, 0, 0)
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(3, 4, 0)      # 4 * 4 bits < one dword
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(5, 3, 0)
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(9, 4, 0)
    finally:
        for r, cfg in old.items():
            hm.hamming_plain_config_set(r, *cfg)


def test_strerror_texts():
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(hm.strerror(code), str) and hm.strerror(code)
    err = hm.HammingError(hm.HAMMING_EALIGN, "x")
    assert "aligned" in str(err)


def test_batch_layout_host_helper():
    import numpy as np

    d = np.zeros(5, dtype=hm.packet_dtype())
    d["n_cw"] = [100, 0, 7, 64, 1]
    d["r"] = [3, 7, 5, 6, 7]
    dw, eb = hm.hamming_batch_layout(d)
    words = [(n * k + 63) // 64 for n, k in zip(d["n_cw"], [4, 120, 26, 57, 120])]
    off = 0
    eoff = 0
    for i in range(5):
        assert d[i]["data_word_off"] == off and d[i]["data_word_off"] % 2 == 0
        assert d[i]["errpos_off"] == eoff and eoff % 16 == 0
        off += words[i] + (words[i] & 1)
        eoff += (int(d["n_cw"][i]) + 15) // 16 * 16
    assert (dw, eb) == (off, eoff)
    bad = d.copy()
    bad[2]["r"] = 2
    before = bad.copy()
    with pytest.raises(hm.HammingError):
        hm.hamming_batch_layout(bad)
    assert np.array_equal(bad, before)


def test_batch_workspace_and_validation_codes():
    lib = hm.library()
    assert hm.hamming_batch_workspace_bytes(0) >= 64
    assert hm.hamming_batch_workspace_bytes(1000) >= 64 + 8 * 1001 + 4 * 3024 + 4 * (1 << 24)
    assert hm.hamming_batch_workspace_bytes(hm.HAMMING_MAX_BATCH + 1) == 0
    A = 1 << 20
    ws = hm.hamming_batch_workspace_bytes(10)
    call = lambda **kw: lib.hamming_decode_batch(
        kw.get("cw", A), 100, kw.get("descs", A), kw.get("n", A), kw.get("maxp", 10), 0, kw.get("data", A), 100,
        A, 100, kw.get("status", A), kw.get("ws", A), kw.get("wsb", ws), 0)
    assert call(maxp=0) == hm.HAMMING_OK
    assert call(maxp=hm.HAMMING_MAX_BATCH + 1) == hm.HAMMING_ERANGE
    assert call(cw=0) == hm.HAMMING_EINVAL
    assert call(descs=0) == hm.HAMMING_EINVAL
    assert call(n=0) == hm.HAMMING_EINVAL
    assert call(ws=0) == hm.HAMMING_EINVAL
    assert call(cw=A + 4) == hm.HAMMING_EALIGN
    assert call(descs=A + 4) == hm.HAMMING_EALIGN
    assert call(status=A + 2) == hm.HAMMING_EALIGN
    wmin = hm.hamming_batch_workspace_min_bytes(10)
    assert call(wsb=wmin - 1) == hm.HAMMING_ENOMEM
    assert call(wsb=0) == hm.HAMMING_ENOMEM


def test_noalloc_batch_limits_and_host_side_codes():
    # the binding's constants are the header's, and the fixed scratch holds the
    # workspace of the largest batch the call accepts
    text = open(os.path.join(ROOT, "include", "hamming.h")).read()
    assert re.search(r"#define HAMMING_NOALLOC_MAX_PACKETS 65536u", text)
    assert re.search(r"#define HAMMING_NOALLOC_SCRATCH_BYTES \(4u << 20\)", text)
    assert hm.HAMMING_NOALLOC_MAX_PACKETS == 65536 and hm.HAMMING_NOALLOC_SCRATCH_BYTES == 4 << 20
    assert hm.hamming_batch_workspace_min_bytes(hm.HAMMING_NOALLOC_MAX_PACKETS) <= hm.HAMMING_NOALLOC_SCRATCH_BYTES
    lib = hm.library()
    A = 1 << 20
    call = lambda maxp: lib.hamming_decode_batch_noalloc(A, 100, A, A, maxp, 0, A, 100, A, 100, A, 0)
    # both return before any HIP call
    assert call(0) == hm.HAMMING_OK
    assert call(hm.HAMMING_NOALLOC_MAX_PACKETS + 1) == hm.HAMMING_ERANGE
    assert call(hm.HAMMING_MAX_BATCH + 1) == hm.HAMMING_ERANGE


def test_batch_workspace_sizes():
    # header (64 bytes) + tile prefix sums (8 per packet + 1) + coarse map (4 * (2n + 1024)) before the fine map
    for n in (0, 1, 10, 1000, 1 << 20):
        fixed = 64 + 8 * (n + 1) + 4 * (2 * n + 1024)
        assert hm.hamming_batch_workspace_min_bytes(n) == fixed + 4
        full = max(4 * n, 1 << 24)
        assert hm.hamming_batch_workspace_bytes(n) == (fixed + 4 * full + 255) // 256 * 256
    assert hm.hamming_batch_workspace_min_bytes(hm.HAMMING_MAX_BATCH + 1) == 0


def test_batch_config_roundtrip():
    old = hm.hamming_batch_config_get()
    try:
        hm.hamming_batch_config_set(1, 4, 4096, 0)
        assert hm.hamming_batch_config_get() == (1, 4, 4096, 0)
        hm.hamming_batch_config_set(2, 1, 0, 1)
        assert hm.hamming_batch_config_get() == (2, 1, 0, 1)
        for args in ((4, 2, 8, 1), (-1, 2, 8, 1), (0, 2, 8, 2), (0, 0, 0, 1), (0, (1 << 20) + 1, 0, 1)):
            with pytest.raises(hm.HammingError):
                hm.hamming_batch_config_set(*args)
    finally:
        hm.hamming_batch_config_set(*old)


def test_server_create_validation_codes():
    lib = hm.library()
    import ctypes

    A = 1 << 20
    h = ctypes.c_void_p()
    good = hm.hamming_server_config(2, 16, 1 << 20, 64, 1)
    assert lib.hamming_server_create(None, A, 100, A, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EINVAL
    assert lib.hamming_server_create(ctypes.byref(good), 0, 100, A, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EINVAL
    assert lib.hamming_server_create(ctypes.byref(good), A, 0, A, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EINVAL
    assert lib.hamming_server_create(ctypes.byref(good), A, 100, A, 100, ctypes.byref(h)) == hm.HAMMING_EINVAL
    assert lib.hamming_server_create(ctypes.byref(good), A + 4, 100, A, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EALIGN
    assert lib.hamming_server_create(ctypes.byref(good), A, 100, A + 8, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EALIGN
    for bad in (hm.hamming_server_config(0, 16, 1, 64, 1), hm.hamming_server_config(17, 16, 1, 64, 1),
                hm.hamming_server_config(2, 0, 1, 64, 1), hm.hamming_server_config(2, 16, 0, 64, 1),
                hm.hamming_server_config(2, 16, 1, 0, 1), hm.hamming_server_config(2, 16, 1, 64, 2)):
        assert lib.hamming_server_create(ctypes.byref(bad), A, 100, A, 1 << 20, ctypes.byref(h)) == hm.HAMMING_EINVAL
    assert lib.hamming_server_destroy(None) == hm.HAMMING_EINVAL
    assert lib.hamming_server_progress(None) == hm.HAMMING_EINVAL
    n = ctypes.c_uint32()
    assert lib.hamming_server_poll(None, None, 0, ctypes.byref(n)) == hm.HAMMING_EINVAL
    assert hm.hamming_server_now_ns() > 0


def test_host_pipeline_workspace_and_validation_codes():
    lib = hm.library()
    for r in range(3, 8):
        wpc = 2 if r == 7 else 1
        one = hm.hamming_host_workspace_bytes(1 << 16, r, 1)
        assert one >= (1 << 16) * 8 * wpc + hm.hamming_data_bytes(1 << 16, r) + (1 << 16)
        assert one % 256 == 0
        assert hm.hamming_host_workspace_bytes(1 << 16, r, 3) == 3 * one
    assert hm.hamming_host_workspace_bytes(100, 4, 1) == 0          # not a multiple of 64
    assert hm.hamming_host_workspace_bytes(0, 4, 1) == 0
    assert hm.hamming_host_workspace_bytes(64, 8, 1) == 0
    assert hm.hamming_host_workspace_bytes(64, 4, 0) == 0
    assert hm.hamming_host_workspace_bytes(64, 4, 9) == 0

    A = 1 << 20   # aligned fake addresses; never dereferenced
    ws = hm.hamming_host_workspace_bytes(64, 4, 2)
    call = lambda **kw: lib.hamming_decode_host(
        kw.get("cw", A), kw.get("n", 1000), kw.get("r", 4), kw.get("data", A), kw.get("ep", A),
        kw.get("chunk", 64), kw.get("mode", hm.HAMMING_TRANSFER_ASYNC), kw.get("streams", 2), kw.get("ws", A),
        kw.get("wsb", ws), None)
    assert call(r=2) == hm.HAMMING_EINVAL
    assert call(mode=2) == hm.HAMMING_EINVAL
    assert call(chunk=65) == hm.HAMMING_EINVAL
    assert call(chunk=0) == hm.HAMMING_EINVAL
    assert call(streams=0) == hm.HAMMING_EINVAL
    assert call(streams=9) == hm.HAMMING_EINVAL
    assert call(n=hm.HAMMING_MAX_CODEWORDS + 1) == hm.HAMMING_ERANGE
    assert call(cw=0) == hm.HAMMING_EINVAL
    assert call(data=0) == hm.HAMMING_EINVAL
    assert call(ws=0) == hm.HAMMING_EINVAL
    assert call(cw=A + 4) == hm.HAMMING_EALIGN
    assert call(data=A + 1) == hm.HAMMING_EALIGN
    assert call(ws=A + 128) == hm.HAMMING_EALIGN
    assert call(wsb=ws - 1) == hm.HAMMING_ENOMEM
    # the synchronous mode stages one chunk at a time, so one stream's share suffices
    assert call(wsb=ws // 2 - 1, mode=hm.HAMMING_TRANSFER_SYNC) == hm.HAMMING_ENOMEM
    assert call(n=0, cw=0, data=0, ws=0) == hm.HAMMING_OK


def test_segmented_layout_matches_the_documented_rule():
    import numpy as np

    assert hm.seg_packet_dtype().itemsize == 32
    k, r, bits = hm.hamming_seg_layout(7, 8)
    assert k == [7] * 8 and r == [4] * 8 and bits == 88
    for mb, t in ((400, 2), (2000, 6), (1, 3), (4096, 1), (4096, 32), (13, 5)):
        k, r, bits = hm.hamming_seg_layout(mb, t)
        assert sum(k) == 8 * mb and max(k) - min(k) <= 1 and k == sorted(k, reverse=True)
        assert all((1 << ri) - 1 - ri >= ki and (ri == 2 or (1 << (ri - 1)) - ri < ki) for ki, ri in zip(k, r))
        assert bits == sum(k) + sum(r)
    for mb, t in ((0, 1), (1, 9), (10, 0), (10, 33), (4097, 2)):
        with pytest.raises(hm.HammingError):
            hm.hamming_seg_layout(mb, t)
    assert np.dtype(hm.seg_packet_dtype()).names[:2] == ("enc_word_off", "msg_word_off")


def test_segmented_validation_codes():
    lib = hm.library()
    A = 1 << 20
    dec = lambda **kw: lib.hamming_decode_segmented(
        kw.get("enc", A), 100, kw.get("descs", A), kw.get("n", 4), kw.get("mx", 2000), kw.get("msg", A), 100,
        kw.get("syn", A), 10, None, None)
    enc = lambda **kw: lib.hamming_encode_segmented(
        kw.get("msg", A), 100, kw.get("descs", A), kw.get("n", 4), kw.get("mx", 2000), kw.get("enc", A), 100, None)
    for call in (dec, enc):
        assert call(mx=0) == hm.HAMMING_EINVAL
        assert call(mx=hm.HAMMING_SEG_MAX_BYTES + 1) == hm.HAMMING_EINVAL
        assert call(n=hm.HAMMING_MAX_BATCH + 1) == hm.HAMMING_ERANGE
        assert call(enc=0) == hm.HAMMING_EINVAL
        assert call(msg=0) == hm.HAMMING_EINVAL
        assert call(descs=0) == hm.HAMMING_EINVAL
        assert call(enc=A + 4) == hm.HAMMING_EALIGN
        assert call(msg=A + 1) == hm.HAMMING_EALIGN
        assert call(descs=A + 4) == hm.HAMMING_EALIGN
        assert call(n=0, enc=0, msg=0, descs=0) == hm.HAMMING_OK
    assert dec(syn=A + 1) == hm.HAMMING_EALIGN


def test_planes_words_and_validation_codes():
    lib = hm.library()
    for r in range(3, 8):
        n = (1 << r) - 1
        assert hm.hamming_planes_words(1, r) == n
        assert hm.hamming_planes_words(64, r) == n
        assert hm.hamming_planes_words(65, r) == 2 * n
        assert hm.hamming_planes_words(0, r) == 0
    assert hm.hamming_planes_words(10, 8) == 0
    A = 1 << 20
    dec = lambda **kw: lib.hamming_decode_planes(kw.get("pl", A), kw.get("pw", 2), kw.get("n", 100),
                                                 kw.get("r", 4), kw.get("d", A), kw.get("e", A), None)
    conv = lambda **kw: lib.hamming_to_planes(kw.get("cw", A), kw.get("n", 100), kw.get("r", 4),
                                              kw.get("pl", A), kw.get("pw", 2), None)
    assert dec(r=2) == hm.HAMMING_EINVAL and conv(r=8) == hm.HAMMING_EINVAL
    assert dec(pl=0) == hm.HAMMING_EINVAL and dec(d=0) == hm.HAMMING_EINVAL
    assert conv(cw=0) == hm.HAMMING_EINVAL and conv(pl=0) == hm.HAMMING_EINVAL
    assert dec(pw=1) == hm.HAMMING_ERANGE and conv(pw=1) == hm.HAMMING_ERANGE
    assert dec(n=hm.HAMMING_MAX_CODEWORDS + 1) == hm.HAMMING_ERANGE
    assert dec(pl=A + 4) == hm.HAMMING_EALIGN and dec(d=A + 4) == hm.HAMMING_EALIGN
    assert conv(cw=A + 4) == hm.HAMMING_EALIGN and conv(pl=A + 2) == hm.HAMMING_EALIGN
    assert dec(n=0, pl=0, d=0) == hm.HAMMING_OK and conv(n=0, cw=0, pl=0) == hm.HAMMING_OK


def test_host_mapped_mode_argument_checks():
    lib = hm.library()
    A = 1 << 20
    M = hm.HAMMING_TRANSFER_MAPPED
    assert lib.hamming_decode_host(A, 10, 4, A, None, 64, 3, 1, None, 0, None) == hm.HAMMING_EINVAL
    assert lib.hamming_decode_host(0, 10, 4, A, None, 64, M, 1, None, 0, None) == hm.HAMMING_EINVAL
    assert lib.hamming_decode_host(A, 10, 4, 0, None, 64, M, 1, None, 0, None) == hm.HAMMING_EINVAL
    assert lib.hamming_decode_host(A + 4, 10, 4, A, None, 64, M, 1, None, 0, None) == hm.HAMMING_EALIGN
    assert lib.hamming_decode_host(A, 10, 9, A, None, 64, M, 1, None, 0, None) == hm.HAMMING_EINVAL
    assert lib.hamming_decode_host(0, 0, 4, 0, None, 0, M, 0, None, 0, None) == hm.HAMMING_OK


def test_segmented_mode_config_roundtrip():
    old = hm.hamming_seg_config_get()
    try:
        for m in (8, 16, 32, 64, 256, 0):
            hm.hamming_seg_config_set(m)
            assert hm.hamming_seg_config_get() == m
        for bad in (1, 4, 128, 512):
            with pytest.raises(hm.HammingError):
                hm.hamming_seg_config_set(bad)
    finally:
        hm.hamming_seg_config_set(old)


DISPATCH_LIMIT_BLOCKS = (2 ** 32 - 1) // 256     # a dispatch holds at most 2^32-1 work-items


def test_plain_grid_is_one_wave_per_tile_clamped_to_the_dispatch_limit():
    old = {r: hm.hamming_plain_config_get(r) for r in range(3, 8)}
    try:
        hm.hamming_plain_config_set(6, 4, 0, 1)
        assert hm.hamming_decode_grid(1 << 26, 6) == (1 << 26) // 256 // 4
        assert hm.hamming_decode_grid(257, 6) == 1 and hm.hamming_decode_grid(4 * 256 + 1, 6) == 2
        assert hm.hamming_decode_grid(0, 6) == 0 and hm.hamming_decode_grid(10, 9) == 0
        # 2^40 codewords = 2^32 tiles = 2^30 workgroups: past the limit, so waves loop
        assert hm.hamming_decode_grid(1 << 40, 6) == DISPATCH_LIMIT_BLOCKS
        assert hm.hamming_decode_grid(hm.HAMMING_MAX_CODEWORDS + 1, 6) == 0
        hm.hamming_plain_config_set(6, 4, 1000, 1)
        assert hm.hamming_decode_grid(1 << 26, 6) == 1000
        hm.hamming_plain_config_set(3, 16, 1 << 31, 1)          # a cap above the limit does not lift it
        assert hm.hamming_decode_grid(1 << 40, 3) == DISPATCH_LIMIT_BLOCKS
        assert hm.hamming_decode_grid(1 << 30, 3) == (1 << 30) // 1024 // 4
    finally:
        for r, (u, mb, xc) in old.items():
            hm.hamming_plain_config_set(r, u, mb, xc)


def test_batch_grid_bound_and_clamp():
    old = hm.hamming_batch_config_get()
    old_chunk = hm.hamming_batch_chunk_get()
    try:
        hm.hamming_batch_config_set(2, old[1], 0, old[3])
        hm.hamming_batch_chunk_set(0)
        # tiles <= cw_words/256 (or hint/128) + one partial tile per packet; one wave per chunk
        assert hm.hamming_decode_batch_grid(1 << 20, 10) == (4096 + 10 + 3) // 4
        assert hm.hamming_decode_batch_grid(1 << 20, 10, 1000) == (7 + 10 + 3) // 4
        assert hm.hamming_decode_batch_grid(1 << 20, 10, 1 << 40) == (4096 + 10 + 3) // 4
        assert hm.hamming_decode_batch_grid(0, 1) == 1
        assert hm.hamming_decode_batch_grid(1 << 20, 0) == 0
        assert hm.hamming_decode_batch_grid(1 << 20, hm.HAMMING_MAX_BATCH + 1) == 0
        assert hm.hamming_decode_batch_grid(1 << 42, 1000) == DISPATCH_LIMIT_BLOCKS
        for c in (1, 3, 6):
            hm.hamming_batch_chunk_set(c)
            chunks = (4096 + 10 + (1 << c) - 1) >> c
            assert hm.hamming_decode_batch_grid(1 << 20, 10) == (chunks + 3) // 4
        # schedule 3: every tile holds at least 256 codewords in 512 words
        hm.hamming_batch_chunk_set(0)
        hm.hamming_batch_config_set(3, old[1], 0, old[3])
        assert hm.hamming_decode_batch_grid(1 << 20, 10) == (2048 + 10 + 3) // 4
        assert hm.hamming_decode_batch_grid(1 << 20, 10, 1000) == (3 + 10 + 3) // 4
        hm.hamming_batch_config_set(2, old[1], 3, old[3])
        assert hm.hamming_decode_batch_grid(1 << 20, 10) == 3
    finally:
        hm.hamming_batch_config_set(*old)
        hm.hamming_batch_chunk_set(old_chunk)


def test_batch_chunk_roundtrip_and_validation():
    old = hm.hamming_batch_chunk_get()
    try:
        for c in range(7):
            hm.hamming_batch_chunk_set(c)
            assert hm.hamming_batch_chunk_get() == c
        with pytest.raises(hm.HammingError):
            hm.hamming_batch_chunk_set(7)
        assert hm.hamming_batch_chunk_get() == 6
    finally:
        hm.hamming_batch_chunk_set(old)


def test_planes_reject_counts_beyond_one_launch():
    A = 1 << 20
    lib = hm.library()
    big = (1 << 37) - (1 << 13) + 1
    assert lib.hamming_decode_planes(A, big, big, 4, A, A, 0) == hm.HAMMING_ERANGE
    assert lib.hamming_to_planes(A, big, 4, A, big, 0) == hm.HAMMING_ERANGE

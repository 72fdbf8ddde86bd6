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
        hm.hamming_plain_config_set(6, 8, 1024)
        assert hm.hamming_plain_config_get(6) == (8, 1024)
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(3, 4, 0)      # 4 * 4 bits < one dword
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(5, 3, 0)
        with pytest.raises(hm.HammingError):
            hm.hamming_plain_config_set(9, 4, 0)
    finally:
        for r, (u, mb) in old.items():
            hm.hamming_plain_config_set(r, u, mb)


def test_strerror_texts():
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(hm.strerror(code), str) and hm.strerror(code)
    err = hm.HammingError(hm.HAMMING_EALIGN, "x")
    assert "aligned" in str(err)

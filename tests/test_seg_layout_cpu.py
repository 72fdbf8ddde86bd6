"""The library's host-side segment layout (closed-form checksum-bit count)
against the oracle's layout (incremental search) over the whole supported
range of packet shapes; both follow the split and checksum-bit readings of
Sec. II / III.A, written independently."""
import pytest

import oracle
import paper_1412_6862_amd as hm


def test_library_layout_equals_oracle_layout_over_all_shapes():
    for mb in list(range(1, 64)) + list(range(64, hm.HAMMING_SEG_MAX_BYTES + 1, 37)) + [hm.HAMMING_SEG_MAX_BYTES]:
        for t in range(1, hm.HAMMING_SEG_MAX_T + 1):
            if 8 * mb < t:
                with pytest.raises(hm.HammingError):
                    hm.hamming_seg_layout(mb, t)
                continue
            k, r, bits = hm.hamming_seg_layout(mb, t)
            ok, orr, on, obits = oracle.seg_layout(mb, t)
            assert (k, r, bits) == (ok, orr, obits), (mb, t)

"""GPU parity of the host-resident decode (copy pipeline, Sec. III.B)
against the CPU oracle.

Tolerance: 0 bits, as for the device-resident decode: chunking and copy
scheduling must not change a single output byte.
"""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words

pytestmark = pytest.mark.gpu

MODES = [hm.HAMMING_TRANSFER_SYNC, hm.HAMMING_TRANSFER_ASYNC]


def _host(a: np.ndarray, pinned: bool):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int64))
    return t.pin_memory() if pinned else t.clone()


def _run(y, r, chunk, mode, streams, pinned, device, errpos=True, times=False):
    import torch

    n_cw = y.size // hm.words_per_codeword(r)
    nbytes = hm.hamming_data_bytes(n_cw, r)
    cw = _host(y, pinned)
    # outputs with 64 canary bytes behind the region the call may write
    data = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, pin_memory=pinned)
    ep = torch.full((n_cw + 64,), 0x5A, dtype=torch.uint8, pin_memory=pinned) if errpos else None
    wsb = hm.hamming_host_workspace_bytes(chunk, r, streams)
    ws = torch.empty(wsb, dtype=torch.uint8, device=device)
    t = hm.hamming_decode_host(cw, n_cw, r, data, ep, chunk, mode, streams, ws, wsb, times=times)
    d = data.numpy()
    assert (d[nbytes:] == 0xA5).all()
    if errpos:
        assert (ep.numpy()[n_cw:] == 0x5A).all()
    return d[:nbytes], (ep.numpy()[:n_cw] if errpos else None), t


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("mode", MODES)
def test_host_pipeline_parity_ragged(gpu_device, r, mode):
    for n_cw, chunk, streams in ((1, 64, 2), (63, 64, 1), (65, 64, 3), (1000, 128, 2), (4097, 1024, 3),
                                 (20000, 4096, 8)):
        y = received_words(synth.workload_seed("gpu-host", r, n_cw), n_cw, r, p_single=0.3, p_double=0.1)
        d_ref, e_ref = oracle.decode(y, r)
        d, e, _ = _run(y, r, chunk, mode, streams, True, gpu_device)
        assert np.array_equal(d, d_ref), (n_cw, chunk, streams)
        assert np.array_equal(e, e_ref), (n_cw, chunk, streams)


@pytest.mark.parametrize("r", [4, 7])
def test_host_pipeline_pageable_and_no_errpos(gpu_device, r):
    n_cw = 30000
    y = received_words(synth.workload_seed("gpu-host-pageable", r), n_cw, r, p_single=0.25, p_double=0.05)
    d_ref, e_ref = oracle.decode(y, r)
    for mode in MODES:
        d, e, _ = _run(y, r, 2048, mode, 3, False, gpu_device)
        assert np.array_equal(d, d_ref) and np.array_equal(e, e_ref)
        d, e, _ = _run(y, r, 2048, mode, 2, True, gpu_device, errpos=False)
        assert np.array_equal(d, d_ref) and e is None


def test_host_pipeline_sync_times(gpu_device):
    r, n_cw = 6, 1 << 18
    y = received_words(synth.workload_seed("gpu-host-times", r), n_cw, r, p_single=0.2)
    d_ref, e_ref = oracle.decode(y, r)
    d, e, t = _run(y, r, 1 << 15, hm.HAMMING_TRANSFER_SYNC, 1, True, gpu_device, times=True)
    assert np.array_equal(d, d_ref) and np.array_equal(e, e_ref)
    assert len(t) == 3 and all(x > 0 for x in t)


def test_host_pipeline_convenience_matches_device_decode(gpu_device):
    import torch

    r, n_cw = 5, 200000
    y = received_words(synth.workload_seed("gpu-host-conv", r), n_cw, r, p_single=0.3)
    cw = _host(y, True)
    d_host, e_host = hm.decode_host(cw, r, chunk_cw=1 << 14, streams=4, device=gpu_device)
    d_dev, e_dev = hm.decode(cw.to(gpu_device), r)
    torch.cuda.synchronize()
    assert torch.equal(d_host, d_dev.cpu()) and torch.equal(e_host, e_dev.cpu())


@pytest.mark.parametrize("r", [3, 6, 7])
def test_host_mapped_mode_parity(gpu_device, r):
    import torch

    n_cw = 70000 + 13
    y = received_words(synth.workload_seed("gpu-host-mapped", r), n_cw, r, p_single=0.3, p_double=0.1)
    d_ref, e_ref = oracle.decode(y, r)
    cw = _host(y, True)
    data, ep = hm.decode_host(cw, r, mode=hm.HAMMING_TRANSFER_MAPPED, device=gpu_device)
    assert np.array_equal(data.numpy(), d_ref) and np.array_equal(ep.numpy(), e_ref)
    # interior pointers of pinned allocations map too
    big = torch.full((d_ref.size + 64,), 0xA5, dtype=torch.uint8, pin_memory=True)
    hm.hamming_decode_host(cw, n_cw, r, big[8:8 + d_ref.size], None, 64, hm.HAMMING_TRANSFER_MAPPED, 1, None, 0)
    b = big.numpy()
    assert np.array_equal(b[8:8 + d_ref.size], d_ref) and (b[:8] == 0xA5).all() and (b[8 + d_ref.size:] == 0xA5).all()


def test_host_mapped_mode_rejects_unmapped_memory(gpu_device):
    import torch

    n_cw = 4096
    y = received_words(synth.workload_seed("gpu-host-mapped-bad", 4), n_cw, 4)
    pageable = _host(y, False)
    pinned = _host(y, True)
    out_pinned = torch.empty(hm.hamming_data_bytes(n_cw, 4), dtype=torch.uint8, pin_memory=True)
    out_pageable = torch.empty(hm.hamming_data_bytes(n_cw, 4), dtype=torch.uint8)
    on_device = torch.empty(n_cw, dtype=torch.int64, device=gpu_device)
    M = hm.HAMMING_TRANSFER_MAPPED
    for cw, out in ((pageable, out_pinned), (pinned, out_pageable), (on_device, out_pinned)):
        with pytest.raises(hm.HammingError) as ei:
            hm.hamming_decode_host(cw, n_cw, 4, out, None, 64, M, 1, None, 0)
        assert ei.value.status == hm.HAMMING_EINVAL

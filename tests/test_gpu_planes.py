"""GPU parity of the bit-plane layout decode and the layout converter
against the CPU oracle.

Tolerance: 0 bits.  The plane decode must produce exactly the oracle's
message stream and error positions for the same received words; the
converter must produce exactly the CPU re-arrangement of the bits.
"""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words, to_device, to_host_u8, to_planes

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 4096 + 31, 20000]


def _decode_planes(planes_np, pw, n_cw, r, device, errpos=True):
    import torch

    pl = torch.from_numpy(np.ascontiguousarray(planes_np).reshape(-1).view(np.int64)).to(device)
    data, ep = hm.decode_planes(pl, pw, n_cw, r, errpos=errpos)
    torch.cuda.synchronize()
    return to_host_u8(data), (to_host_u8(ep) if errpos else None)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("n_cw", SIZES)
def test_planes_parity_ragged_sizes(gpu_device, r, n_cw):
    y = received_words(synth.workload_seed("gpu-planes", r, n_cw), n_cw, r, p_single=0.3, p_double=0.1)
    d_ref, e_ref = oracle.decode(y, r)
    d, e = _decode_planes(to_planes(y, n_cw, r), (n_cw + 63) // 64, n_cw, r, gpu_device)
    assert np.array_equal(d, d_ref) and np.array_equal(e, e_ref)


@pytest.mark.parametrize("r", [3, 5, 7])
def test_planes_parity_error_rates_padding_and_stride(gpu_device, r):
    n_cw = 70000
    for p in synth.PLAIN_ERROR_RATES:
        y = received_words(synth.workload_seed("gpu-planes-rates", r, str(p)), n_cw, r, p_single=p)
        d_ref, e_ref = oracle.decode(y, r)
        pw = (n_cw + 63) // 64 + 5          # planes further apart than needed
        planes = to_planes(y, n_cw, r, pw)
        # bits past n_cw in the last plane word are ignored
        tail = np.uint64(~((1 << (n_cw % 64)) - 1) & ((1 << 64) - 1))
        planes[:, n_cw // 64] |= tail
        planes[:, n_cw // 64 + 1:] = np.uint64(0xDEADBEEFDEADBEEF)
        d, e = _decode_planes(planes, pw, n_cw, r, gpu_device)
        assert np.array_equal(d, d_ref) and np.array_equal(e, e_ref), p
    d, e = _decode_planes(planes, pw, n_cw, r, gpu_device, errpos=False)
    assert np.array_equal(d, d_ref) and e is None


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_planes_unaligned_outputs_and_canaries(gpu_device, r):
    import torch

    n_cw = 5000 + 17
    y = received_words(synth.workload_seed("gpu-planes-align", r), n_cw, r, p_single=0.5)
    d_ref, e_ref = oracle.decode(y, r)
    pl = torch.from_numpy(to_planes(y, n_cw, r).reshape(-1).view(np.int64)).to(gpu_device)
    nb = hm.hamming_data_bytes(n_cw, r)
    big = torch.full((nb + 64,), 0x5A, dtype=torch.uint8, device=gpu_device)
    ep = torch.full((n_cw + 64,), 0xA5, dtype=torch.uint8, device=gpu_device)
    data = big[8:8 + nb]                      # 8-byte but not 16-byte aligned
    e = ep[3:3 + n_cw]                        # unaligned errpos
    hm.hamming_decode_planes(pl, (n_cw + 63) // 64, n_cw, r, data, e)
    torch.cuda.synchronize()
    b = to_host_u8(big)
    assert np.array_equal(b[8:8 + nb], d_ref) and (b[:8] == 0x5A).all() and (b[8 + nb:] == 0x5A).all()
    x = to_host_u8(ep)
    assert np.array_equal(x[3:3 + n_cw], e_ref) and (x[:3] == 0xA5).all() and (x[3 + n_cw:] == 0xA5).all()


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("n_cw", [1, 33, 2049, 20000])
def test_to_planes_matches_cpu_rearrangement(gpu_device, r, n_cw):
    import torch

    y = received_words(synth.workload_seed("gpu-to-planes", r, n_cw), n_cw, r, p_single=0.3)
    planes, pw = hm.to_planes(to_device(y, gpu_device), r)
    torch.cuda.synchronize()
    got = planes.cpu().numpy().view(np.uint64).reshape((1 << r) - 1, pw)
    assert np.array_equal(got, to_planes(y, n_cw, r))


@pytest.mark.parametrize("r,n_cw", [(3, 1 << 26), (5, 1 << 26), (7, 1 << 25)])
def test_planes_full_size_equals_plain_decode_and_oracle_samples(gpu_device, r, n_cw):
    """Full-size packets: the plane decode equals the plain decode of the
    same received words byte for byte, and sampled slices equal the oracle."""
    import torch

    seed = synth.workload_seed("gpu-planes-full", r)
    cw = hm.encode(synth.message_stream_torch(seed, n_cw, r, gpu_device), n_cw, r)
    cw ^= synth.flip_masks_torch(seed, n_cw, r, 0.1, gpu_device)
    d_plain, e_plain = hm.decode(cw, r)
    planes, pw = hm.to_planes(cw, r)
    d, e = hm.decode_planes(planes, pw, n_cw, r)
    torch.cuda.synchronize()
    assert torch.equal(d, d_plain) and torch.equal(e, e_plain)
    k = hm.hamming_message_bits(r)
    wpc = hm.words_per_codeword(r)
    for first in (0, n_cw // 3 * 64 // 64, n_cw - 64):
        first -= first % 64
        y = cw[first * wpc:(first + 64) * wpc].cpu().numpy().view(np.uint64)
        d_ref, e_ref = oracle.decode(y, r)
        got = d[first * k // 8:first * k // 8 + d_ref.size].cpu().numpy()
        assert np.array_equal(got, d_ref) and np.array_equal(e[first:first + 64].cpu().numpy(), e_ref)

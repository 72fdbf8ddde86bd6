"""The allocation-free batched decode, hamming_decode_batch_noalloc, against
hamming_decode_batch with a caller workspace: byte-identical messages, error
positions and statuses on two calls in a row through the C ABI, the first
with more tiles than the fixed scratch's tile map holds (probe path), the
second a smaller mixed batch (also checked packet by packet against the
oracle).  Tolerance: 0 bits."""
import numpy as np
import pytest

import oracle
import paper_1412_6862_amd as hm
import synth
from _inputs import received_words

pytestmark = pytest.mark.gpu


def _run_both(cw, descs, max_packets, dev, data_words, errpos_bytes):
    """Decode one batch (descriptors already laid out) with both entry points
    into separate, prefilled outputs; returns (data, errpos, status) of each."""
    import torch

    raw = torch.from_numpy(np.ascontiguousarray(descs).view(np.uint8).copy()).to(dev)
    n_dev = torch.tensor([descs.size], dtype=torch.int32, device=dev)
    outs = []
    for noalloc in (False, True):
        data = torch.full((max(1, data_words),), 0x3C3C3C3C3C3C3C3C, dtype=torch.int64, device=dev)
        ep = torch.full((max(1, errpos_bytes),), 0xC3, dtype=torch.uint8, device=dev)
        st = torch.full((max_packets,), -7, dtype=torch.int32, device=dev)
        if noalloc:
            hm.hamming_decode_batch_noalloc(cw, cw.numel(), raw, n_dev, max_packets, 0, data, data.numel(), ep,
                                            ep.numel(), st)
        else:
            wsb = hm.hamming_batch_workspace_bytes(max_packets)
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            hm.hamming_decode_batch(cw, cw.numel(), raw, n_dev, max_packets, 0, data, data.numel(), ep, ep.numel(),
                                    st, ws, wsb)
            torch.cuda.synchronize()
            tiles = int(ws[:8].cpu().numpy().view(np.uint64)[0])      # workspace header: total tiles
        torch.cuda.synchronize()
        outs.append((data, ep, st))
    return outs, tiles


def test_noalloc_matches_workspace_entry_two_calls(gpu_device):
    import torch

    rng = np.random.default_rng(0x6862)
    # call 1: 2000 packets of 2^16..2^20 codewords, r = 3..7, random words:
    # about 1.8 M tiles, more than the scratch's fine map (~1.04 M entries
    # at 2000 packets), so waves find their packets by probing
    n1 = 2000
    sizes = np.exp2(rng.uniform(16, 20, n1)).astype(np.uint64)
    rs = rng.integers(3, 8, n1)
    d1 = np.zeros(n1, dtype=hm.packet_dtype())
    off = 0
    for i in range(n1):
        d1[i]["in_word_off"] = off
        d1[i]["n_cw"] = int(sizes[i])
        d1[i]["r"] = int(rs[i])
        off += int(sizes[i]) * (2 if rs[i] == 7 else 1) + int(rng.integers(0, 2))
    print("noalloc call 1: %d packets, %d input words" % (n1, off), flush=True)
    g = torch.Generator(device=gpu_device)
    g.manual_seed(1)
    cw1 = torch.randint(-(1 << 62), 1 << 62, (off + 2,), dtype=torch.int64, device=gpu_device, generator=g)
    ((a_d, a_e, a_s), (b_d, b_e, b_s)), tiles = _run_both(cw1, d1, n1, gpu_device, *hm.hamming_batch_layout(d1))
    fixed = hm.hamming_batch_workspace_min_bytes(n1) - 4
    assert tiles > (hm.HAMMING_NOALLOC_SCRATCH_BYTES - fixed) // 4, "call 1 must outgrow the scratch's fine map"
    assert torch.equal(a_s[:n1], torch.zeros(n1, dtype=torch.int32, device=gpu_device))
    assert torch.equal(a_d, b_d) and torch.equal(a_e, b_e) and torch.equal(a_s, b_s)
    del cw1, a_d, a_e, b_d, b_e

    # call 2: a smaller mixed batch with one rejected descriptor
    n2 = 300
    sizes2 = [int(rng.choice([0, 1, 63, 64, 65, 255, 256, 257, 1000, 4097])) for _ in range(n2)]
    rs2 = [int(rng.integers(3, 8)) for _ in range(n2)]
    d2 = np.zeros(n2, dtype=hm.packet_dtype())
    chunks, ys, off = [], [], 0
    for i, (n_cw, r) in enumerate(zip(sizes2, rs2)):
        y = (received_words(synth.workload_seed("noalloc", r, i), n_cw, r, p_single=0.3, p_double=0.1)
             if n_cw else np.zeros(0, dtype=np.uint64))
        d2[i]["in_word_off"] = off
        d2[i]["n_cw"] = n_cw
        d2[i]["r"] = r
        chunks.append(y)
        ys.append(y)
        off += y.size
    layout2 = hm.hamming_batch_layout(d2)
    d2[17]["r"] = 9                                            # rejected: HAMMING_EINVAL
    arena = np.concatenate(chunks + [np.zeros(2, dtype=np.uint64)])
    print("noalloc call 2: %d packets, %d input words" % (n2, arena.size), flush=True)
    cw2 = torch.from_numpy(arena.view(np.int64)).to(gpu_device)
    max2 = 512
    ((a_d, a_e, a_s), (b_d, b_e, b_s)), _ = _run_both(cw2, d2, max2, gpu_device, *layout2)
    assert torch.equal(a_d, b_d) and torch.equal(a_e, b_e) and torch.equal(a_s[:n2], b_s[:n2])
    st = b_s.cpu().numpy()
    assert st[17] == hm.HAMMING_EINVAL and (np.delete(st[:n2], 17) == 0).all()
    data = b_d.cpu().numpy().view(np.uint8)
    ep = b_e.cpu().numpy()
    for i, (y, d) in enumerate(zip(ys, d2)):
        if i == 17:
            continue
        dref, eref = oracle.decode(y, int(d["r"]))
        o, e = int(d["data_word_off"]) * 8, int(d["errpos_off"])
        assert np.array_equal(data[o:o + dref.size], dref), "packet %d data" % i
        assert np.array_equal(ep[e:e + eref.size], eref), "packet %d errpos" % i


def test_noalloc_rejects_oversized_batch(gpu_device):
    import torch

    one = torch.zeros(8, dtype=torch.int64, device=gpu_device)
    n_dev = torch.zeros(1, dtype=torch.int32, device=gpu_device)
    with pytest.raises(hm.HammingError) as ei:
        hm.hamming_decode_batch_noalloc(one, 8, one, n_dev, hm.HAMMING_NOALLOC_MAX_PACKETS + 1, 0, one, 8, None, 0,
                                        None)
    assert ei.value.status == hm.HAMMING_ERANGE

"""GPU parity of the allocation-free batched entry point
(aes_ctr_xcrypt_batched_noalloc) against aes_ctr_xcrypt_batched.

Two calls in a row on the library's static workspace, the second with fewer
and shorter messages, must each equal the workspace form on the same
segments byte for byte (tolerance 0), including the status word and bytes
outside every segment; a third call with one invalid segment reports
AES_ERR_SEGMENT through the status pointer and leaves that segment untouched.
"""
import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am
from paper_1506_08503_amd import batch as bt
from paper_1506_08503_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(seed, nmsg, max_len):
    g = np.random.Generator(np.random.PCG64(seed))
    lengths = np.array([0, 1, 15, 16, 17, 16 * 256 + 3] +
                       wl.log_uniform_lengths(g, nmsg, max_len).tolist(), np.int64)
    n = lengths.size
    keys = [g.bytes(int(k)) for k in g.choice([16, 24, 32], size=n)]
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    ctr0 = np.where(g.random(n) < 0.5, 0, g.integers(0, 2 ** 20, size=n)).astype(np.uint32)
    in_off, total = wl.pack_offsets(lengths)
    pt = np.frombuffer(g.bytes(max(total, 16)), np.uint8).copy()
    segs = bt.segment_table(in_off, in_off, lengths, np.arange(n, dtype=np.uint32), ctr0, nonces)
    return dict(segs=segs, keys=keys, pt=pt, lengths=lengths, in_off=in_off, ctr0=ctr0,
                nonces=nonces)


def _run_both(case, tune=None):
    segs = torch.from_numpy(case["segs"].view(np.uint8).copy()).to(DEV)
    kt = torch.stack([am.key_schedule(k, DEV) for k in case["keys"]])
    x = torch.from_numpy(case["pt"]).to(DEV)
    ref = torch.full_like(x, 0x5A)
    ws = bt.workspace(case["lengths"].size, DEV)
    am.ctr_xcrypt_batched(segs, kt, x, ref, ws, tune)
    ref_status = am.batched_read_status(ws)
    got = torch.full_like(x, 0x5A)
    status = torch.full((1,), 12345, dtype=torch.int32, device=DEV)
    am.ctr_xcrypt_batched_noalloc(segs, kt, x, got, tune, status)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), ref_status, got.cpu().numpy(), int(status.item())


@pytest.mark.parametrize("tune", [None, {"layout": am.LAYOUT_TTABLE, "tile_blocks": 256},
                                  {"layout": am.LAYOUT_BITSLICE}],
                         ids=["default", "ttable-t256", "bitslice"])
def test_noalloc_equals_workspace_form_twice(oracle, tune):
    big = _case(0xA110C, 600, 1 << 17)
    small = _case(0xA110D, 40, 1 << 12)
    assert small["lengths"].size < big["lengths"].size
    assert small["pt"].size < big["pt"].size
    for case in (big, small):
        ref, ref_st, got, st = _run_both(case, tune)
        assert ref_st == 0 and st == 0
        assert np.array_equal(got, ref)
    # the small call against the oracle too, message by message
    for i in range(small["lengths"].size):
        a, n = int(small["in_off"][i]), int(small["lengths"][i])
        exp = oracle.ctr_xcrypt(small["keys"][i], small["nonces"][i].tobytes(),
                                int(small["ctr0"][i]), small["pt"][a:a + n])
        assert np.array_equal(got[a:a + n], exp), i


def test_noalloc_reports_bad_segment():
    case = _case(0xA110E, 30, 1 << 12)
    case["segs"]["reserved"][3] = 1          # invalid: reserved field set
    ref, ref_st, got, st = _run_both(case)
    assert ref_st == -7 and st == -7          # AES_ERR_SEGMENT
    assert np.array_equal(got, ref)
    a, n = int(case["in_off"][3]), int(case["lengths"][3])
    assert np.all(got[a:a + n] == 0x5A)

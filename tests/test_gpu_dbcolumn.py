"""Deterministic encryption of a database column (AES-256 ECB, the CryptDB
style use the paper cites for equality queries over encrypted data, sec. I):
2^26 int64 values, Zipf-distributed (s = 1.1) over 2^20 distinct values, each
zero-padded to a 16-byte block.  Checks the round trip, that equal values give
equal ciphertexts and distinct values distinct ones, and every row against the
oracle: ECB is deterministic, so the oracle enciphers each of the 2^20
distinct values once and row i must equal the oracle block of its value."""
import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am
from paper_1506_08503_amd import workloads as wl

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
DEV = "cuda"


def test_dbcolumn_aes256_ecb(oracle):
    col = wl.dbcolumn_inputs()
    values = torch.from_numpy(col.values).to(DEV)
    ranks = torch.from_numpy(col.ranks).to(DEV)
    blocks = torch.zeros((ranks.numel(), 2), dtype=torch.int64, device=DEV)
    blocks[:, 0] = values[ranks]
    pt = blocks.view(torch.uint8).view(-1)
    ks = am.key_schedule(col.key, DEV)
    ct = am.ecb_encrypt(ks, pt)
    back = am.ecb_decrypt(ks, ct)
    assert torch.equal(back, pt)
    assert torch.count_nonzero(back.view(-1, 16)[:, 8:]) == 0
    # equality preserved both ways (1-D ops only: 2^26 rows)
    words = ct.view(torch.int64).view(-1, 2)
    c0, c1 = words[:, 0].contiguous(), words[:, 1].contiguous()
    order = torch.argsort(ranks)
    r = ranks.index_select(0, order)
    s0, s1 = c0.index_select(0, order), c1.index_select(0, order)
    same = r[1:] == r[:-1]
    eq = (s0[1:] == s0[:-1]) & (s1[1:] == s1[:-1])
    assert bool(torch.all(eq | ~same))                    # equal values -> equal ciphertexts
    n_distinct_vals = int(same.numel() - same.sum().item()) + 1
    # distinct ciphertext blocks: lexicographic sort by (c0, c1), count changes
    _, o1 = torch.sort(c1, stable=True)
    _, o0 = torch.sort(c0.index_select(0, o1), stable=True)
    o = o1.index_select(0, o0)
    t0, t1 = c0.index_select(0, o), c1.index_select(0, o)
    n_distinct_ct = int(((t0[1:] != t0[:-1]) | (t1[1:] != t1[:-1])).sum().item()) + 1
    assert n_distinct_ct == n_distinct_vals == int(np.unique(col.ranks).size)
    # oracle on sampled rows
    g = np.random.Generator(np.random.PCG64(4))
    idx = np.unique(np.concatenate([[0, ranks.numel() - 1],
                                    g.integers(0, ranks.numel(), 20000)]))
    it = torch.from_numpy(idx).to(DEV)
    pt_s = pt.view(-1, 16).index_select(0, it).cpu().numpy().reshape(-1)
    ct_s = ct.view(-1, 16).index_select(0, it).cpu().numpy().reshape(-1)
    assert np.array_equal(ct_s, oracle.ecb_encrypt(col.key, pt_s, threads=8))
    packed = wl.pack_int64_blocks(col.values[col.ranks[idx]])
    assert np.array_equal(pt_s, packed)
    # every row: oracle ciphertext of each distinct value, gathered by rank
    table = oracle.ecb_encrypt(col.key, wl.pack_int64_blocks(col.values), threads=8)
    tw = torch.from_numpy(np.ascontiguousarray(table).view("<i8").reshape(-1, 2)).to(DEV)
    for k, ck in enumerate((c0, c1)):             # 1-D gathers (2^26 rows)
        assert torch.equal(ck, tw[:, k].contiguous().index_select(0, ranks))

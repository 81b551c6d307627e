"""GCM and GHASH on the GPU against the oracle (NIST SP 800-38D).

Exact parity with the oracle wherever it finishes in seconds: the GCM
specification's test vectors, ragged message and AAD lengths that reach every
pass shape of the parallel GHASH (final wave only, narrow passes, the wide
replicated-table pass), AES-128/192/256, in place, decryption.  At 4 GiB, where
the oracle's bitwise GHASH would take minutes, linearity pins the result: the
tags of two messages that differ in a few blocks differ by sum_i D_i H^(m-i+1),
which the oracle's GF(2^128) product computes block by block.
"""
import os

import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gcm_vectors.txt")


def _dev(a):
    return torch.from_numpy(np.array(a, dtype=np.uint8, copy=True)).cuda()


def _np(t):
    return t.cpu().numpy()


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _vectors():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("gcm "):
                v = line.split()
                h = lambda s: b"" if s == "-" else bytes.fromhex(s)
                out.append((h(v[1]), h(v[2]), h(v[3]), h(v[4]), h(v[5]), h(v[6])))
    return out


@pytest.mark.parametrize("case", range(6))
def test_gcm_spec_vectors(case):
    key, iv, aad, pt, ct, tag = _vectors()[case]
    ks = am.key_schedule(key)
    x = _dev(np.frombuffer(pt, np.uint8)) if pt else torch.empty(0, dtype=torch.uint8,
                                                                 device="cuda")
    c, t = am.gcm_encrypt(ks, iv, x, aad)
    assert _np(c).tobytes() == ct and _np(t).tobytes() == tag
    p, t2 = am.gcm_decrypt(ks, iv, c, aad)
    assert _np(p).tobytes() == pt and _np(t2).tobytes() == tag


# (key bytes, message bytes, AAD bytes): GHASH block counts from 1 (empty) to
# ~2^20 cover the final wave alone, one and several narrow passes, the wide
# pass over A, ragged A and C tails and zero-length parts.
CASES = [(16, 0, 0), (16, 1, 0), (16, 0, 1), (16, 15, 13), (16, 16, 16), (16, 17, 17),
         (24, 31, 0), (32, 1000, 100), (16, 16 * 62, 0), (16, 16 * 63, 16), (16, 16 * 64, 0),
         (16, 16 * 63 + 1, 15), (32, 4096 + 7, 4096 + 5), (16, 65536 + 3, 0),
         (24, 16 * 1023, 16), (16, 16 * 1024, 0), (16, (1 << 20) + 9, 33),
         (32, (1 << 22) - 5, 1 << 12),
         (16, 33, (1 << 24) + 3)]          # AAD through the wide pass, ragged A tail


@pytest.mark.parametrize("kb,n,na", CASES)
def test_gcm_matches_oracle(oracle, kb, n, na):
    g = _rng(0x6C30 + 7 * n + na + kb)
    key, iv = g.bytes(kb), g.bytes(12)
    pt = np.frombuffer(g.bytes(n), np.uint8)
    aad = g.bytes(na)
    ct_exp, tag_exp = oracle.gcm_encrypt(key, iv, aad, pt)
    ks = am.key_schedule(key)
    x = _dev(pt) if n else torch.empty(0, dtype=torch.uint8, device="cuda")
    c, t = am.gcm_encrypt(ks, iv, x, aad)
    assert np.array_equal(_np(c), ct_exp)
    assert np.array_equal(_np(t), tag_exp)
    p, t2 = am.gcm_decrypt(ks, iv, c, aad)
    assert np.array_equal(_np(p), pt) and np.array_equal(_np(t2), tag_exp)


def test_gcm_in_place_and_reused_workspace(oracle):
    g = _rng(0x6C31)
    key, iv, aad = g.bytes(16), g.bytes(12), g.bytes(40)
    pt = np.frombuffer(g.bytes(300000), np.uint8)
    ct_exp, tag_exp = oracle.gcm_encrypt(key, iv, aad, pt)
    ks = am.key_schedule(key)
    ws = torch.empty(am.gcm_workspace_bytes(len(aad), len(pt)) + 4096, dtype=torch.uint8,
                     device="cuda")
    ws.fill_(0xA5)
    buf = _dev(pt)
    _, t = am.gcm_encrypt(ks, iv, buf, aad, out=buf, ws=ws)
    assert np.array_equal(_np(buf), ct_exp) and np.array_equal(_np(t), tag_exp)
    _, t2 = am.gcm_decrypt(ks, iv, buf, aad, out=buf, ws=ws)
    assert np.array_equal(_np(buf), pt) and np.array_equal(_np(t2), tag_exp)


def test_gcm_tag_detects_changes(oracle):
    g = _rng(0x6C32)
    key, iv, aad = g.bytes(32), g.bytes(12), g.bytes(20)
    pt = np.frombuffer(g.bytes(5000), np.uint8)
    ks = am.key_schedule(key)
    c, t = am.gcm_encrypt(ks, iv, _dev(pt), aad)
    ref = _np(t)
    bad = c.clone()
    bad[4321] ^= 1
    assert not np.array_equal(_np(am.gcm_decrypt(ks, iv, bad, aad)[1]), ref)
    aad2 = bytearray(aad)
    aad2[0] ^= 0x80
    assert not np.array_equal(_np(am.gcm_decrypt(ks, iv, c, bytes(aad2))[1]), ref)
    iv2 = bytes([iv[0] ^ 1]) + iv[1:]
    assert not np.array_equal(_np(am.gcm_decrypt(ks, iv2, c, aad)[1]), ref)


@pytest.mark.parametrize("nblocks", [0, 1, 2, 63, 64, 65, 1000, 1024, 1025, 4096 * 16 + 1,
                                     (1 << 20) + 3])
def test_ghash_matches_oracle(oracle, nblocks):
    g = _rng(0x6C40 + nblocks)
    h = g.bytes(16)
    x = np.frombuffer(g.bytes(16 * nblocks), np.uint8)
    exp = oracle.ghash(h, x)
    xd = _dev(x) if nblocks else torch.empty(0, dtype=torch.uint8, device="cuda")
    assert np.array_equal(_np(am.ghash(h, xd)), exp)


def _pow(oracle, h, e):
    """H^e by square-and-multiply with the oracle's GF(2^128) product."""
    one = bytes([0x80]) + bytes(15)
    r, b = one, h
    while e:
        if e & 1:
            r = oracle.gf128_mul(r, b).tobytes()
        b = oracle.gf128_mul(b, b).tobytes()
        e >>= 1
    return r


def _xor(a, b):
    return bytes(x ^ y for x, y in zip(a, b))


def test_ghash_wide_pass_single_blocks(oracle):
    """A lone nonzero block X_i at 2^22 + 5 blocks: GHASH = X_i * H^(m-i+1)
    for positions in the first, a middle and the last lane of a pass."""
    m = (1 << 22) + 5
    g = _rng(0x6C41)
    h = g.bytes(16)
    x = torch.zeros(16 * m, dtype=torch.uint8, device="cuda")
    for i in (1, 2, 1 << 19, (1 << 19) + 1, m // 2, m - 1, m):
        blk = g.bytes(16)
        x[16 * (i - 1):16 * i] = _dev(np.frombuffer(blk, np.uint8))
        got = _np(am.ghash(h, x)).tobytes()
        x[16 * (i - 1):16 * i] = 0
        assert got == oracle.gf128_mul(blk, _pow(oracle, h, m - i + 1)).tobytes(), i


@pytest.mark.slow
def test_gcm_4gib_linearity_and_samples(oracle):
    """4 GiB AES-128-GCM: sampled ciphertext blocks against the oracle's
    keystream, and the tag difference of two messages that differ in a few
    blocks against sum_i D_i * H^(m-i+1) from the oracle's GF(2^128) product."""
    n = 4 << 30
    na = 48
    g = _rng(0x6C42)
    key, iv, aad = g.bytes(16), g.bytes(12), g.bytes(na)
    ks = am.key_schedule(key)
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    x.view(torch.int64).random_(generator=torch.Generator(device="cuda").manual_seed(5))
    out = torch.empty_like(x)
    ws = torch.empty(am.gcm_workspace_bytes(na, n), dtype=torch.uint8, device="cuda")
    _, t1 = am.gcm_encrypt(ks, iv, x, aad, out=out, ws=ws)
    t1 = _np(t1).tobytes()
    nb = n // 16
    for b in (0, 1, 12345, nb // 3, nb - 2, nb - 1):
        ks_exp = oracle.ctr_keystream_at(key, iv, 2, [b])[0]
        got = _np(out[16 * b:16 * b + 16])
        assert np.array_equal(got, ks_exp ^ _np(x[16 * b:16 * b + 16])), b
    h = oracle.ecb_encrypt(key, np.zeros(16, np.uint8)).tobytes()
    m = (na + 15) // 16 + nb + 1
    expected = bytes(16)
    for b in (0, 7, (1 << 19) - 1, 1 << 19, nb // 2 + 3, nb - 1):
        d = g.bytes(16)
        x[16 * b:16 * b + 16] ^= _dev(np.frombuffer(d, np.uint8))
        i = (na + 15) // 16 + b + 1          # 1-based GHASH position of block b
        expected = _xor(expected, oracle.gf128_mul(d, _pow(oracle, h, m - i + 1)).tobytes())
    _, t2 = am.gcm_encrypt(ks, iv, x, aad, out=out, ws=ws)
    assert _xor(t1, _np(t2).tobytes()) == expected


@pytest.mark.slow
def test_gcm_4gib_exact_tag(oracle):
    """4 GiB AES-128-GCM with the plaintext set to the oracle's own keystream
    (counters 2, 3, ...): every ciphertext byte must be 0, and the tag is then
    E(J0) ^ GHASH_A * H^(c+1) ^ L * H (c = 2^28 ciphertext blocks), computed
    from the oracle's block cipher and GF(2^128) product alone."""
    n = 4 << 30
    na = 48
    g = _rng(0x6C43)
    key, iv, aad = g.bytes(16), g.bytes(12), g.bytes(na)
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    piece = 256 << 20
    zeros = np.zeros(piece, np.uint8)
    threads = min(16, os.cpu_count() or 1)
    for off in range(0, n, piece):
        ks_piece = oracle.ctr_xcrypt(key, iv, 2 + off // 16, zeros, threads=threads)
        x[off:off + piece].copy_(torch.from_numpy(ks_piece))
    ks = am.key_schedule(key)
    out = torch.empty_like(x)
    ws = torch.empty(am.gcm_workspace_bytes(na, n), dtype=torch.uint8, device="cuda")
    _, tag = am.gcm_encrypt(ks, iv, x, aad, out=out, ws=ws)
    assert int(torch.count_nonzero(out).item()) == 0
    h = oracle.ecb_encrypt(key, np.zeros(16, np.uint8)).tobytes()
    ej0 = oracle.ecb_encrypt(key, np.frombuffer(iv + b"\0\0\0\1", np.uint8)).tobytes()
    ya = oracle.ghash(h, np.frombuffer(aad, np.uint8)).tobytes()
    c = n // 16
    lens = (8 * na).to_bytes(8, "big") + (8 * n).to_bytes(8, "big")
    expected = _xor(_xor(ej0, oracle.gf128_mul(ya, _pow(oracle, h, c + 1)).tobytes()),
                    oracle.gf128_mul(lens, h).tobytes())
    assert _np(tag).tobytes() == expected
    # decryption of the all-zero ciphertext gives the keystream back, same tag
    back, tag2 = am.gcm_decrypt(ks, iv, out, aad, out=out, ws=ws)
    assert torch.equal(back, x) and _np(tag2).tobytes() == expected

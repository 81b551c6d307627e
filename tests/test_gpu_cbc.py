"""CBC over a matrix of messages (the paper's mode, App. A1 / A4) on the GPU,
against the C oracle row by row and against the independent numpy
construction of the paper's vectorized algorithm."""
import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am
from oracle import paper_vectorized as pv

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("key_bytes", [16, 24, 32])
@pytest.mark.parametrize("nmsg,msg_bytes", [(1, 16), (1, 16 * 37), (63, 16), (64, 32),
                                            (1000, 160), (3001, 16 * 9), (129, 1024)])
def test_cbc_rows_match_oracle(oracle, key_bytes, nmsg, msg_bytes):
    g = _rng(nmsg * 31 + msg_bytes + key_bytes)
    key = g.bytes(key_bytes)
    ks = am.key_schedule(key)
    pt = np.frombuffer(g.bytes(nmsg * msg_bytes), np.uint8).reshape(nmsg, msg_bytes)
    ivs = np.frombuffer(g.bytes(16 * nmsg), np.uint8).reshape(nmsg, 16)
    x = torch.from_numpy(pt.copy()).to(DEV).view(-1)
    iv = torch.from_numpy(ivs.copy()).to(DEV).view(-1)
    ct = am.cbc_encrypt(ks, iv, x, nmsg).cpu().numpy().reshape(nmsg, msg_bytes)
    rows = range(nmsg) if nmsg <= 200 else np.linspace(0, nmsg - 1, 120).astype(int)
    for r in rows:
        assert np.array_equal(ct[r], oracle.cbc_encrypt(key, ivs[r].tobytes(), pt[r])), r
    back = am.cbc_decrypt(ks, iv, torch.from_numpy(ct.copy()).to(DEV).view(-1), nmsg)
    assert np.array_equal(back.cpu().numpy().reshape(nmsg, msg_bytes), pt)
    # one IV shared by every row (App. A1 broadcasts a single IV)
    ct1 = am.cbc_encrypt(ks, iv[:16].contiguous(), x, nmsg).cpu().numpy().reshape(nmsg, msg_bytes)
    for r in list(rows)[:20]:
        assert np.array_equal(ct1[r], oracle.cbc_encrypt(key, ivs[0].tobytes(), pt[r])), r


def test_cbc_matches_paper_vectorized():
    """The numpy construction of sec. II (N messages x M bytes, per-row IVs,
    AES-128) gives the same matrix as the GPU kernels."""
    g = _rng(2024)
    key = g.bytes(16)
    n, m = 257, 48
    P = np.frombuffer(g.bytes(n * m), np.uint8).reshape(n, m)
    V = np.frombuffer(g.bytes(16 * n), np.uint8).reshape(n, 16)
    ref = pv.PaperAES128(key)
    C = ref.cbc_encrypt(V, P)
    ks = am.key_schedule(key)
    got = am.cbc_encrypt(ks, torch.from_numpy(V.copy()).to(DEV).view(-1),
                         torch.from_numpy(P.copy()).to(DEV).view(-1), n)
    assert np.array_equal(got.cpu().numpy().reshape(n, m), C)


def test_cbc_in_place_encrypt_and_errors(oracle):
    g = _rng(7)
    key = g.bytes(16)
    ks = am.key_schedule(key)
    pt = np.frombuffer(g.bytes(50 * 64), np.uint8)
    iv = torch.from_numpy(np.frombuffer(g.bytes(16), np.uint8).copy()).to(DEV)
    x = torch.from_numpy(pt.copy()).to(DEV)
    am.cbc_encrypt(ks, iv, x, 50, out=x)
    exp = np.concatenate([oracle.cbc_encrypt(key, iv.cpu().numpy().tobytes(), pt[64 * r:64 * r + 64])
                          for r in range(50)])
    assert np.array_equal(x.cpu().numpy(), exp)
    with pytest.raises(am.AesError, match="AES_ERR_OVERLAP"):
        am.cbc_decrypt(ks, iv, x, 50, out=x)
    with pytest.raises(am.AesError, match="AES_ERR_LENGTH"):
        am.cbc_encrypt(ks, iv, torch.zeros(50 * 20, dtype=torch.uint8, device=DEV), 50)


@pytest.mark.parametrize("nmsg,msg_bytes", [((1 << 20) + 77, 16), (1_100_003, 32)])
def test_cbc_million_rows(oracle, nmsg, msg_bytes):
    """A million rows and more (every lane of the grid takes several rows,
    every thread of the decryption several blocks).  Sampled rows (the first
    and last ones, and rows on lane, workgroup and grid-stride borders)
    against the oracle in both directions; the round trip of every row on
    the device."""
    g = _rng(nmsg + msg_bytes)
    key = g.bytes(16)
    ks = am.key_schedule(key)
    pt = np.frombuffer(g.bytes(nmsg * msg_bytes), np.uint8).reshape(nmsg, msg_bytes)
    ivs = np.frombuffer(g.bytes(16 * nmsg), np.uint8).reshape(nmsg, 16)
    x = torch.from_numpy(pt.copy()).to(DEV).view(-1)
    iv = torch.from_numpy(ivs.copy()).to(DEV).view(-1)
    ct_d = am.cbc_encrypt(ks, iv, x, nmsg)
    ct = ct_d.cpu().numpy().reshape(nmsg, msg_bytes)
    rows = set(range(0, 70)) | set(range(nmsg - 70, nmsg))
    for b in (64, 256, 1024, 2048, 4096, 1 << 18, 1 << 20):
        for k in range(1, 4):
            for d in (-2, -1, 0, 1):
                r = k * b + d
                if 0 <= r < nmsg:
                    rows.add(r)
    rows |= set(int(r) for r in g.integers(0, nmsg, 1500))
    for r in sorted(rows):
        assert np.array_equal(ct[r], oracle.cbc_encrypt(key, ivs[r].tobytes(), pt[r])), r
    # decryption of unrelated ciphertext rows, against the oracle
    cr = np.frombuffer(g.bytes(nmsg * msg_bytes), np.uint8).reshape(nmsg, msg_bytes)
    dec = am.cbc_decrypt(ks, iv, torch.from_numpy(cr.copy()).to(DEV).view(-1), nmsg)
    dec = dec.cpu().numpy().reshape(nmsg, msg_bytes)
    for r in sorted(rows):
        assert np.array_equal(dec[r], oracle.cbc_decrypt(key, ivs[r].tobytes(), cr[r])), r
    back = am.cbc_decrypt(ks, iv, ct_d, nmsg)
    assert torch.equal(back, x)


@pytest.mark.parametrize("nmsg", [65536, 65537])
def test_cbc_encrypt_quad_threshold(oracle, nmsg):
    """Encryption runs four lanes per row up to 65,536 rows and one lane per
    row above: both sides of the switch, sampled rows against the oracle
    (first, last, workgroup and grid borders) and the round trip of every row."""
    msg_bytes = 48
    g = _rng(nmsg)
    key = g.bytes(24)
    ks = am.key_schedule(key)
    pt = np.frombuffer(g.bytes(nmsg * msg_bytes), np.uint8).reshape(nmsg, msg_bytes)
    ivs = np.frombuffer(g.bytes(16 * nmsg), np.uint8).reshape(nmsg, 16)
    x = torch.from_numpy(pt.copy()).to(DEV).view(-1)
    iv = torch.from_numpy(ivs.copy()).to(DEV).view(-1)
    ct_d = am.cbc_encrypt(ks, iv, x, nmsg)
    ct = ct_d.cpu().numpy().reshape(nmsg, msg_bytes)
    rows = set(range(0, 40)) | set(range(nmsg - 40, nmsg))
    for b in (16, 64, 256, 1024, 4096, 16384):
        for k in range(1, 5):
            for d in (-1, 0, 1):
                if 0 <= k * b + d < nmsg:
                    rows.add(k * b + d)
    rows |= set(int(r) for r in g.integers(0, nmsg, 300))
    for r in sorted(rows):
        assert np.array_equal(ct[r], oracle.cbc_encrypt(key, ivs[r].tobytes(), pt[r])), r
    assert torch.equal(am.cbc_decrypt(ks, iv, ct_d, nmsg), x)


def test_cbc_fig3_long_rows_sampled(oracle):
    """The Fig. 3 length sweep's largest shape: 128 messages of 1 MiB (65,536
    chained blocks per row) with per-row IVs.  Sixteen rows spread over the
    matrix (first and last included) equal the oracle's CBC encryption of
    that row byte for byte; every row decrypts back to its plaintext."""
    from concurrent.futures import ThreadPoolExecutor
    g = _rng(0xF1603)
    key = g.bytes(16)
    ks = am.key_schedule(key)
    nmsg, msg_bytes = 128, 1 << 20
    pt = np.frombuffer(g.bytes(nmsg * msg_bytes), np.uint8).reshape(nmsg, msg_bytes)
    ivs = np.frombuffer(g.bytes(16 * nmsg), np.uint8).reshape(nmsg, 16)
    x = torch.from_numpy(pt.copy()).to(DEV).view(-1)
    iv = torch.from_numpy(ivs.copy()).to(DEV).view(-1)
    ct_d = am.cbc_encrypt(ks, iv, x, nmsg)
    ct = ct_d.cpu().numpy().reshape(nmsg, msg_bytes)
    rows = sorted(set(np.linspace(0, nmsg - 1, 16).astype(int).tolist()))

    def row_ok(r):
        return np.array_equal(ct[r], oracle.cbc_encrypt(key, ivs[r].tobytes(), pt[r]))
    with ThreadPoolExecutor(16) as ex:
        bad = [r for r, ok in zip(rows, ex.map(row_ok, rows)) if not ok]
    assert not bad, bad
    back = am.cbc_decrypt(ks, iv, ct_d, nmsg)
    assert torch.equal(back, x)

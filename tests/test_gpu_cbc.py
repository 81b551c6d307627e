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

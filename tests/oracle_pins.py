"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each ``pin_*`` takes an ``Oracle`` object and raises ``AssertionError`` when the
oracle disagrees with what the paper, the mathematics or an independent source
fixes.  ``test_oracle_pins.py`` runs them on the real oracle;
``test_oracle_mutants.py`` runs them on deliberately broken builds of it and
requires every broken build to fail at least one pin.

Sources of truth used here:
* values printed in the paper (sec. II GF examples, App. A1/A4 ShiftRows index
  vectors, App. A1/A4 mix-matrix rows) -- ``golden/paper_*.txt``;
* field identities checked by brute force over all 256 / 65,536 cases;
* the independent numpy construction of the paper's vectorized algorithm
  (``oracle/paper_vectorized.py``: exhaustive-search inverses, bit-plane
  products, GF(2) matrix affine maps, row-form key schedule);
* the FIPS-197 / SP 800-38A example vectors -- ``golden/standard_vectors.txt``;
* the system OpenSSL command-line tool on seeded random inputs.
"""
from __future__ import annotations

import os

import numpy as np

import openssl_cli
from oracle import paper_vectorized as pv

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _poly_to_byte(text):
    v = 0
    for term in text.split("+"):
        if term == "1":
            v |= 1
        elif term == "x":
            v |= 2
        else:
            v |= 1 << int(term.split("^")[1])
    return v


_INDEPENDENT = {}


def independent():
    """Tables from the independent numpy construction (built once)."""
    if not _INDEPENDENT:
        table = pv.product_table()
        inv = pv.inverse_by_search(table)
        _INDEPENDENT.update(table=table, inv=inv, sbox=pv.gen_sbox(inv),
                            sbox_inv=pv.gen_sbox_inv(inv))
    return _INDEPENDENT


# ------------------------------------------------------------------ sec. II
def pin_paper_gf_examples(o):
    """sec. II: 1 + 3 = 2 and x^7 * x^5 mod 0x11B = x^7 + x^5 + x^3 + x + 1."""
    seen = set()
    for f in _lines("paper_gf_examples.txt"):
        if f[0] == "add":
            assert o.gf_add(int(f[1], 16), int(f[2], 16)) == int(f[3], 16)
        elif f[0] == "mul":
            assert o.gf_mul(int(f[1], 16), int(f[2], 16)) == int(f[3], 16)
        elif f[0] == "repr":
            # the byte is the coefficient vector of the printed polynomial
            assert int(f[1], 16) == _poly_to_byte(f[2])
        elif f[0] == "poly":
            # reduction: x^8 = x^4 + x^3 + x + 1 (the low 8 bits of the polynomial)
            assert o.gf_mul(0x80, 0x02) == int(f[1], 16) & 0xFF
        seen.add(f[0])
    assert seen == {"add", "mul", "repr", "poly"}


def pin_gf_field(o):
    """Brute force: the oracle's product equals the independent bit-plane product
    on all 65,536 pairs, and a * inv(a) = 1 for every nonzero a, inv(0) = 0."""
    ind = independent()
    mine = np.array([[o.gf_mul(a, b) for b in range(256)] for a in range(256)],
                    dtype=np.uint8)
    assert np.array_equal(mine, ind["table"])
    for a in range(1, 256):
        assert o.gf_mul(a, o.gf_inv(a)) == 1
    assert o.gf_inv(0) == 0
    assert all(o.gf_add(a, a) == 0 for a in range(256))


def pin_rcon(o):
    """App. A3: rcon(j) = x^(j-1).  The first eight are single bits (no
    reduction); x^8 reduces by 0x11B to x^4+x^3+x+1 = 0x1b, and x^9 = 0x36."""
    expected = [1 << j for j in range(8)] + [0x1B, 0x36]
    assert [o.rcon(j) for j in range(1, 11)] == expected


# ---------------------------------------------------------------- S-boxes
def pin_sbox(o):
    """App. A2: S = affine(inv(x)).  S(0) is the affine constant b = 0x63
    (inv(0) = 0); S is a permutation with no fixed and no opposite fixed
    points; S equals the independent numpy construction entry by entry."""
    s = o.sbox()
    assert s[0] == 0x63
    assert sorted(s.tolist()) == list(range(256))
    assert all(int(s[x]) != x for x in range(256))
    assert all(int(s[x]) != (x ^ 0xFF) for x in range(256))
    assert np.array_equal(s, independent()["sbox"])


def pin_inv_sbox(o):
    """App. A5: the inverse S-box, built from its own affine map, undoes S on
    all 256 bytes; S^-1(0x63) = 0 (the special case of App. A5)."""
    s, si = o.sbox(), o.inv_sbox()
    assert all(int(si[int(s[x])]) == x for x in range(256))
    assert si[0x63] == 0
    assert np.array_equal(si, independent()["sbox_inv"])


# -------------------------------------------------------------- round steps
def pin_shift_rows_paper(o):
    """App. A1 / A4 index vectors: byte dst <- byte src (1-based)."""
    rows = {f[0]: [int(v) for v in f[1:]] for f in _lines("paper_shiftrows.txt")}
    ident = np.arange(16, dtype=np.uint8)
    enc = o.shift_rows(ident)
    dec = o.inv_shift_rows(ident)
    exp_enc, exp_dec = ident.copy(), ident.copy()
    for d, s in zip(rows["enc_dst"], rows["enc_src"]):
        exp_enc[d - 1] = s - 1
    for d, s in zip(rows["dec_dst"], rows["dec_src"]):
        exp_dec[d - 1] = s - 1
    assert np.array_equal(enc, exp_enc)
    assert np.array_equal(dec, exp_dec)
    # ShiftRows applied four times is the identity.
    x = ident
    for _ in range(4):
        x = o.shift_rows(x)
    assert np.array_equal(x, ident)


def pin_mix_columns(o):
    """App. A1 / A4 mix matrices: the oracle's MixColumns equals the product by
    circ[2 3 1 1] (row printed in the paper) computed here with the independent
    product table, and the inverse matrix circ[14 11 13 9] undoes it."""
    rows = {f[0]: [int(v) for v in f[1:]] for f in _lines("paper_mix_matrices.txt")}
    table = independent()["table"]
    g = _rng(11)
    for _ in range(64):
        blk = g.integers(0, 256, 16, dtype=np.uint8)
        for name, fn in (("mix", o.mix_columns), ("inv_mix", o.inv_mix_columns)):
            row = rows[name]
            exp = np.zeros(16, np.uint8)
            for c in range(4):
                for i in range(4):
                    acc = 0
                    for j in range(4):
                        acc ^= int(table[row[(j - i) % 4], blk[4 * c + j]])
                    exp[4 * c + i] = acc
            assert np.array_equal(fn(blk), exp), name
        assert np.array_equal(o.inv_mix_columns(o.mix_columns(blk)), blk)


# ------------------------------------------------------------ full cipher
def pin_standard_vectors(o):
    """FIPS-197 App. A/B/C and SP 800-38A F.5.1/F.5.5 known answers; each ECB
    and CTR line is also run through the system OpenSSL tool when it exists
    (the key-schedule lines have no OpenSSL counterpart)."""
    kinds = set()
    checked = 0
    for f in _lines("standard_vectors.txt"):
        kinds.add(f[0])
        if f[0] == "ecb":
            key, pt, ct = (bytes.fromhex(v) for v in f[1:4])
            assert o.encrypt_block(key, pt).tobytes() == ct
            assert o.decrypt_block(key, ct).tobytes() == pt
            assert o.ecb_encrypt(key, np.frombuffer(pt, np.uint8)).tobytes() == ct
            if openssl_cli.available():
                assert openssl_cli.ecb_encrypt(key, pt).tobytes() == ct
                assert openssl_cli.ecb_decrypt(key, ct).tobytes() == pt
                checked += 1
        elif f[0] == "lastkey":
            nr, rk = o.expand_key(bytes.fromhex(f[1]))
            assert rk[:16].tobytes() == bytes.fromhex(f[1])[:16]
            assert rk[16 * nr:].tobytes() == bytes.fromhex(f[2])
        elif f[0] == "ctr":
            key, nonce = bytes.fromhex(f[1]), bytes.fromhex(f[2])
            ctr0 = int(f[3], 16)
            pt = np.frombuffer(bytes.fromhex(f[4]), np.uint8)
            assert o.ctr_xcrypt(key, nonce, ctr0, pt).tobytes() == bytes.fromhex(f[5])
            if openssl_cli.available():
                assert openssl_cli.ctr_xcrypt(key, nonce, ctr0, pt).tobytes() == bytes.fromhex(f[5])
                checked += 1
    assert kinds == {"ecb", "lastkey", "ctr"}
    assert checked == 0 or checked >= 6


def pin_paper_vectorized(o):
    """The C oracle equals the independent numpy construction of the paper's
    vectorized CBC (App. A1 / A4 semantics) on N random rows, and its ECB equals
    the CBC with zero IV and one block per row."""
    g = _rng(7)
    key = g.bytes(16)
    ref = pv.PaperAES128(key)
    nr, rk = o.expand_key(key)
    assert nr == 10 and np.array_equal(rk.reshape(11, 16), ref.K)
    P = g.integers(0, 256, (5, 37), dtype=np.uint8)     # 5 messages, padded to 48 B
    V = g.integers(0, 256, 16, dtype=np.uint8)
    C = ref.cbc_encrypt(V, P)
    for n in range(P.shape[0]):
        row = np.zeros(48, np.uint8)
        row[:37] = P[n]
        assert np.array_equal(o.cbc_encrypt(key, V.tobytes(), row), C[n])
        assert np.array_equal(o.cbc_decrypt(key, V.tobytes(), C[n]), row)
    assert np.array_equal(ref.cbc_decrypt(V, C)[:, :37], P)
    blocks = g.integers(0, 256, 16 * 9, dtype=np.uint8)
    assert np.array_equal(o.ecb_encrypt(key, blocks), ref.ecb_encrypt(blocks))
    assert np.array_equal(o.ecb_decrypt(key, blocks), ref.ecb_decrypt(blocks))


def _seeded_keys(g):
    keys = [g.bytes(n) for n in (16, 24, 32) for _ in range(2)]
    # Keys whose schedule feeds 0xff through the S-box (the saturating-index
    # reading of App. A3 would diverge exactly here).
    keys += [b"\x00" * 12 + b"\xff" * 4, b"\xff" * 16, b"\xff" * 32,
             bytes(range(8)) + b"\xff" * 16 + bytes(8)]
    return keys


def pin_openssl(o):
    """The oracle equals the system OpenSSL tool (a black box) on seeded random
    keys, nonces and data: ECB-128/192/256 both ways, CBC-128, CTR with a
    ragged tail and a counter carry."""
    assert openssl_cli.available(), "openssl command-line tool not found"
    g = _rng(0xC0FFEE)
    for key in _seeded_keys(g):
        data = np.frombuffer(g.bytes(16 * 5), np.uint8)
        ct = o.ecb_encrypt(key, data)
        assert np.array_equal(ct, openssl_cli.ecb_encrypt(key, data))
        assert np.array_equal(o.ecb_decrypt(key, data), openssl_cli.ecb_decrypt(key, data))
        nonce = g.bytes(12)
        ctr0 = int.from_bytes(g.bytes(4), "big") % (2 ** 32 - 64)
        ctr0 = ctr0 | 0xFE if key[0] & 1 else ctr0     # sometimes force a byte carry
        tail = np.frombuffer(g.bytes(16 * 7 + 9), np.uint8)
        assert np.array_equal(o.ctr_xcrypt(key, nonce, ctr0, tail),
                              openssl_cli.ctr_xcrypt(key, nonce, ctr0, tail))
        if len(key) == 16:
            iv = g.bytes(16)
            assert np.array_equal(o.cbc_encrypt(key, iv, data),
                                  openssl_cli.cbc_encrypt(key, iv, data))


# ------------------------------------------------------------------ modes
def pin_modes(o):
    """Mode identities: decrypt(encrypt(x)) = x (sec. II, decryption reverses
    the steps); CTR(P) = P + E(counter blocks) with the counter blocks built
    here byte by byte; CTR applied twice is the identity; zero-length inputs;
    error codes for bad key length, ragged ECB length and counter overflow."""
    g = _rng(5)
    for nbytes_key in (16, 24, 32):
        key = g.bytes(nbytes_key)
        data = np.frombuffer(g.bytes(16 * 33), np.uint8)
        assert np.array_equal(o.ecb_decrypt(key, o.ecb_encrypt(key, data)), data)
        nonce, ctr0 = g.bytes(12), 0xFFFFFE00 - 3
        msg = np.frombuffer(g.bytes(16 * 300 + 5), np.uint8)
        nblk = -(-msg.size // 16)
        cblocks = np.zeros((nblk, 16), np.uint8)
        for i in range(nblk):
            cblocks[i, :12] = np.frombuffer(nonce, np.uint8)
            cblocks[i, 12:] = np.frombuffer(int(ctr0 + i).to_bytes(4, "big"), np.uint8)
        ks = o.ecb_encrypt(key, cblocks.reshape(-1))[:msg.size]
        out = o.ctr_xcrypt(key, nonce, ctr0, msg)
        assert np.array_equal(out, msg ^ ks)
        assert np.array_equal(o.ctr_xcrypt(key, nonce, ctr0, out), msg)
        idx = np.array([0, 1, 7, nblk - 1], np.uint64)
        picked = cblocks[idx.astype(np.int64)].reshape(-1)
        assert np.array_equal(o.ctr_keystream_at(key, nonce, ctr0, idx),
                              o.ecb_encrypt(key, picked).reshape(-1, 16))
        assert o.ctr_xcrypt(key, nonce, 5, np.zeros(0, np.uint8)).size == 0
    for bad in (0, 15, 17, 31, 33):
        try:
            o.ecb_encrypt(b"k" * bad, np.zeros(16, np.uint8))
        except ValueError as e:
            assert "key length" in str(e)
        else:
            raise AssertionError("bad key length accepted")
    for fn in (o.ecb_encrypt, o.ecb_decrypt):
        try:
            fn(b"k" * 16, np.zeros(17, np.uint8))
        except ValueError as e:
            assert "multiple of 16" in str(e)
        else:
            raise AssertionError("ragged ECB accepted")
    # exactly 2^32 blocks of counter space is fine, one more is not
    o.ctr_xcrypt(b"k" * 16, b"n" * 12, 2 ** 32 - 2, np.zeros(32, np.uint8))
    try:
        o.ctr_xcrypt(b"k" * 16, b"n" * 12, 2 ** 32 - 2, np.zeros(33, np.uint8))
    except ValueError as e:
        assert "counter" in str(e)
    else:
        raise AssertionError("counter overflow accepted")


# -------------------------------------------------------------------- GCM
def gf128_reference(x: bytes, y: bytes) -> bytes:
    """GF(2^128) product written as integer polynomial arithmetic -- a
    different method from the oracle's shift-and-add (SP 800-38D Algorithm
    1): map each block to a polynomial (bit 0 = MSB of byte 0 = x^0),
    carry-less multiply, reduce by x^128 + x^7 + x^2 + x + 1, map back."""
    def to_poly(b):
        v = int.from_bytes(b, "big")
        return int(format(v, "0128b")[::-1], 2)

    def from_poly(p):
        return int(format(p, "0128b")[::-1], 2).to_bytes(16, "big")
    a, b = to_poly(x), to_poly(y)
    prod = 0
    while b:
        if b & 1:
            prod ^= a
        a <<= 1
        b >>= 1
    poly = (1 << 128) | 0x87
    for deg in range(prod.bit_length() - 1, 127, -1):
        if (prod >> deg) & 1:
            prod ^= poly << (deg - 128)
    return from_poly(prod)


def pin_gf128(o):
    """The oracle's GF(2^128) product equals the integer-polynomial product on
    random and structured operands; x^0 (0x80 00..) is the identity; the
    product commutes and distributes; H^(2^128) = H (Frobenius)."""
    g = _rng(128)
    one = bytes([0x80]) + bytes(15)
    cases = [(g.bytes(16), g.bytes(16)) for _ in range(40)]
    cases += [(bytes(15) + b"\x01", bytes(15) + b"\x01"), (b"\xff" * 16, b"\xff" * 16),
              (one, g.bytes(16))]
    for x, y in cases:
        assert o.gf128_mul(x, y).tobytes() == gf128_reference(x, y)
        assert o.gf128_mul(y, x).tobytes() == o.gf128_mul(x, y).tobytes()
    for _ in range(10):
        x, y, z = g.bytes(16), g.bytes(16), g.bytes(16)
        yz = bytes(a ^ b for a, b in zip(y, z))
        lhs = o.gf128_mul(x, yz)
        rhs = o.gf128_mul(x, y) ^ o.gf128_mul(x, z)
        assert np.array_equal(lhs, rhs)
        assert o.gf128_mul(one, x).tobytes() == x
    h = g.bytes(16)
    p = h
    for _ in range(128):
        p = o.gf128_mul(p, p).tobytes()
    assert p == h


def pin_ghash(o):
    """GHASH by Horner equals the sum of X_i * H^(m-i+1) built from the
    reference product, and is linear in the data."""
    g = _rng(129)
    h = g.bytes(16)
    blocks = np.frombuffer(g.bytes(16 * 7), np.uint8)
    acc = bytes(16)
    hp = h
    for i in range(6, -1, -1):
        term = gf128_reference(blocks[16 * i:16 * i + 16].tobytes(), hp)
        acc = bytes(a ^ b for a, b in zip(acc, term))
        hp = gf128_reference(hp, h)
    assert o.ghash(h, blocks).tobytes() == acc
    other = np.frombuffer(g.bytes(16 * 7), np.uint8)
    assert np.array_equal(o.ghash(h, blocks ^ other), o.ghash(h, blocks) ^ o.ghash(h, other))


def pin_gcm_vectors(o):
    """GCM specification test cases 1-4, 13, 14; decryption reproduces the
    plaintext and the same tag."""
    n = 0
    for f in _lines("gcm_vectors.txt"):
        key, iv = bytes.fromhex(f[1]), bytes.fromhex(f[2])
        aad = b"" if f[3] == "-" else bytes.fromhex(f[3])
        pt = np.frombuffer(b"" if f[4] == "-" else bytes.fromhex(f[4]), np.uint8)
        ct_exp = b"" if f[5] == "-" else bytes.fromhex(f[5])
        ct, tag = o.gcm_encrypt(key, iv, aad, pt)
        assert ct.tobytes() == ct_exp and tag.tobytes() == bytes.fromhex(f[6])
        back, tag2 = o.gcm_decrypt(key, iv, aad, ct)
        assert np.array_equal(back, pt) and np.array_equal(tag, tag2)
        n += 1
    assert n == 6
    # GCM's encryption is CTR from counter 2 (J0 = IV || 1 is kept for the tag)
    g = _rng(130)
    key, iv = g.bytes(16), g.bytes(12)
    msg = np.frombuffer(g.bytes(16 * 5 + 3), np.uint8)
    ct, tag = o.gcm_encrypt(key, iv, b"", msg)
    assert np.array_equal(ct, o.ctr_xcrypt(key, iv, 2, msg))


ALL_PINS = [pin_paper_gf_examples, pin_gf_field, pin_rcon, pin_sbox, pin_inv_sbox,
            pin_shift_rows_paper, pin_mix_columns, pin_standard_vectors,
            pin_paper_vectorized, pin_openssl, pin_modes, pin_gf128, pin_ghash,
            pin_gcm_vectors]

"""Second, independent CPU construction of the paper's vectorized algebraic AES.

TEST INFRASTRUCTURE ONLY: used by the test suite to cross-check the C oracle
(``aes_oracle.c``) on small inputs.  It shares no code with the C oracle nor with
the GPU library.

It follows sec. II of Kepner et al. (arXiv 1506.08503): N messages are the rows of
a matrix over GF(2^8) and every step of the cipher is applied to all rows at once
("vectorization").  Notation of sec. II:

    P, C : N x M plaintext / ciphertext matrices over GF(2^8)
    V    : N x 16 matrix of IVs
    K    : (R+1) x 16 key schedule (one key shared by all rows, as in App. A1)
    s    : the 256-entry S-box
    M    : the 4 x 4 mix matrix

The arithmetic is done here differently from the C oracle on purpose, so the two
cross-check each other rather than repeat each other:

* GF(2^8) products are computed on whole arrays, bit-plane by bit-plane
  (``_gf_mul_arrays``), reducing by 0x11B (sec. II);
* inverses are found by exhaustive search over the 256 x 256 product table
  (the C oracle uses a^254);
* the affine maps of App. A2 / A5 are done as GF(2) matrix products on the
  8 x 256 bit matrix of all bytes at once;
* the key schedule is written in the 16-byte row form of App. A3 (128-bit keys).

Only 128-bit keys are covered, like the paper (sec. II, App. A1-A5).
"""
from __future__ import annotations

import numpy as np

AES_POLY = 0x11B


def _gf_mul_arrays(a, b):
    """Elementwise GF(2^8) product of two uint8 arrays (broadcasting)."""
    a = np.asarray(a, dtype=np.uint16)
    b = np.asarray(b, dtype=np.uint16)
    a, b = np.broadcast_arrays(a, b)
    acc = np.zeros(a.shape, dtype=np.uint16)
    term = a.copy()
    for i in range(8):
        acc ^= np.where((b >> i) & 1, term, 0).astype(np.uint16)
        term = term << 1
        term = np.where(term & 0x100, term ^ AES_POLY, term).astype(np.uint16)
    return acc.astype(np.uint8)


def product_table():
    """256 x 256 table of GF(2^8) products."""
    x = np.arange(256, dtype=np.uint8)
    return _gf_mul_arrays(x[:, None], x[None, :])


def inverse_by_search(table=None):
    """inv[a] = the b with a*b = 1, found by exhaustive search; inv[0] = 0."""
    if table is None:
        table = product_table()
    inv = np.zeros(256, dtype=np.uint8)
    for a in range(1, 256):
        hits = np.nonzero(table[a] == 1)[0]
        assert hits.size == 1
        inv[a] = hits[0]
    return inv


def _circulant(row):
    n = len(row)
    return np.array([[row[(j - i) % n] for j in range(n)] for i in range(n)],
                    dtype=np.uint8)


def _bits_msb_first(values):
    """8 x len(values) matrix, column k = bits of values[k], MSB on top."""
    values = np.asarray(values, dtype=np.uint8)
    return np.array([(values >> (7 - k)) & 1 for k in range(8)], dtype=np.uint8)


def _bytes_from_bits_msb_first(bits):
    out = np.zeros(bits.shape[1], dtype=np.uint16)
    for k in range(8):
        out |= bits[k].astype(np.uint16) << (7 - k)
    return out.astype(np.uint8)


def gen_sbox(inv):
    """App. A2: s = A * bits(inv(x)) + b over GF(2), A = circ[1 1 1 1 1 0 0 0]."""
    A = _circulant([1, 1, 1, 1, 1, 0, 0, 0])
    b = np.array([0, 1, 1, 0, 0, 0, 1, 1], dtype=np.uint8)[:, None]
    z = (A.astype(np.int64) @ _bits_msb_first(inv).astype(np.int64) + b) % 2
    return _bytes_from_bits_msb_first(z.astype(np.uint8))


def gen_sbox_inv(inv):
    """App. A5: s^-1 = inv(A' * bits(y) + b'), A' = circ[0 1 0 1 0 0 1 0]."""
    A = _circulant([0, 1, 0, 1, 0, 0, 1, 0])
    b = np.array([0, 0, 0, 0, 0, 1, 0, 1], dtype=np.uint8)[:, None]
    y = np.arange(256, dtype=np.uint8)
    z = (A.astype(np.int64) @ _bits_msb_first(y).astype(np.int64) + b) % 2
    return inv[_bytes_from_bits_msb_first(z.astype(np.uint8))]


def gen_keys(key, n_round, s):
    """App. A3 (128-bit key): row r+1 of K from row r.

    The first four bytes of the new row are the last four bytes of the previous
    row rotated left by one byte, substituted through s, plus x^r in the first
    byte, plus the previous row's first four bytes; each later group of four adds
    the previous row's group to the new row's preceding group.
    """
    key = np.frombuffer(bytes(key), dtype=np.uint8)
    assert key.size == 16
    K = np.zeros((n_round + 1, 16), dtype=np.uint8)
    K[0] = key
    rc = 1
    for r in range(n_round):
        first = s[np.roll(K[r, 12:16], -1)]
        first = first.copy()
        first[0] ^= rc
        K[r + 1, 0:4] = K[r, 0:4] ^ first
        for g in range(1, 4):
            K[r + 1, 4 * g:4 * g + 4] = K[r, 4 * g:4 * g + 4] ^ K[r + 1, 4 * g - 4:4 * g]
        rc = int(_gf_mul_arrays(np.uint8(rc), np.uint8(2)))
    return K


def _shift_rows_gather():
    """Byte j of a shifted block comes from byte gather[j] (row r rotates left by r).

    Byte k of a block is row k % 4, column k // 4.
    """
    return np.array([(k % 4) + 4 * (((k // 4) + (k % 4)) % 4) for k in range(16)])


def _inv_shift_rows_gather():
    return np.array([(k % 4) + 4 * (((k // 4) - (k % 4)) % 4) for k in range(16)])


def _mix_all(C, M):
    """Multiply each group of 4 columns by M over GF(2^8) for all N rows at once:
    C(:, 4c:4c+4) <- (M C(:, 4c:4c+4)^T)^T."""
    out = np.zeros_like(C)
    for c in range(4):
        cols = C[:, 4 * c:4 * c + 4]                  # N x 4
        for i in range(4):
            acc = np.zeros(C.shape[0], dtype=np.uint8)
            for j in range(4):
                acc ^= _gf_mul_arrays(M[i, j], cols[:, j])
            out[:, 4 * c + i] = acc
    return out


class PaperAES128:
    """Vectorized AES-128 over N rows at once (sec. II), CBC as in App. A1/A4."""

    N_ROUND = 10

    def __init__(self, key):
        table = product_table()
        inv = inverse_by_search(table)
        self.s = gen_sbox(inv)
        self.s_inv = gen_sbox_inv(inv)
        self.K = gen_keys(key, self.N_ROUND, self.s)
        self.M = _circulant([2, 3, 1, 1])
        self.M_inv = _circulant([14, 11, 13, 9])

    def _encrypt_rows(self, X):
        """Encrypt one 16-byte block of every row (N x 16)."""
        C = X ^ self.K[0]
        g = _shift_rows_gather()
        for r in range(1, self.N_ROUND + 1):
            C = self.s[C]
            C = C[:, g]
            if r < self.N_ROUND:
                C = _mix_all(C, self.M)
            C = C ^ self.K[r]
        return C

    def _decrypt_rows(self, Y):
        g = _inv_shift_rows_gather()
        S = Y.copy()
        for r in range(self.N_ROUND, 0, -1):
            S = S ^ self.K[r]
            if r < self.N_ROUND:
                S = _mix_all(S, self.M_inv)
            S = S[:, g]
            S = self.s_inv[S]
        return S ^ self.K[0]

    def cbc_encrypt(self, V, P):
        """P: N x M uint8 (M padded with zeros to a multiple of 16), V: N x 16."""
        P = np.asarray(P, dtype=np.uint8)
        n, m = P.shape
        nblock = -(-m // 16)
        Pp = np.zeros((n, 16 * nblock), dtype=np.uint8)
        Pp[:, :m] = P
        V = np.broadcast_to(np.asarray(V, dtype=np.uint8), (n, 16)).copy()
        C = np.zeros_like(Pp)
        for b in range(nblock):
            i = slice(16 * b, 16 * b + 16)
            V = self._encrypt_rows(Pp[:, i] ^ V)
            C[:, i] = V
        return C

    def cbc_decrypt(self, V, C):
        C = np.asarray(C, dtype=np.uint8)
        n, m = C.shape
        assert m % 16 == 0
        V = np.broadcast_to(np.asarray(V, dtype=np.uint8), (n, 16)).copy()
        P = np.zeros_like(C)
        for b in range(m // 16):
            i = slice(16 * b, 16 * b + 16)
            P[:, i] = self._decrypt_rows(C[:, i]) ^ V
            V = C[:, i]
        return P

    def ecb_encrypt(self, P):
        """ECB = the CBC of App. A1 with a zero IV and one block per row."""
        P = np.asarray(P, dtype=np.uint8).reshape(-1, 16)
        return self.cbc_encrypt(np.zeros(16, np.uint8), P).reshape(-1)

    def ecb_decrypt(self, C):
        C = np.asarray(C, dtype=np.uint8).reshape(-1, 16)
        return self.cbc_decrypt(np.zeros(16, np.uint8), C).reshape(-1)

"""ctypes front end of the C oracle (``aes_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never does.

All buffers are host numpy uint8 arrays.  ``threads > 1`` splits a CTR / ECB job
into contiguous block ranges run on Python threads (ctypes releases the GIL for
the duration of each foreign call); the arithmetic per block is unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aes_oracle.c")
LIB_PATH = os.path.join(_HERE, "libaes_oracle.so")

_lib = None

ERRORS = {-1: "bad key length", -2: "length not a multiple of 16",
          -3: "counter range exceeds 2^32 blocks"}


def build(force: bool = True, src: str = _SRC, out: str = LIB_PATH) -> str:
    """Compile the oracle with gcc (plain -O2, no SIMD intrinsics)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Werror",
                               "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _bind(lib):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    c = ctypes
    lib.oracle_gf_add.argtypes = [c.c_uint8, c.c_uint8]
    lib.oracle_gf_add.restype = c.c_uint8
    lib.oracle_gf_mul.argtypes = [c.c_uint8, c.c_uint8]
    lib.oracle_gf_mul.restype = c.c_uint8
    lib.oracle_gf_pow.argtypes = [c.c_uint8, c.c_uint]
    lib.oracle_gf_pow.restype = c.c_uint8
    lib.oracle_gf_inv.argtypes = [c.c_uint8]
    lib.oracle_gf_inv.restype = c.c_uint8
    lib.oracle_sbox_entry.argtypes = [c.c_uint8]
    lib.oracle_sbox_entry.restype = c.c_uint8
    lib.oracle_inv_sbox_entry.argtypes = [c.c_uint8]
    lib.oracle_inv_sbox_entry.restype = c.c_uint8
    lib.oracle_sbox.argtypes = [u8p]
    lib.oracle_inv_sbox.argtypes = [u8p]
    lib.oracle_rcon.argtypes = [c.c_int]
    lib.oracle_rcon.restype = c.c_uint8
    lib.oracle_num_rounds.argtypes = [c.c_int]
    lib.oracle_num_rounds.restype = c.c_int
    lib.oracle_expand_key.argtypes = [u8p, c.c_int, u8p]
    lib.oracle_expand_key.restype = c.c_int
    for name in ("oracle_encrypt_block", "oracle_decrypt_block"):
        f = getattr(lib, name)
        f.argtypes = [u8p, c.c_int, u8p, u8p]
        f.restype = c.c_int
    for name in ("oracle_ecb_encrypt", "oracle_ecb_decrypt"):
        f = getattr(lib, name)
        f.argtypes = [u8p, c.c_int, u8p, u8p, c.c_size_t]
        f.restype = c.c_int
    for name in ("oracle_apply_shift_rows", "oracle_apply_inv_shift_rows",
                 "oracle_apply_mix_columns", "oracle_apply_inv_mix_columns"):
        getattr(lib, name).argtypes = [u8p]
    lib.oracle_ctr_xcrypt.argtypes = [u8p, c.c_int, u8p, c.c_uint32, u8p, u8p,
                                      c.c_size_t]
    lib.oracle_ctr_xcrypt.restype = c.c_int
    lib.oracle_ctr_keystream_at.argtypes = [u8p, c.c_int, u8p, c.c_uint32,
                                            c.POINTER(c.c_uint64), c.c_size_t, u8p]
    lib.oracle_ctr_keystream_at.restype = c.c_int
    for name in ("oracle_cbc_encrypt", "oracle_cbc_decrypt"):
        f = getattr(lib, name)
        f.argtypes = [u8p, c.c_int, u8p, u8p, u8p, c.c_size_t]
        f.restype = c.c_int
    lib.oracle_gf128_mul.argtypes = [u8p, u8p, u8p]
    lib.oracle_ghash.argtypes = [u8p, u8p, c.c_size_t, u8p]
    for name in ("oracle_gcm_encrypt", "oracle_gcm_decrypt"):
        f = getattr(lib, name)
        f.argtypes = [u8p, c.c_int, u8p, u8p, c.c_size_t, u8p, u8p, c.c_size_t, u8p]
        f.restype = c.c_int
    return lib


def load(path: str = LIB_PATH):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path != LIB_PATH:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check(rc):
    if rc != 0:
        raise ValueError("oracle: " + ERRORS.get(rc, "error %d" % rc))


class Oracle:
    """Thin object wrapper so tests can swap in a deliberately broken build."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- field and tables ---------------------------------------------------
    def gf_add(self, a, b):
        return int(self.lib.oracle_gf_add(a, b))

    def gf_mul(self, a, b):
        return int(self.lib.oracle_gf_mul(a, b))

    def gf_pow(self, a, e):
        return int(self.lib.oracle_gf_pow(a, e))

    def gf_inv(self, a):
        return int(self.lib.oracle_gf_inv(a))

    def sbox(self):
        out, p = _u8(np.zeros(256, np.uint8))
        self.lib.oracle_sbox(p)
        return out

    def inv_sbox(self):
        out, p = _u8(np.zeros(256, np.uint8))
        self.lib.oracle_inv_sbox(p)
        return out

    def rcon(self, j):
        return int(self.lib.oracle_rcon(j))

    def expand_key(self, key):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        rk, rp = _u8(np.zeros(240, np.uint8))
        nr = self.lib.oracle_expand_key(kp, key.size, rp)
        _check(0 if nr > 0 else nr)
        return nr, rk[:16 * (nr + 1)].copy()

    def _step(self, fn, block):
        blk, bp = _u8(np.array(np.frombuffer(bytes(block), np.uint8)))
        fn(bp)
        return blk

    def shift_rows(self, block):
        return self._step(self.lib.oracle_apply_shift_rows, block)

    def inv_shift_rows(self, block):
        return self._step(self.lib.oracle_apply_inv_shift_rows, block)

    def mix_columns(self, block):
        return self._step(self.lib.oracle_apply_mix_columns, block)

    def inv_mix_columns(self, block):
        return self._step(self.lib.oracle_apply_inv_mix_columns, block)

    # -- block / modes -------------------------------------------------------
    def encrypt_block(self, key, block):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        blk, bp = _u8(np.frombuffer(bytes(block), np.uint8))
        out, op = _u8(np.zeros(16, np.uint8))
        _check(self.lib.oracle_encrypt_block(kp, key.size, bp, op))
        return out

    def decrypt_block(self, key, block):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        blk, bp = _u8(np.frombuffer(bytes(block), np.uint8))
        out, op = _u8(np.zeros(16, np.uint8))
        _check(self.lib.oracle_decrypt_block(kp, key.size, bp, op))
        return out

    def _ecb(self, fn, key, data, threads):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        data, dp = _u8(data)
        out = np.zeros_like(data)
        if data.size % 16:
            _check(-2)
        nblk = data.size // 16
        threads = max(1, min(threads, nblk))

        def run(lo, hi):
            if hi <= lo:
                return 0
            src = data[16 * lo:16 * hi]
            dst = out[16 * lo:16 * hi]
            return fn(kp, key.size, src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                      dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), src.size)

        bounds = [nblk * t // threads for t in range(threads + 1)]
        if threads == 1:
            _check(run(0, nblk) if nblk else (fn(kp, key.size, dp, dp, 0)))
        else:
            with ThreadPoolExecutor(threads) as ex:
                for rc in ex.map(run, bounds[:-1], bounds[1:]):
                    _check(rc)
        return out

    def ecb_encrypt(self, key, data, threads=1):
        return self._ecb(self.lib.oracle_ecb_encrypt, key, data, threads)

    def ecb_decrypt(self, key, data, threads=1):
        return self._ecb(self.lib.oracle_ecb_decrypt, key, data, threads)

    def ctr_xcrypt(self, key, nonce, ctr0, data, threads=1):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        nonce, np_ = _u8(np.frombuffer(bytes(nonce), np.uint8))
        assert nonce.size == 12
        data, dp = _u8(data)
        out = np.zeros_like(data)
        nblk = -(-data.size // 16)
        threads = max(1, min(threads, nblk))
        bounds = [nblk * t // threads for t in range(threads + 1)]

        def run(lo, hi):
            if hi <= lo:
                return 0
            src = data[16 * lo:min(16 * hi, data.size)]
            dst = out[16 * lo:min(16 * hi, data.size)]
            return self.lib.oracle_ctr_xcrypt(
                kp, key.size, np_, ctr0 + lo,
                src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), src.size)

        if threads == 1:
            _check(run(0, nblk) if nblk else 0)
        else:
            with ThreadPoolExecutor(threads) as ex:
                for rc in ex.map(run, bounds[:-1], bounds[1:]):
                    _check(rc)
        return out

    def ctr_keystream_at(self, key, nonce, ctr0, idx):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        nonce, np_ = _u8(np.frombuffer(bytes(nonce), np.uint8))
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        ks, kp2 = _u8(np.zeros((idx.size, 16), np.uint8))
        _check(self.lib.oracle_ctr_keystream_at(
            kp, key.size, np_, ctr0,
            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), idx.size, kp2))
        return ks

    def _cbc(self, fn, key, iv, data):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        iv, ivp = _u8(np.frombuffer(bytes(iv), np.uint8))
        data, dp = _u8(data)
        out, op = _u8(np.zeros_like(data))
        _check(fn(kp, key.size, ivp, dp, op, data.size))
        return out

    def cbc_encrypt(self, key, iv, data):
        return self._cbc(self.lib.oracle_cbc_encrypt, key, iv, data)

    def cbc_decrypt(self, key, iv, data):
        return self._cbc(self.lib.oracle_cbc_decrypt, key, iv, data)

    # -- GCM (SP 800-38D) -------------------------------------------------------
    def gf128_mul(self, x, y):
        x, xp = _u8(np.frombuffer(bytes(x), np.uint8))
        y, yp = _u8(np.frombuffer(bytes(y), np.uint8))
        out, op = _u8(np.zeros(16, np.uint8))
        self.lib.oracle_gf128_mul(xp, yp, op)
        return out

    def ghash(self, h, blocks):
        h, hp = _u8(np.frombuffer(bytes(h), np.uint8))
        blocks, bp = _u8(blocks)
        assert blocks.size % 16 == 0
        out, op = _u8(np.zeros(16, np.uint8))
        self.lib.oracle_ghash(hp, bp, blocks.size // 16, op)
        return out

    def _gcm(self, fn, key, iv, aad, data):
        key, kp = _u8(np.frombuffer(bytes(key), np.uint8))
        iv, ivp = _u8(np.frombuffer(bytes(iv), np.uint8))
        assert iv.size == 12
        aad, ap = _u8(np.frombuffer(bytes(aad), np.uint8) if not isinstance(aad, np.ndarray)
                      else aad)
        data, dp = _u8(data)
        out, op = _u8(np.zeros_like(data))
        tag, tp = _u8(np.zeros(16, np.uint8))
        _check(fn(kp, key.size, ivp, ap, aad.size, dp, op, data.size, tp))
        return out, tag

    def gcm_encrypt(self, key, iv, aad, data):
        """(ciphertext, tag)"""
        return self._gcm(self.lib.oracle_gcm_encrypt, key, iv, aad, data)

    def gcm_decrypt(self, key, iv, aad, data):
        """(plaintext, tag computed over the received ciphertext)"""
        return self._gcm(self.lib.oracle_gcm_decrypt, key, iv, aad, data)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default

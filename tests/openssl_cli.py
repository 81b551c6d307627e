"""Independent known answers from the system OpenSSL command-line tool.

The tool is run as a black box (``openssl enc``); nothing of it is read or
linked.  Its CTR mode increments the whole 128-bit counter block, which equals
the 12-byte nonce + 32-bit big-endian counter format on every input whose
counter range stays below 2^32 (the only inputs the library accepts).
"""
from __future__ import annotations

import shutil
import subprocess

import numpy as np

OPENSSL = shutil.which("openssl")


def available() -> bool:
    return OPENSSL is not None


def _enc(cipher: str, key: bytes, data: bytes, iv: bytes | None = None,
         decrypt: bool = False) -> bytes:
    cmd = [OPENSSL, "enc", "-" + cipher, "-K", key.hex(), "-nosalt"]
    if iv is not None:
        cmd += ["-iv", iv.hex()]
    if cipher.endswith("ecb") or cipher.endswith("cbc"):
        cmd += ["-nopad"]
    if decrypt:
        cmd += ["-d"]
    res = subprocess.run(cmd, input=bytes(data), stdout=subprocess.PIPE,
                         stderr=subprocess.PIPE, check=True)
    return res.stdout


def _name(key: bytes, mode: str) -> str:
    return "aes-%d-%s" % (8 * len(key), mode)


def ecb_encrypt(key: bytes, data) -> np.ndarray:
    return np.frombuffer(_enc(_name(key, "ecb"), key, bytes(data)), np.uint8)


def ecb_decrypt(key: bytes, data) -> np.ndarray:
    return np.frombuffer(_enc(_name(key, "ecb"), key, bytes(data), decrypt=True), np.uint8)


def cbc_encrypt(key: bytes, iv: bytes, data) -> np.ndarray:
    return np.frombuffer(_enc(_name(key, "cbc"), key, bytes(data), iv=iv), np.uint8)


def ctr_xcrypt(key: bytes, nonce: bytes, ctr0: int, data) -> np.ndarray:
    iv = bytes(nonce) + int(ctr0).to_bytes(4, "big")
    return np.frombuffer(_enc(_name(key, "ctr"), key, bytes(data), iv=iv), np.uint8)

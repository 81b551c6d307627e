"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random bytes and sizes only; it holds none of the cipher's
arithmetic.  Every generator is numpy PCG64 with a fixed seed, so the GPU library
and the CPU oracle are fed the very same bytes.

Workloads (sizes follow the paper's framing of "many independent 16-byte blocks"
and "many short messages", sec. II-III; the paper's own inputs were synthetic
messages, sec. IV):

* ``small``     AES-128 ECB + CTR, 1 MiB uniform plaintext (65,536 blocks)
* ``stream``    AES-128 CTR, 4 GiB uniform plaintext in one buffer
* ``batched``   10,000 messages, own key and nonce each, log-uniform length
                1 B .. 1 MiB, packed at 16-byte aligned offsets
* ``dbcolumn``  AES-256 ECB over 2^26 int64 values (Zipf s = 1.1 over 2^20
                distinct values), each zero-padded to a 16-byte block
* ``serving``   Poisson arrivals, lognormal sizes (median 4 KiB, sigma 2,
                clipped to [1, 16 MiB]), 1,024 keys (half 128-bit, half 256-bit)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_SMALL = 0xAE501
SEED_STREAM = 0xAE502
SEED_BATCHED = 0xAE503
SEED_DBCOLUMN = 0xAE504
SEED_SERVING = 0xAE505

MiB = 1 << 20
GiB = 1 << 30


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_bytes(g: np.random.Generator, n: int) -> np.ndarray:
    return np.frombuffer(g.bytes(n), dtype=np.uint8).copy() if n else np.zeros(0, np.uint8)


# --------------------------------------------------------------- one stream
@dataclass
class StreamInputs:
    key: bytes
    nonce: bytes
    ctr0: int
    nbytes: int
    seed: int

    def plaintext_chunks(self, chunk: int = 256 * MiB):
        """Yield (offset, uint8 array) pieces of the plaintext, in order."""
        g = rng(self.seed + 1)
        off = 0
        while off < self.nbytes:
            n = min(chunk, self.nbytes - off)
            yield off, random_bytes(g, n)
            off += n

    def plaintext(self) -> np.ndarray:
        out = np.empty(self.nbytes, dtype=np.uint8)
        for off, piece in self.plaintext_chunks():
            out[off:off + piece.size] = piece
        return out


def stream_inputs(seed: int, nbytes: int, key_bytes: int = 16, ctr0: int = 0) -> StreamInputs:
    g = rng(seed)
    key = g.bytes(key_bytes)
    nonce = g.bytes(12)
    return StreamInputs(key=key, nonce=nonce, ctr0=ctr0, nbytes=nbytes, seed=seed)


def small_inputs() -> StreamInputs:
    """1 MiB, AES-128, one key and nonce, ctr0 = 0."""
    return stream_inputs(SEED_SMALL, MiB)


def stream_4g_inputs(nbytes: int = 4 * GiB) -> StreamInputs:
    """4 GiB, AES-128, one key and nonce, ctr0 = 0."""
    return stream_inputs(SEED_STREAM, nbytes)


# ------------------------------------------------------------ many messages
@dataclass
class Batch:
    keys: np.ndarray        # nmsg x key_bytes uint8
    nonces: np.ndarray      # nmsg x 12 uint8
    ctr0: np.ndarray        # nmsg uint32
    lengths: np.ndarray     # nmsg int64
    offsets: np.ndarray     # nmsg int64, 16-byte aligned offsets into the packed buffer
    total: int              # packed buffer size in bytes
    seed: int

    def packed_plaintext(self) -> np.ndarray:
        g = rng(self.seed + 1)
        buf = np.zeros(self.total, dtype=np.uint8)
        for off, n in zip(self.offsets.tolist(), self.lengths.tolist()):
            buf[off:off + n] = random_bytes(g, n)
        return buf


def log_uniform_lengths(g: np.random.Generator, n: int, max_len: int) -> np.ndarray:
    """L = clip(round(exp(U(0, ln max_len))), 1, max_len)."""
    u = g.uniform(0.0, math.log(max_len), size=n)
    return np.clip(np.rint(np.exp(u)), 1, max_len).astype(np.int64)


def pack_offsets(lengths: np.ndarray, align: int = 16) -> tuple[np.ndarray, int]:
    padded = (lengths + align - 1) // align * align
    offsets = np.zeros(lengths.size, dtype=np.int64)
    if lengths.size:
        offsets[1:] = np.cumsum(padded)[:-1]
    return offsets, int(padded.sum())


def batched_inputs(nmsg: int = 10_000, max_len: int = MiB, seed: int = SEED_BATCHED,
                   key_bytes: int = 16) -> Batch:
    g = rng(seed)
    lengths = log_uniform_lengths(g, nmsg, max_len)
    keys = random_bytes(g, nmsg * key_bytes).reshape(nmsg, key_bytes)
    nonces = random_bytes(g, nmsg * 12).reshape(nmsg, 12)
    offsets, total = pack_offsets(lengths)
    return Batch(keys=keys, nonces=nonces, ctr0=np.zeros(nmsg, np.uint32),
                 lengths=lengths, offsets=offsets, total=total, seed=seed)


# ----------------------------------------------------------- database column
@dataclass
class DbColumn:
    key: bytes              # 32-byte AES-256 key
    values: np.ndarray      # ndistinct distinct int64 values
    ranks: np.ndarray       # nrows int64 in [0, ndistinct)
    seed: int

    def column(self) -> np.ndarray:
        return self.values[self.ranks]


def zipf_ranks(g: np.random.Generator, nrows: int, ndistinct: int, s: float,
               chunk: int = 1 << 24) -> np.ndarray:
    """Truncated Zipf(s) on {1..ndistinct} by inverse CDF; returns 0-based ranks."""
    w = np.arange(1, ndistinct + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(nrows, dtype=np.int64)
    for lo in range(0, nrows, chunk):
        hi = min(nrows, lo + chunk)
        out[lo:hi] = np.searchsorted(cdf, g.uniform(size=hi - lo), side="right")
    return np.minimum(out, ndistinct - 1)


def distinct_int64(g: np.random.Generator, n: int) -> np.ndarray:
    vals = np.unique(g.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max,
                                size=n, dtype=np.int64, endpoint=True))
    while vals.size < n:
        more = g.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max,
                          size=n - vals.size, dtype=np.int64, endpoint=True)
        vals = np.unique(np.concatenate([vals, more]))
    return g.permutation(vals[:n])


def dbcolumn_inputs(nrows: int = 1 << 26, ndistinct: int = 1 << 20, s: float = 1.1,
                    seed: int = SEED_DBCOLUMN) -> DbColumn:
    g = rng(seed)
    key = g.bytes(32)
    values = distinct_int64(g, ndistinct)
    ranks = zipf_ranks(g, nrows, ndistinct, s)
    return DbColumn(key=key, values=values, ranks=ranks, seed=seed)


def pack_int64_blocks(col: np.ndarray) -> np.ndarray:
    """Each int64 little-endian in bytes 0..7 of its own 16-byte block, zeros after."""
    blocks = np.zeros((col.size, 2), dtype="<i8")
    blocks[:, 0] = col
    return blocks.view(np.uint8).reshape(-1)


# ----------------------------------------------------------------- serving
@dataclass
class RequestStream:
    arrival_s: np.ndarray   # scheduled arrival times, seconds from start
    sizes: np.ndarray       # bytes
    key_slot: np.ndarray    # index into the key set
    nonces: np.ndarray      # n x 12
    keys: list              # key set (bytes), 16- or 32-byte keys
    seed: int

    def payload(self, i: int) -> np.ndarray:
        g = rng((self.seed << 24) ^ (i + 1))
        return random_bytes(g, int(self.sizes[i]))


def serving_inputs(nreq: int, rate_per_s: float, nkeys: int = 1024,
                   median: int = 4096, sigma: float = 2.0, max_size: int = 16 * MiB,
                   seed: int = SEED_SERVING) -> RequestStream:
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=nreq)
    arrival = np.cumsum(gaps) - gaps[0]
    sizes = np.clip(np.rint(g.lognormal(math.log(median), sigma, size=nreq)), 1,
                    max_size).astype(np.int64)
    key_slot = g.integers(0, nkeys, size=nreq)
    nonces = random_bytes(g, nreq * 12).reshape(nreq, 12)
    keys = [g.bytes(16 if k < nkeys // 2 else 32) for k in range(nkeys)]
    return RequestStream(arrival_s=arrival, sizes=sizes, key_slot=key_slot,
                         nonces=nonces, keys=keys, seed=seed)

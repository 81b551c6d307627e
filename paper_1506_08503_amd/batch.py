"""Many messages with their own keys in one launch (aes_ctr_xcrypt_batched).

``DeviceBatch`` packs a set of messages into one device buffer at 16-byte
aligned offsets, expands their keys on the device (aes_expand_keys_device) and
builds the segment table the persistent kernel reads.  It can run the batch as
one launch, as a captured HIP graph, or -- for comparison -- as a loop of plain
aes_ctr_xcrypt calls, one per message.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import aesmi
from .workloads import Batch


def segment_table(in_off, out_off, nbytes, key_slot, ctr0, nonces) -> np.ndarray:
    """Host segment records (numpy, aes_segment_t layout)."""
    n = len(nbytes)
    t = np.zeros(n, dtype=aesmi.segment_dtype())
    t["in_off"] = in_off
    t["out_off"] = out_off
    t["nbytes"] = nbytes
    t["key_slot"] = key_slot
    t["ctr0"] = ctr0
    t["nonce"] = np.asarray(nonces, dtype=np.uint8).reshape(n, 12)
    return t


def workspace(nsegs: int, device) -> torch.Tensor:
    """A 256-byte aligned workspace for nsegs segments."""
    need = aesmi.batched_workspace_bytes(nsegs)
    raw = torch.empty(need + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + need]


class DeviceBatch:
    """One batch of messages resident on the device."""

    def __init__(self, batch: Batch, device="cuda", plaintext: np.ndarray | None = None):
        self.batch = batch
        self.device = torch.device(device)
        pt = batch.packed_plaintext() if plaintext is None else plaintext
        self.x = torch.from_numpy(pt).to(self.device)
        self.out = torch.zeros_like(self.x)
        keys = torch.from_numpy(np.ascontiguousarray(batch.keys)).to(self.device)
        self.ks_table = aesmi.expand_keys_device(keys)
        n = batch.lengths.size
        self.host_segs = segment_table(batch.offsets, batch.offsets, batch.lengths,
                                       np.arange(n, dtype=np.uint32), batch.ctr0, batch.nonces)
        self.segs = torch.from_numpy(self.host_segs.view(np.uint8).copy()).to(self.device)
        self.ws = workspace(n, self.device)
        self._graph = None

    @property
    def nbytes(self) -> int:
        return int(self.batch.lengths.sum())

    def run(self, tune=None):
        aesmi.ctr_xcrypt_batched(self.segs, self.ks_table, self.x, self.out, self.ws, tune)
        return self.out

    def status(self) -> int:
        return aesmi.batched_read_status(self.ws)

    def graph(self, tune=None) -> aesmi.BatchedGraph:
        if self._graph is None:
            self._graph = aesmi.BatchedGraph(self.segs, self.ks_table, self.x, self.out,
                                             self.ws, tune)
        return self._graph

    def run_plain_loop(self):
        """Every message through its own aes_ctr_xcrypt launch (the baseline
        the persistent kernel replaces)."""
        l = aesmi.lib()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        xb, ob, kb = self.x.data_ptr(), self.out.data_ptr(), self.ks_table.data_ptr()
        nonces = [ctypes.create_string_buffer(bytes(n), 12) for n in self.batch.nonces]
        f = l.aes_ctr_xcrypt
        with torch.cuda.device(self.device):
            for i, (off, n) in enumerate(zip(self.batch.offsets.tolist(),
                                             self.batch.lengths.tolist())):
                st = f(kb + aesmi.SCHEDULE_BYTES * i, nonces[i], int(self.batch.ctr0[i]),
                       xb + off, ob + off, n, stream)
                if st:
                    raise aesmi.AesError(st, "aes_ctr_xcrypt")
        return self.out

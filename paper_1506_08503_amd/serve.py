"""Continuous-batching request loop for AES-CTR encryption requests.

Requests arrive over time (open-loop arrival schedule), each with its own key
(from a key set), nonce, first counter and payload.  The loop

* admits requests in arrival order while the device bytes they hold (input
  plus output) fit an HBM budget; a request larger than the whole budget is
  rejected;
* keeps expanded key schedules in a fixed-size device cache (LRU; a schedule
  used by an in-flight batch is pinned and never evicted); misses are expanded
  on the device (aes_expand_keys_device) right before the batch that needs
  them;
* closes a batch when a launch slot is free and either nothing is running,
  the queued bytes reach a size threshold or the oldest queued request has
  waited longer than a time window; each batch is one aes_ctr_xcrypt_batched
  launch over a segment table on one of several streams, so batches overlap
  on the device and requests keep being admitted while others run;
* retires batches as their events complete, releasing budget and key pins,
  and records per-request latency = completion - scheduled arrival.

The many-rows-at-once framing is the paper's (sec. II-III: many short
messages, each with its own IV and key); the scheduling is this library's.

The executor (what runs a batch) is pluggable: ``GpuExecutor`` launches the
HIP kernels; the CPU tests drive the same loop with an executor of their own
(tests/test_serve_cpu.py) to check admission, caching and accounting without a
GPU.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------- requests
@dataclass
class Requests:
    """Struct-of-arrays request set, sorted by arrival time."""
    arrival: np.ndarray      # seconds from the start, non-decreasing
    key_id: np.ndarray       # index into the key set
    nonce: np.ndarray        # n x 12 uint8
    ctr0: np.ndarray         # uint32
    size: np.ndarray         # bytes
    in_off: np.ndarray       # byte offset of the payload in the input pool (16-aligned)

    def __len__(self):
        return int(self.size.size)


def requests_from_stream(rs, pool_bytes: int, seed: int = 1) -> Requests:
    """Place the payloads of a workloads.RequestStream in an input pool of
    pool_bytes bytes (random 16-aligned offsets; payloads may share bytes)."""
    g = np.random.Generator(np.random.PCG64(seed))
    size = np.minimum(rs.sizes, pool_bytes).astype(np.int64)
    room = (pool_bytes - size) // 16
    in_off = (g.integers(0, np.iinfo(np.int64).max, size=size.size) % (room + 1)) * 16
    return Requests(arrival=np.asarray(rs.arrival_s, np.float64),
                    key_id=np.asarray(rs.key_slot, np.int64), nonce=rs.nonces,
                    ctr0=np.zeros(size.size, np.uint32), size=size, in_off=in_off)


# ---------------------------------------------------------------- key cache
class KeyCache:
    """Which keys of the key set have their schedule in which cache slot.

    Bookkeeping only (host side); the executor owns the device table.  A slot
    is pinned once per in-flight batch that uses it."""

    def __init__(self, nslots: int, nkeys: int):
        self.nslots = nslots
        self.slot_of = np.full(nkeys, -1, np.int64)
        self.key_of = np.full(nslots, -1, np.int64)
        self.last_use = np.zeros(nslots, np.int64)
        self.pins = np.zeros(nslots, np.int64)
        self.tick = 0
        self.hits = 0
        self.misses = 0

    def acquire(self, key_ids: np.ndarray):
        """Slots for a batch's keys.  Returns (slot per request, distinct slots,
        [(slot, key_id) to fill]) or None when too few slots are unpinned."""
        uniq = np.unique(key_ids)
        slot_u = self.slot_of[uniq]
        have = slot_u >= 0
        nmiss = int((~have).sum())
        if nmiss:
            # unpinned slots that do not hold a key this batch hits
            free = self.pins == 0
            free[slot_u[have]] = False
            if int(free.sum()) < nmiss:
                return None
        return self._acquire_unique(key_ids, uniq, slot_u)

    def max_prefix(self, key_ids: np.ndarray) -> int:
        """Largest k such that acquire(key_ids[:k]) can succeed: the missing
        keys of the prefix must fit into the unpinned slots that do not hold a
        key the prefix hits."""
        if key_ids.size == 0:
            return 0
        _, first = np.unique(key_ids, return_index=True)
        new = np.zeros(key_ids.size, np.int64)
        new[first] = 1
        slot = self.slot_of[key_ids]
        miss = new * (slot < 0)
        hit_free = new * ((slot >= 0) & (self.pins[np.maximum(slot, 0)] == 0))
        need = np.cumsum(miss + hit_free)
        return int(np.searchsorted(need, int((self.pins == 0).sum()), "right"))

    def take(self, key_ids: np.ndarray, row_cap: int | None = None):
        """max_prefix and acquire in one pass (one sort of the keys): returns
        (k, acquire(key_ids[:k])), k = 0 with None when not even the first
        request fits.  With row_cap, the prefix takes at most that many of
        the unpinned slots."""
        if key_ids.size == 0:
            return 0, None
        uniq, first = np.unique(key_ids, return_index=True)
        slot_u = self.slot_of[uniq]
        # a distinct key takes an unpinned slot if it misses, or if it hits a
        # slot nobody has pinned (it is pinned now); in order of first use
        needs = (slot_u < 0) | (self.pins[np.maximum(slot_u, 0)] == 0)
        order = np.argsort(first, kind="stable")
        cum = np.cumsum(needs[order])
        limit = int((self.pins == 0).sum())
        if row_cap is not None:
            limit = min(limit, int(row_cap))
        m = int(np.searchsorted(cum, limit, "right"))
        if m == 0:
            return 0, None
        if m == uniq.size:
            k = int(key_ids.size)
        else:
            k = int(first[order[m]])
            keep = first < k
            uniq, slot_u = uniq[keep], slot_u[keep]
        return k, self._acquire_unique(key_ids[:k], uniq, slot_u)

    def _acquire_unique(self, key_ids, uniq, slot_u):
        """acquire() given the distinct keys and their current slots: misses
        take empty slots first, then the least recently used unpinned ones."""
        have = slot_u >= 0
        missing = uniq[~have]
        if missing.size:
            candidates = np.nonzero(self.pins == 0)[0]
            keep = np.zeros(self.nslots, bool)
            keep[slot_u[have]] = True
            candidates = candidates[~keep[candidates]]
            assert candidates.size >= missing.size
            order = np.lexsort((self.last_use[candidates], self.key_of[candidates] >= 0))
            victims = candidates[order[:missing.size]]
            old = self.key_of[victims]
            self.slot_of[old[old >= 0]] = -1
            self.key_of[victims] = missing
            self.slot_of[missing] = victims
        self.tick += 1
        slots = self.slot_of[uniq]
        self.last_use[slots] = self.tick
        self.pins[slots] += 1
        per_req = self.slot_of[key_ids]
        nmiss_req = int(np.isin(key_ids, missing).sum()) if missing.size else 0
        self.misses += nmiss_req
        self.hits += int(key_ids.size) - nmiss_req
        fills = list(zip(self.slot_of[missing].tolist(), missing.tolist()))
        return per_req, slots, fills

    def release(self, slots: np.ndarray):
        self.pins[slots] -= 1
        assert np.all(self.pins >= 0)


# ---------------------------------------------------------------- out ring
class OutRing:
    """The output area as a ring: batches take contiguous byte ranges in
    submission order and give them back as they retire, in any order; space
    is reused once every range before it has been given back.  Ranges are
    never empty.  Allocation moves forward and goes back to offset 0 only
    when a range does not fit before the end, so an area as large as all the
    outputs together is never reused.  (The same rules as the library's
    loop.)"""

    def __init__(self, cap: int):
        self.cap = int(cap)
        self.head = 0
        self.wrapped = False
        self.live: deque = deque()      # [off, len, freed] in allocation order
        self.used = 0
        self.peak = 0

    def max_alloc(self) -> int:
        if not self.live:
            return self.cap
        tail = self.live[0][0]
        if self.wrapped:
            return tail - self.head
        return max(self.cap - self.head, tail)

    def alloc(self, n: int) -> int:
        if not self.live:
            off, self.wrapped = (self.head if self.cap - self.head >= n else 0), False
        elif not self.wrapped and self.cap - self.head >= n:
            off = self.head
        elif not self.wrapped:
            off, self.wrapped = 0, True
        else:
            off = self.head
        self.head = off + n
        self.live.append([off, n, False])
        self.used += n
        self.peak = max(self.peak, self.used)
        return off

    def release(self, off: int):
        for r in self.live:
            if r[0] == off and not r[2]:
                r[2] = True
                self.used -= r[1]
                break
        while self.live and self.live[0][2]:
            self.live.popleft()
        if not self.live:
            self.wrapped = False
        elif self.wrapped and self.live[0][0] < self.head:
            self.wrapped = False


# -------------------------------------------------------------------- batches
@dataclass
class Batch:
    first: int                  # request index range [first, last)
    last: int
    nbytes: int                 # payload bytes
    held: int                   # budget bytes held (input + output)
    slots: np.ndarray           # distinct key slots pinned
    handle: object = None
    out_off: np.ndarray = None  # output offset of each request in the batch buffer
    out_base: int = 0           # offset of the batch's range in the output ring


class ServedResults:
    """Outputs of a run, materialized on demand (request i -> a view into the
    output buffer of the batch that served it; None when rejected)."""

    def __init__(self, executor, n):
        self.ex = executor
        self.batch_of = np.full(n, -1, np.int64)
        self.index_in = np.zeros(n, np.int64)
        self.handles = []

    def add(self, handle, first, last):
        self.batch_of[first:last] = len(self.handles)
        self.index_in[first:last] = np.arange(last - first)
        self.handles.append(handle)

    def __len__(self):
        return self.batch_of.size

    def __getitem__(self, i):
        b = int(self.batch_of[i])
        if b < 0:
            return None
        return self.ex.output(self.handles[b], int(self.index_in[i]))


@dataclass
class Stats:
    completed: int = 0
    rejected: int = 0
    bytes: int = 0
    batches: int = 0
    elapsed_s: float = 0.0
    latency_s: np.ndarray = field(default_factory=lambda: np.zeros(0))
    admission_wait_s: np.ndarray = field(default_factory=lambda: np.zeros(0))
    key_hits: int = 0
    key_misses: int = 0
    max_inflight: int = 0
    max_held: int = 0
    max_out_used: int = 0

    def summary(self, skip: int = 0) -> dict:
        """Counts and rates of the whole run; latency percentiles over the
        requests from index `skip` on (the ones after a warm-up period)."""
        lat = self.latency_s[skip:]
        lat = lat[np.isfinite(lat)]
        q = (lambda p: float(np.percentile(lat, p)) * 1e3) if lat.size else (lambda p: None)
        return {"requests": self.completed, "rejected": self.rejected,
                "GBps": self.bytes / self.elapsed_s / 1e9 if self.elapsed_s else None,
                "req_per_s": self.completed / self.elapsed_s if self.elapsed_s else None,
                "p50_ms": q(50), "p99_ms": q(99), "max_ms": q(100),
                "mean_batch": self.completed / max(self.batches, 1), "batches": self.batches,
                "key_hit_rate": self.key_hits / max(self.key_hits + self.key_misses, 1),
                "max_inflight": self.max_inflight, "max_held_bytes": self.max_held}


class Server:
    """The request loop (see the module docstring)."""

    def __init__(self, executor, key_cache: KeyCache, hbm_budget: int,
                 max_batch_bytes: int = 64 << 20, max_batch_reqs: int = 8192,
                 window_s: float = 25e-6, clock=time.perf_counter,
                 out_bytes: int | None = None, row_cap: int | None = None, on_batch=None):
        """out_bytes: size of the output ring (None: unbounded); row_cap: key
        cache rows one batch may take (None: all unpinned ones); on_batch(first,
        count, results): consumer of a completed batch, called before its
        output range is reused."""
        self.ex = executor
        self.kc = key_cache
        self.budget = hbm_budget
        self.max_batch_bytes = max_batch_bytes
        self.max_batch_reqs = max_batch_reqs
        self.window_s = window_s
        self.clock = clock
        self.out_bytes = out_bytes
        self.row_cap = row_cap
        self.on_batch = on_batch

    @staticmethod
    def footprint(size: np.ndarray) -> np.ndarray:
        """Device bytes a request holds while in flight: its input and its
        16-byte padded output."""
        return size + (size + 15) // 16 * 16

    def run(self, reqs: Requests, realtime: bool = True) -> tuple[Stats, ServedResults]:
        n = len(reqs)
        fp = self.footprint(reqs.size)
        outsz = (reqs.size + 15) // 16 * 16
        ring_cap = self.out_bytes if self.out_bytes is not None else int(outsz.sum()) + 16
        ring = OutRing(ring_cap)
        complete = np.full(n, np.nan)
        admitted = np.full(n, np.nan)
        results = ServedResults(self.ex, n)
        st = Stats()
        held = 0
        inflight: deque[Batch] = deque()
        qh = 0          # first request not yet admitted
        t0 = self.clock()
        while qh < n or inflight:
            now = self.clock() - t0
            arrived = n if not realtime else int(np.searchsorted(reqs.arrival, now, "right"))
            # retire finished batches (in completion order per slot)
            progressed = False
            for b in list(inflight):
                if self.ex.done(b.handle):
                    inflight.remove(b)
                    tdone = self.clock() - t0
                    complete[b.first:b.last] = tdone
                    results.add(b.handle, b.first, b.last)
                    if self.on_batch is not None:
                        self.on_batch(b.first, b.last - b.first, results)
                    held -= b.held
                    self.kc.release(b.slots)
                    ring.release(b.out_base)
                    self.ex.release(b.handle)
                    st.completed += b.last - b.first
                    st.bytes += b.nbytes
                    progressed = True
            # reject what can never fit
            while qh < arrived and (fp[qh] > self.budget or outsz[qh] > ring_cap):
                st.rejected += 1
                complete[qh] = np.inf
                qh += 1
                progressed = True
            if qh < arrived and self.ex.free_slots() > 0:
                queued_bytes = int(reqs.size[qh:arrived].sum())
                oldest_wait = now - reqs.arrival[qh] if realtime else 0.0
                if (not inflight or queued_bytes >= self.max_batch_bytes
                        or oldest_wait >= self.window_s or arrived == n):
                    b = self._form_batch(reqs, fp, outsz, qh, arrived, held, ring)
                    if b is not None:
                        admitted[b.first:b.last] = self.clock() - t0
                        b.handle = self.ex.submit(reqs, b.first, b.last, b.per_req_slots,
                                                  b.fills, out_base=b.out_base)
                        held += b.held
                        inflight.append(b)
                        st.batches += 1
                        st.max_inflight = max(st.max_inflight, len(inflight))
                        st.max_held = max(st.max_held, held)
                        qh = b.last
                        progressed = True
            if not progressed:
                self.ex.idle()
        st.elapsed_s = self.clock() - t0
        ok = np.isfinite(complete)
        st.latency_s = np.where(ok, complete - reqs.arrival, np.inf)
        st.admission_wait_s = np.where(ok, admitted - reqs.arrival, np.inf)
        st.key_hits, st.key_misses = self.kc.hits, self.kc.misses
        st.max_out_used = ring.peak
        return st, results

    def _form_batch(self, reqs, fp, outsz, qh, arrived, held, ring):
        """Largest FIFO prefix of the queue within the budget, the free output
        range, the batch limits and the key cache."""
        room = self.budget - held
        cum_fp = np.cumsum(fp[qh:arrived])
        cum_out = np.cumsum(outsz[qh:arrived])
        cum_b = np.cumsum(reqs.size[qh:arrived])
        k = int(np.searchsorted(cum_fp, room, "right"))
        k = min(k, int(np.searchsorted(cum_out, ring.max_alloc(), "right")))
        k = min(k, int(np.searchsorted(cum_b, self.max_batch_bytes, "right")) or 1,
                self.max_batch_reqs, arrived - qh)
        if k == 0:
            return None
        k, got = self.kc.take(reqs.key_id[qh:qh + k], self.row_cap)
        if k == 0:
            return None
        per_req, slots, fills = got
        b = Batch(first=qh, last=qh + k, nbytes=int(cum_b[k - 1]), held=int(cum_fp[k - 1]),
                  slots=slots, out_base=ring.alloc(int(cum_out[k - 1])))
        b.per_req_slots = per_req
        b.fills = fills
        return b


# ------------------------------------------------------------------ executors
class GpuExecutor:
    """Runs batches with aes_ctr_xcrypt_batched on `nstreams` streams.

    Per stream it owns a workspace, pinned host staging for the segment table
    and for missing keys, and their device copies, so a batch costs two small
    host-to-device copies, at most three key-expansion launches (one per key
    length), one scatter into the key table and the two batched kernels."""

    def __init__(self, pool, keys: list, nslots: int, nstreams: int = 2,
                 max_segs: int = 8192, tune=None, out_arena_bytes: int = 0):
        import torch
        from . import aesmi
        from .batch import workspace
        self.torch, self.am = torch, aesmi
        self.pool = pool
        self.dev = pool.device
        self.keys = keys
        self.key_len = np.array([len(k) for k in keys], np.int64)
        key_pad = np.zeros((len(keys), 32), np.uint8)
        for i, k in enumerate(keys):
            key_pad[i, :len(k)] = np.frombuffer(k, np.uint8)
        self.key_pad = key_pad
        self.table = torch.zeros((nslots, aesmi.SCHEDULE_BYTES), dtype=torch.uint8,
                                 device=self.dev)
        self.tune = tune
        self.max_segs = max_segs
        sb = aesmi.SEGMENT_BYTES
        self.slots = []
        for _ in range(nstreams):
            self.slots.append({
                "stream": torch.cuda.Stream(self.dev),
                "ws": workspace(max_segs, self.dev),
                "segs_h": torch.empty(max_segs * sb, dtype=torch.uint8, pin_memory=True),
                "segs_d": torch.empty(max_segs * sb, dtype=torch.uint8, device=self.dev),
                "keys_h": torch.empty(max_segs * 40 + 8, dtype=torch.uint8, pin_memory=True),
                "keys_d": torch.empty(max_segs * 40 + 8, dtype=torch.uint8, device=self.dev),
                "sched_d": torch.empty((max_segs, aesmi.SCHEDULE_BYTES), dtype=torch.uint8,
                                       device=self.dev),
                "busy": False})
        # The buffers above are checked once here; each batch then calls the
        # library directly with their pointers (the checked Python wrappers
        # cost tens of microseconds of host time per batch).
        for t, name in ((pool, "pool"), (self.table, "key table")):
            aesmi._dev_u8(t, name)
        self.lib = aesmi.lib()
        self.table_ptr = ctypes.c_void_p(self.table.data_ptr())
        self.pool_ptr = ctypes.c_void_p(pool.data_ptr())
        tn = aesmi._tune(tune)
        self.tune_ref = ctypes.byref(tn) if tn else None
        self._tune_keep = tn
        for sl in self.slots:
            # one batch per slot at a time: its events and staging are reused
            # once the batch has been released
            sl["ev"] = torch.cuda.Event()
            sl["kev"] = torch.cuda.Event()
            sl["segs_tab"] = sl["segs_h"].numpy().view(aesmi.segment_dtype())
            sl["stream_ptr"] = ctypes.c_void_p(sl["stream"].cuda_stream)
            sl["ws_ptr"] = ctypes.c_void_p(sl["ws"].data_ptr())
            sl["segs_ptr"] = ctypes.c_void_p(sl["segs_d"].data_ptr())
        # key slot -> (stream slot, event) of an in-flight batch that filled it
        self.filled_by = {}
        # Batch outputs are carved from one preallocated arena while it lasts
        # (a fresh allocation per batch cost ~70 us of host time, a quarter
        # of a batch's submission); past its end each batch gets its own
        # buffer.  Outputs stay valid for the executor's lifetime either way.
        self.arena = (torch.empty(out_arena_bytes, dtype=torch.uint8, device=self.dev)
                      if out_arena_bytes else None)
        self.arena_used = 0

    def free_slots(self):
        return sum(not s["busy"] for s in self.slots)

    def _fill_keys(self, slot, fills):
        """Expand the missing keys into their cache slots on this stream."""
        torch, am = self.torch, self.am
        n = len(fills)
        sl = np.array([f[0] for f in fills], np.int64)
        kid = np.array([f[1] for f in fills], np.int64)
        order = np.argsort(self.key_len[kid], kind="stable")
        sl, kid = sl[order], kid[order]
        lens = self.key_len[kid]
        # staging: the keys of each length packed back to back, then the n
        # int64 cache slots (8-byte aligned), in one host-to-device copy
        raw = slot["keys_h"].numpy()
        groups, pos = [], 0
        for kb in (16, 24, 32):
            lo, hi = int(np.searchsorted(lens, kb)), int(np.searchsorted(lens, kb, "right"))
            if hi > lo:
                raw[pos:pos + (hi - lo) * kb] = self.key_pad[kid[lo:hi], :kb].reshape(-1)
                groups.append((kb, lo, hi, pos))
                pos += (hi - lo) * kb
        ipos = (pos + 7) // 8 * 8
        raw[ipos:ipos + 8 * n] = sl.astype("<i8").view(np.uint8)
        slot["keys_d"][:ipos + 8 * n].copy_(slot["keys_h"][:ipos + 8 * n], non_blocking=True)
        kbase = slot["keys_d"].data_ptr()
        sched = slot["sched_d"]
        for kb, lo, hi, p in groups:
            am._check(self.lib.aes_expand_keys_device(
                ctypes.c_void_p(kbase + p), kb, hi - lo,
                ctypes.c_void_p(sched[lo:hi].data_ptr()), slot["stream_ptr"]),
                "aes_expand_keys_device")
        idx = slot["keys_d"][ipos:ipos + 8 * n].view(torch.int64)
        self.table.index_copy_(0, idx, sched[:n])

    def submit(self, reqs, first, last, key_slots, fills, out_base=None):
        """Launch one batch.  Its outputs go to a buffer of the executor's own
        (carved from the arena while it lasts); out_base, the loop's ring
        offset, is not used: results stay valid for the executor's life."""
        torch, am = self.torch, self.am
        slot = next(s for s in self.slots if not s["busy"])
        n = last - first
        if n > self.max_segs:
            raise ValueError("batch larger than max_segs")
        slot["busy"] = True
        size = reqs.size[first:last]
        pad = (size + 15) // 16 * 16
        out_off = np.zeros(n, np.int64)
        np.cumsum(pad[:-1], out=out_off[1:])
        total = int(pad.sum())
        # the segment table is written straight into the pinned staging
        tab = slot["segs_tab"][:n]
        tab["in_off"] = reqs.in_off[first:last]
        tab["out_off"] = out_off
        tab["nbytes"] = size
        tab["key_slot"] = key_slots
        tab["ctr0"] = reqs.ctr0[first:last]
        tab["nonce"] = reqs.nonce[first:last]
        s = slot["stream"]
        with torch.cuda.stream(s):
            out = self._out_buffer(max(total, 16))
            # schedules another stream's in-flight batch is still writing
            if self.filled_by:
                used = np.zeros(self.table.shape[0], bool)
                used[key_slots] = True
                for ks, fb in self.filled_by.items():
                    if fb[0] is not slot and used[ks]:
                        s.wait_event(fb[1])
            if fills:
                self._fill_keys(slot, fills)
                slot["kev"].record(s)
                for sl, _ in fills:
                    self.filled_by[sl] = (slot, slot["kev"])
            db = slot["segs_d"][:n * am.SEGMENT_BYTES]
            db.copy_(slot["segs_h"][:n * am.SEGMENT_BYTES], non_blocking=True)
            am._check(self.lib.aes_ctr_xcrypt_batched(
                slot["segs_ptr"], n, self.table_ptr, self.table.shape[0], self.pool_ptr,
                ctypes.c_void_p(out.data_ptr()), self.tune_ref, slot["ws_ptr"],
                slot["ws"].numel(), slot["stream_ptr"]), "aes_ctr_xcrypt_batched")
            slot["ev"].record(s)
        return {"slot": slot, "event": slot["ev"], "out": out, "out_off": out_off,
                "size": size, "fills": [f[0] for f in fills]}

    def _out_buffer(self, nbytes):
        if self.arena is not None:
            lo = self.arena_used
            hi = lo + (nbytes + 255) // 256 * 256
            if hi <= self.arena.numel():
                self.arena_used = hi
                return self.arena[lo:lo + nbytes]
        return self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.dev)

    def done(self, h):
        return h["event"].query()

    def output(self, h, j):
        o = int(h["out_off"][j])
        return h["out"][o:o + int(h["size"][j])]

    def release(self, h):
        h["slot"]["busy"] = False
        for sl in h["fills"]:
            fb = self.filled_by.get(sl)
            if fb is not None and fb[0] is h["slot"]:
                del self.filled_by[sl]

    def idle(self):
        pass


# ------------------------------------------------------------- native loop
class NativeResults:
    """Outputs of a native run: request i -> a view into the output area
    (None when rejected)."""

    def __init__(self, out, out_off, size):
        self.out, self.out_off, self.size = out, out_off, size

    def __len__(self):
        return int(self.size.size)

    def __getitem__(self, i):
        o = int(self.out_off[i])
        if o == np.iinfo(np.uint64).max:
            return None
        return self.out[o:o + int(self.size[i])]


def _request_table(reqs: Requests):
    from . import aesmi
    tab = np.zeros(len(reqs), dtype=aesmi.serve_request_dtype())
    tab["arrival_s"] = reqs.arrival
    tab["in_off"] = reqs.in_off
    tab["nbytes"] = reqs.size
    tab["key_id"] = reqs.key_id
    tab["ctr0"] = reqs.ctr0
    tab["nonce"] = reqs.nonce
    return tab


def _key_arrays(keys: list):
    keys32 = np.zeros((len(keys), 32), np.uint8)
    klen = np.zeros(len(keys), np.uint8)
    for i, k in enumerate(keys):
        keys32[i, :len(k)] = np.frombuffer(k, np.uint8)
        klen[i] = len(k)
    return keys32, klen


def _stats_of(st, lat, n):
    return Stats(completed=int(st.completed), rejected=int(st.rejected), bytes=int(st.bytes),
                 batches=int(st.batches), elapsed_s=float(st.elapsed_s), latency_s=lat,
                 admission_wait_s=np.zeros(n), key_hits=int(st.key_hits),
                 key_misses=int(st.key_misses), max_inflight=int(st.max_inflight),
                 max_held=int(st.max_held), max_out_used=int(st.max_out_used))


class NativeServer:
    """aes_server_create / _run / _destroy: the library's request loop set up
    once (key table, streams, staging) for many runs on the current device;
    the key cache carries over from run to run.  on_batch(first, count,
    out_off) is called as each batch completes (see run_native)."""

    def __init__(self, keys: list, nslots: int, nstreams: int = 2, hbm_budget: int = 4 << 30,
                 max_batch_reqs: int = 8192, max_batch_bytes: int = 64 << 20,
                 window_s: float = 25e-6, realtime: bool = True, on_batch=None):
        from . import aesmi
        self._am = aesmi
        self.keys = keys
        self._keys32, self._klen = _key_arrays(keys)
        self._errors = []
        self._off = None
        self._cb = aesmi.SERVE_BATCH_FN()
        if on_batch is not None:
            def _cb(user, first, count):
                try:
                    on_batch(int(first), int(count), self._off)
                except BaseException as e:     # an exception cannot cross the C frame
                    self._errors.append(e)
            self._cb = aesmi.SERVE_BATCH_FN(_cb)
        self._prm = aesmi.ServeParams(nslots, nstreams, max_batch_reqs, 1 if realtime else 0,
                                      hbm_budget, max_batch_bytes, window_s, self._cb, None)
        h = ctypes.c_void_p()
        aesmi._check(aesmi.lib().aes_server_create(
            self._keys32.ctypes.data, self._klen.ctypes.data, len(keys), ctypes.byref(self._prm),
            ctypes.byref(h)), "aes_server_create")
        self._h = h

    def run(self, pool, reqs: Requests, out=None):
        """Play one trace; returns (Stats, NativeResults) as run_native."""
        import torch
        am = self._am
        if not self._h:
            raise RuntimeError("server is closed")
        am._dev_u8(pool, "pool")
        n = len(reqs)
        tab = _request_table(reqs)
        if out is None:
            need = int(((reqs.size + 15) // 16 * 16).sum())
            out = torch.empty(max(need, 16), dtype=torch.uint8, device=pool.device)
        am._dev_u8(out, "output area")
        lat = np.empty(n, np.float64)
        self._off = off = np.empty(n, np.uint64)
        self._errors.clear()
        st = am.ServeStats()
        with torch.cuda.device(pool.device):
            torch.cuda.synchronize(pool.device)
            am._check(am.lib().aes_server_run(
                self._h, tab.ctypes.data, n, pool.data_ptr(), pool.numel(), out.data_ptr(),
                out.numel(), lat.ctypes.data, off.ctypes.data, ctypes.byref(st)),
                "aes_server_run")
        if self._errors:
            raise self._errors[0]
        return _stats_of(st, lat, n), NativeResults(out, off, reqs.size)

    def close(self):
        if self._h:
            self._am._check(self._am.lib().aes_server_destroy(self._h), "aes_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_native(pool, keys: list, reqs: Requests, nslots: int, nstreams: int = 2,
               hbm_budget: int = 4 << 30, max_batch_reqs: int = 8192,
               max_batch_bytes: int = 64 << 20, window_s: float = 25e-6,
               realtime: bool = True, out=None, on_batch=None):
    """The same request loop as Server with GpuExecutor, run in the library
    (aes_serve_run): admission, the key-schedule cache, batch formation and
    launches happen in C++ without returning to Python per batch.  Returns
    (Stats, NativeResults).  `out` (uint8 device tensor) is the output ring;
    by default one that holds every request's 16-padded output, so nothing
    is reused and every result is still there afterwards.  With a smaller
    ring, on_batch(first, count, out_off) is called as each batch completes
    (out_off: the offsets filled so far) and must copy out what it needs
    before it returns."""
    import torch
    from . import aesmi
    aesmi._dev_u8(pool, "pool")
    n = len(reqs)
    tab = _request_table(reqs)
    keys32, klen = _key_arrays(keys)
    need = int(((reqs.size + 15) // 16 * 16).sum())
    if out is None:
        out = torch.empty(max(need, 16), dtype=torch.uint8, device=pool.device)
    aesmi._dev_u8(out, "output area")
    lat = np.empty(n, np.float64)
    off = np.empty(n, np.uint64)
    errors = []
    cb = aesmi.SERVE_BATCH_FN()
    if on_batch is not None:
        def _cb(user, first, count):
            try:
                on_batch(int(first), int(count), off)
            except BaseException as e:     # an exception cannot cross the C frame
                errors.append(e)
        cb = aesmi.SERVE_BATCH_FN(_cb)
    prm = aesmi.ServeParams(nslots, nstreams, max_batch_reqs, 1 if realtime else 0,
                            hbm_budget, max_batch_bytes, window_s, cb, None)
    st = aesmi.ServeStats()
    with torch.cuda.device(pool.device):
        torch.cuda.synchronize(pool.device)
        aesmi._check(aesmi.lib().aes_serve_run(
            tab.ctypes.data, n, keys32.ctypes.data, klen.ctypes.data, len(keys),
            pool.data_ptr(), pool.numel(), out.data_ptr(), out.numel(), ctypes.byref(prm),
            lat.ctypes.data, off.ctypes.data, ctypes.byref(st)), "aes_serve_run")
    if errors:
        raise errors[0]
    return _stats_of(st, lat, n), NativeResults(out, off, reqs.size)

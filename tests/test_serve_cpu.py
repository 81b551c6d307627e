"""The serving loop's host logic on the CPU, with the oracle as the executor.

Admission by HBM budget, FIFO order, rejection of requests that can never fit,
the key-schedule cache (LRU eviction, pinning while in flight, no stale slot
ever handed out), latency accounting, and that every served result equals the
oracle's CTR of that request alone.
"""
import numpy as np
import pytest

from paper_1506_08503_amd import serve
from paper_1506_08503_amd import workloads as wl


class StepClock:
    """Deterministic clock: every reading advances time by dt."""

    def __init__(self, dt=2e-6):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


class OracleExecutor:
    """CPU executor for tests: results from the CPU oracle, completion after a
    modelled device time (launch latency + bytes / rate) on the server clock."""

    def __init__(self, oracle, pool: np.ndarray, keys: list, nslots: int, clock,
                 nstreams: int = 2, latency_s: float = 20e-6, rate_Bps: float = 1e9):
        self.o, self.pool, self.keys = oracle, pool, keys
        self.clock = clock
        self.latency, self.rate = latency_s, rate_Bps
        self.nstreams = nstreams
        self.busy = 0
        self.resident = {}      # key slot -> key id whose schedule is "on the device"
        self.fill_log = []
        self.next_free = 0.0

    def free_slots(self):
        return self.nstreams - self.busy

    def submit(self, reqs, first, last, key_slots, fills, out_base=None):
        self.busy += 1
        for sl, kid in fills:
            self.resident[sl] = kid
            self.fill_log.append((sl, kid))
        outs = []
        for j, i in enumerate(range(first, last)):
            kid = self.resident[int(key_slots[j])]
            assert kid == reqs.key_id[i], "key cache handed out a stale slot"
            a, n = int(reqs.in_off[i]), int(reqs.size[i])
            outs.append(self.o.ctr_xcrypt(self.keys[kid], reqs.nonce[i].tobytes(),
                                          int(reqs.ctr0[i]), self.pool[a:a + n]))
        start = max(self.clock(), self.next_free)
        t_done = start + self.latency + int(reqs.size[first:last].sum()) / self.rate
        self.next_free = t_done
        return {"t": t_done, "outs": outs}

    def done(self, h):
        return self.clock() >= h["t"]

    def output(self, h, j):
        return h["outs"][j]

    def release(self, h):
        self.busy -= 1

    def idle(self):
        pass


def make_requests(n=300, nkeys=20, pool_bytes=1 << 20, rate=2e5, seed=3, big=()):
    rs = wl.serving_inputs(n, rate, nkeys=nkeys, median=1024, sigma=1.5, max_size=64 << 10,
                           seed=seed)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=seed)
    for i, size in big:
        reqs.size[i] = size
        reqs.in_off[i] = 0
    g = np.random.Generator(np.random.PCG64(seed))
    pool = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    return rs, reqs, pool


def run(oracle, reqs, pool, keys, nslots=4, budget=256 << 10, **kw):
    clock = StepClock()
    kc = serve.KeyCache(nslots, len(keys))
    ex = OracleExecutor(oracle, pool, keys, nslots, clock, latency_s=30e-6, rate_Bps=2e9)
    srv = serve.Server(ex, kc, budget, clock=clock, **kw)
    st, res = srv.run(reqs)
    return st, res, kc, ex


def test_results_equal_standalone(oracle):
    rs, reqs, pool = make_requests()
    st, res, kc, ex = run(oracle, reqs, pool, rs.keys)
    assert st.completed == len(reqs) and st.rejected == 0
    for i in range(len(reqs)):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(), 0,
                                pool[a:a + n])
        assert np.array_equal(res[i], exp), i
    assert np.all(np.isfinite(st.latency_s)) and np.all(st.latency_s > 0)
    assert np.all(st.admission_wait_s >= 0)


def test_budget_and_fifo(oracle):
    rs, reqs, pool = make_requests(rate=5e6)            # arrivals faster than service
    budget = 200 << 10
    st, res, kc, ex = run(oracle, reqs, pool, rs.keys, budget=budget)
    assert st.max_held <= budget
    assert st.max_inflight <= 2
    # admitted in arrival order
    adm = st.admission_wait_s + reqs.arrival
    assert np.all(np.diff(adm) >= -1e-12)
    s = st.summary()
    assert s["requests"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_oversize_rejected(oracle):
    budget = 128 << 10
    rs, reqs, pool = make_requests(big=[(10, 100 << 10), (20, 64 << 10)])
    st, res, kc, ex = run(oracle, reqs, pool, rs.keys, budget=budget)
    # 100 KiB in + 100 KiB out > 128 KiB: rejected; 64 KiB + 64 KiB fits exactly
    assert st.rejected == 1 and res[10] is None and res[20] is not None
    assert np.isinf(st.latency_s[10])
    a = int(reqs.in_off[20])
    assert np.array_equal(res[20], oracle.ctr_xcrypt(rs.keys[reqs.key_id[20]],
                                                     reqs.nonce[20].tobytes(), 0,
                                                     pool[a:a + (64 << 10)]))


def test_key_cache_evicts_and_refills(oracle):
    rs, reqs, pool = make_requests(n=400, nkeys=30)
    st, res, kc, ex = run(oracle, reqs, pool, rs.keys, nslots=3, max_batch_reqs=8)
    assert st.key_misses > 0 and st.key_hits > 0
    assert st.key_hits + st.key_misses == st.completed
    assert np.all(kc.pins == 0)
    # some slot was refilled with a different key over time
    by_slot = {}
    for sl, kid in ex.fill_log:
        by_slot.setdefault(sl, set()).add(kid)
    assert any(len(v) > 1 for v in by_slot.values())


def test_key_cache_lru_and_pins():
    kc = serve.KeyCache(3, 10)
    a = kc.acquire(np.array([1, 2, 1]))
    assert a is not None and len(a[2]) == 2
    kc.release(a[1])
    b = kc.acquire(np.array([3]))                  # fills the last empty slot
    kc.release(b[1])
    c = kc.acquire(np.array([2]))                  # hit: key 2 becomes most recent
    assert c[2] == []
    kc.release(c[1])
    d = kc.acquire(np.array([4]))                  # evicts LRU = key 1
    assert kc.slot_of[1] == -1 and kc.slot_of[2] >= 0 and kc.slot_of[3] >= 0
    # with every slot pinned a miss cannot be served
    e = kc.acquire(np.array([2, 3]))
    assert e is not None
    assert kc.acquire(np.array([7])) is None
    kc.release(d[1])
    kc.release(e[1])
    assert np.all(kc.pins == 0)
    with pytest.raises(AssertionError):
        kc.release(e[1])


def test_key_cache_max_prefix_is_exact():
    """max_prefix(ids) is the largest k for which acquire(ids[:k]) succeeds."""
    g = np.random.Generator(np.random.PCG64(8))
    for trial in range(200):
        kc = serve.KeyCache(6, 15)
        held = []
        for _ in range(int(g.integers(0, 4))):
            got = kc.acquire(g.integers(0, 15, size=int(g.integers(1, 4))))
            if got is not None and g.random() < 0.6:
                held.append(got[1])
            elif got is not None:
                kc.release(got[1])
        ids = g.integers(0, 15, size=12)
        k = kc.max_prefix(ids)
        for j in range(ids.size + 1):
            snap = (kc.slot_of.copy(), kc.key_of.copy(), kc.last_use.copy(), kc.pins.copy(),
                    kc.tick, kc.hits, kc.misses)
            ok = kc.acquire(ids[:j]) is not None if j else True
            (kc.slot_of, kc.key_of, kc.last_use, kc.pins, kc.tick, kc.hits, kc.misses) = snap
            assert ok == (j <= k), (trial, j, k)


def test_summary_skips_warmup():
    """Latency percentiles can leave out the first requests of a run (its
    warm-up); counts and rates still cover the whole run."""
    st = serve.Stats(completed=6, bytes=600, batches=2, elapsed_s=1e-3)
    st.latency_s = np.array([9e-3, 8e-3, 1e-3, 1e-3, 2e-3, np.inf])
    s_all, s_late = st.summary(), st.summary(skip=2)
    assert s_all["max_ms"] == pytest.approx(9.0)
    assert s_late["max_ms"] == pytest.approx(2.0) and s_late["p50_ms"] == pytest.approx(1.0)
    assert s_late["requests"] == s_all["requests"] == 6
    assert s_late["GBps"] == s_all["GBps"]


def test_key_cache_take_equals_max_prefix_then_acquire():
    """take() is max_prefix() followed by acquire() of that prefix: same
    prefix length, same slots and fills, same cache state afterwards."""
    g = np.random.Generator(np.random.PCG64(12))
    for trial in range(300):
        nslots, nkeys = int(g.integers(1, 9)), int(g.integers(1, 25))
        a, b = serve.KeyCache(nslots, nkeys), serve.KeyCache(nslots, nkeys)
        held = []
        for step in range(int(g.integers(1, 8))):
            ids = g.integers(0, nkeys, size=int(g.integers(0, 14)))
            k_ref = a.max_prefix(ids)
            ref = a.acquire(ids[:k_ref]) if k_ref else None
            k, got = b.take(ids)
            assert k == k_ref, (trial, step)
            if k:
                for x, y in zip(ref[:2], got[:2]):
                    assert np.array_equal(x, y), (trial, step)
                assert ref[2] == got[2]
                held.append(ref[1])
            for name in ("slot_of", "key_of", "last_use", "pins"):
                assert np.array_equal(getattr(a, name), getattr(b, name)), (trial, step, name)
            assert (a.tick, a.hits, a.misses) == (b.tick, b.hits, b.misses)
            if held and g.random() < 0.5:
                sl = held.pop(int(g.integers(0, len(held))))
                a.release(sl)
                b.release(sl)

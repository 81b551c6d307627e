"""The library's serving loop (csrc/serve_loop.hpp, the code aes_serve_run
runs, built here with g++ against a simulated device, no GPU) against the
Python loop serve.Server driven by the same simulated device and clock.

On random traces both must cut the same batches (first request, count,
output-ring offset, key rows filled), give every request the same latency and
report the same counters -- with budgets, output rings and key caches small
enough that admission waits on each of them, and with "no limit" values of
2^64 - 1 for the budget and the batch size (which must not wrap around and
stall the loop).  The output ring alone is checked against its own rules on
random allocate/free sequences: live ranges never overlap and stay inside
the area, and whatever max_alloc() reports can be allocated."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1506_08503_amd import serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1506_08503_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
U64_MAX = 2 ** 64 - 1

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = tmp_path_factory.mktemp("loop") / "serve_loop_driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-I", INCLUDE,
                    os.path.join(ROOT, "tests", "serve_loop_driver.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


class SimClock:
    """Time that moves only when the loop reports a pass without progress."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class SimExecutor:
    """One batch at a time in submission order: a batch submitted at t ends at
    max(t, previous end) + latency + payload bytes / rate (the model of the simulated
    device in serve_loop_driver.cpp)."""

    def __init__(self, clock, nstreams, latency, rate, tick):
        self.clock, self.nstreams = clock, nstreams
        self.latency, self.rate, self.tick = latency, rate, tick
        self.busy = 0
        self.next_free = 0.0
        self.log = []

    def free_slots(self):
        return self.nstreams - self.busy

    def submit(self, reqs, first, last, key_slots, fills, out_base=None):
        self.busy += 1
        start = max(self.clock(), self.next_free)
        t_done = start + self.latency + int(reqs.size[first:last].sum()) / self.rate
        self.next_free = t_done
        self.log.append("B %d %d %d %d%s" % (first, last - first, out_base, len(fills),
                                             "".join(" %d %d" % f for f in fills)))
        return {"t": t_done}

    def done(self, h):
        return self.clock() >= h["t"]

    def release(self, h):
        self.busy -= 1

    def idle(self):
        self.clock.t += self.tick


def trace(seed, n, nkeys, rate, median, sigma, max_size):
    g = np.random.Generator(np.random.PCG64(seed))
    arrival = np.cumsum(g.exponential(1.0 / rate, n))
    size = np.clip(np.round(np.exp(g.normal(np.log(median), sigma, n))), 1, max_size)
    p = 1.0 / np.arange(1, nkeys + 1) ** 0.9
    key = g.choice(nkeys, size=n, p=p / p.sum())
    return arrival, size.astype(np.int64), key.astype(np.int64)


def run_both(driver, arrival, size, key, nkeys, nslots, nstreams, maxb, budget, max_bytes,
             window, out_bytes, latency=20e-6, rate=2e9, tick=1e-6, realtime=True):
    n = size.size
    lines = ["loop %d %d %d %d %d %d %d %d %.17g %d %.17g %.17g %.17g" % (
        n, nkeys, nslots, nstreams, maxb, int(realtime), budget, max_bytes, window, out_bytes,
        latency, rate, tick)]
    lines += ["%.17g %d %d" % (a, s, k) for a, s, k in zip(arrival, size, key)]
    res = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, timeout=60)
    assert res.returncode == 0, res.stderr
    out = res.stdout.splitlines()
    c_batches = [l for l in out if l.startswith("B ")]
    c_lat = np.array([float(l.split()[1]) for l in out if l.startswith("L ")])
    c_stats = [int(x) for x in out[-1].split()[1:]]

    reqs = serve.Requests(arrival=arrival, key_id=key, nonce=np.zeros((n, 12), np.uint8),
                          ctr0=np.zeros(n, np.uint32), size=size,
                          in_off=np.zeros(n, np.int64))
    clock = SimClock()
    ex = SimExecutor(clock, nstreams, latency, rate, tick)
    srv = serve.Server(ex, serve.KeyCache(nslots, nkeys), budget, max_batch_bytes=max_bytes,
                       max_batch_reqs=maxb, window_s=window, clock=clock, out_bytes=out_bytes,
                       row_cap=max(1, nslots // nstreams))
    st, _ = srv.run(reqs, realtime=realtime)
    p_stats = [st.completed, st.rejected, st.batches, st.bytes, st.key_hits, st.key_misses,
               st.max_held, st.max_out_used, st.max_inflight]
    return (c_batches, c_lat, c_stats), (ex.log, st.latency_s, p_stats)


CASES = [
    # nkeys, nslots, nstreams, budget, out_bytes, rate (req/s)
    (64, 64, 2, 4 << 30, 1 << 40, 2e5),        # nothing binds but time
    (64, 16, 2, 256 << 10, 1 << 40, 5e5),      # the budget binds
    (64, 16, 2, 1 << 40, 96 << 10, 5e5),       # the output ring binds (and wraps)
    (200, 12, 3, 512 << 10, 160 << 10, 8e5),   # key cache, budget and ring all bind
    (40, 8, 4, 1 << 40, 64 << 10, 1e6),        # many streams on a small ring
    (30, 30, 1, 300 << 10, 200 << 10, 3e5),    # one stream
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_loop_equals_python_model(driver, case):
    nkeys, nslots, nstreams, budget, out_bytes, rate = CASES[case]
    arrival, size, key = trace(100 + case, 1500, nkeys, rate, 2048, 1.5, 48 << 10)
    size[::97] = 70 << 10                      # some requests larger than the ring allows
    (cb, cl, cs), (pb, pl, ps) = run_both(driver, arrival, size, key, nkeys, nslots, nstreams,
                                          maxb=256, budget=budget, max_bytes=1 << 20,
                                          window=25e-6, out_bytes=out_bytes)
    assert len(cb) == len(pb)
    for i, (a, b) in enumerate(zip(cb, pb)):
        assert a == b, (i, a[:120], b[:120])
    assert np.array_equal(cl, pl)
    assert cs == ps
    completed, rejected, batches = cs[0], cs[1], cs[2]
    assert completed + rejected == size.size and batches == len(cb)
    assert cs[6] <= budget and cs[7] <= out_bytes and 1 <= cs[8] <= nstreams
    lin = np.concatenate([[0], np.cumsum((size + 15) // 16 * 16)])
    if out_bytes < int(lin[-1]):
        # the ring was reused: some output range started again at offset 0
        assert sum(1 for l in cb if l.split()[3] == "0") > 1
    else:
        # an area that holds every output is never reused: batch outputs are
        # laid out one after the other in request order (rejected requests
        # take no room)
        pos = 0
        for l in cb:
            first, count, base = (int(v) for v in l.split()[1:4])
            assert base == pos, l[:80]
            pos += int(lin[first + count] - lin[first])


def test_closed_loop_equals_python_model(driver):
    """The whole trace present at the start (realtime off): a backlog cut by
    the batch limits, the ring and a small key cache."""
    arrival, size, key = trace(8, 1200, 60, 1e6, 4096, 1.5, 64 << 10)
    arrival[:] = 0.0
    (cb, cl, cs), (pb, pl, ps) = run_both(driver, arrival, size, key, 60, 12, 3, maxb=200,
                                          budget=2 << 20, max_bytes=512 << 10, window=25e-6,
                                          out_bytes=300 << 10, realtime=False)
    assert cb == pb and np.array_equal(cl, pl) and cs == ps
    assert cs[0] == size.size and cs[8] == 3 and len(cb) > 10


def test_loop_with_no_limits_makes_progress(driver):
    """Budget and batch size of 2^64 - 1 ("no limit"): the batch cut must not
    wrap around; every request is served, each batch up to max_batch_reqs."""
    arrival, size, key = trace(7, 2000, 50, 5e6, 4096, 1.0, 1 << 20)
    (cb, cl, cs), (pb, pl, ps) = run_both(driver, arrival, size, key, 50, 50, 2, maxb=128,
                                          budget=U64_MAX, max_bytes=U64_MAX, window=25e-6,
                                          out_bytes=U64_MAX)
    assert cb == pb and np.array_equal(cl, pl) and cs == ps
    assert cs[0] == size.size and cs[1] == 0
    counts = [int(l.split()[2]) for l in cb]
    assert max(counts) == 128                    # the request limit, not one per batch
    # max_batch_bytes near 2^64 (the case that used to give one request per batch)
    (cb2, _, cs2), _ = run_both(driver, arrival, size, key, 50, 50, 2, maxb=128,
                                budget=U64_MAX - 5, max_bytes=U64_MAX - 3, window=25e-6,
                                out_bytes=1 << 40)
    assert cs2[0] == size.size and max(int(l.split()[2]) for l in cb2) == 128


def _ring_ops(seed, cap, nops):
    g = np.random.Generator(np.random.PCG64(seed))
    ops, live = [], []
    nalloc = 0
    for _ in range(nops):
        if live and (len(live) > 6 or g.random() < 0.45):
            i = live.pop(int(g.integers(0, len(live))))
            ops.append(("F", i))
        else:
            ops.append(("A", int(g.integers(1, cap // 3 + 2)) * 16 if g.random() < 0.9 else cap))
            live.append(nalloc)
            nalloc += 1
    return ops


@pytest.mark.parametrize("seed,cap", [(1, 1024), (2, 4096), (3, 160), (4, 100000)])
def test_out_ring(driver, seed, cap):
    ops = _ring_ops(seed, cap, 3000)
    text = "ring %d %d\n" % (cap, len(ops)) + "".join("%s %d\n" % o for o in ops)
    out = subprocess.run([driver], input=text, capture_output=True, text=True, timeout=60,
                         check=True).stdout.split("\n")
    ring = serve.OutRing(cap)
    offs, live = [], {}
    pos = 0
    for op, v in ops:
        if op == "A":
            fits = v <= ring.max_alloc()
            got = ring.alloc(v) if fits else -1
            assert out[pos] == "A %d" % got
            pos += 1
            offs.append(got)
            if fits:
                # inside the area and disjoint from every live range
                assert 0 <= got and got + v <= cap
                for o, n in live.values():
                    assert got + v <= o or o + n <= got
                live[len(offs) - 1] = (got, v)
        else:
            if offs[v] >= 0:
                ring.release(offs[v])
                live.pop(v)
        assert out[pos] == "M %d" % ring.max_alloc()
        pos += 1
    # an empty ring offers the whole area again
    for i in list(live):
        ring.release(live.pop(i)[0])
    assert ring.max_alloc() == cap and ring.used == 0

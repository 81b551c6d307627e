"""The serving loop on the GPU: every request served in the mix equals the
same request run alone (aes_ctr_xcrypt with its own key) and the oracle's CTR
of that request; batches overlap on two streams and keys are evicted and
refilled."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am
from paper_1506_08503_amd import serve
from paper_1506_08503_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_served_equals_alone(oracle):
    nreq, pool_bytes = 3000, 32 << 20
    rs = wl.serving_inputs(nreq, 3e5, nkeys=64, median=4096, sigma=2.0, max_size=1 << 20,
                           seed=21)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=21)
    g = np.random.Generator(np.random.PCG64(22))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    nslots = 16
    # an output arena smaller than the run's output: the first batches are
    # carved from it, the later ones get buffers of their own
    ex = serve.GpuExecutor(pool, rs.keys, nslots, nstreams=2, max_segs=1024,
                           out_arena_bytes=8 << 20)
    kc = serve.KeyCache(nslots, len(rs.keys))
    srv = serve.Server(ex, kc, hbm_budget=48 << 20, max_batch_reqs=1024)
    st, res = srv.run(reqs)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.rejected == 0
    assert st.key_misses > 0 and st.key_hits > 0 and np.all(kc.pins == 0)
    assert st.max_held <= 48 << 20
    assert 0 < ex.arena_used <= 8 << 20 and int(reqs.size.sum()) > 8 << 20
    for i in range(nreq):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        ks = am.key_schedule(rs.keys[reqs.key_id[i]], DEV)
        alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
        assert torch.equal(res[i], alone), i
    got = [res[i].cpu().numpy() for i in range(nreq)]

    def agrees(i):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        return np.array_equal(got[i], exp)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool_ex:
        bad = [i for i, ok in zip(range(nreq), pool_ex.map(agrees, range(nreq))) if not ok]
    assert not bad, bad[:10]
    s = st.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0


@pytest.mark.parametrize("nslots", [1024, 256])
def test_native_bench_configuration(oracle, nslots):
    """The serving benchmark's configuration on a backlogged slice of its
    workload: lognormal sizes (median 4 KiB, sigma 2, up to 16 MiB), 1,024
    keys (half AES-128, half AES-256), a 256 MiB pool, a 4 GiB budget, two
    streams, batches up to 256 MiB / 16,384 requests, a 25 us window, key
    caches of 1,024 and 256 rows.  Every request equals the same request run
    alone; a sample of 400 equals the oracle."""
    nreq, pool_bytes = 20000, 256 << 20
    rs = wl.serving_inputs(nreq, 1e5, nkeys=1024, seed=51)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=52)
    reqs.arrival[:] = 0.0
    g = np.random.Generator(np.random.PCG64(53))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    st, res = serve.run_native(pool, rs.keys, reqs, nslots, nstreams=2, hbm_budget=4 << 30,
                               max_batch_reqs=16384, max_batch_bytes=256 << 20,
                               window_s=25e-6)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.rejected == 0
    assert st.key_hits + st.key_misses == nreq
    assert st.batches < nreq // 100 and st.max_inflight == 2     # backlogged: large batches
    scheds = {}
    for i in range(nreq):
        kid = int(reqs.key_id[i])
        if kid not in scheds:
            scheds[kid] = am.key_schedule(rs.keys[kid], DEV)
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        alone = am.ctr_xcrypt(scheds[kid], reqs.nonce[i].tobytes(), int(reqs.ctr0[i]),
                              pool[a:a + n])
        assert torch.equal(res[i], alone), i
    sample = np.random.Generator(np.random.PCG64(54)).choice(nreq, 400, replace=False)
    got = {int(i): res[int(i)].cpu().numpy() for i in sample}

    def agrees(i):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        return np.array_equal(got[i], exp)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool_ex:
        bad = [i for i, ok in zip(got, pool_ex.map(agrees, list(got))) if not ok]
    assert not bad, bad[:10]


@pytest.mark.parametrize("nstreams,realtime", [(2, True), (4, False), (1, True), (3, True),
                                               (8, False)])
def test_native_served_equals_alone(oracle, nstreams, realtime):
    """The request loop run inside the library (aes_serve_run): every request
    equals the same request run alone and the oracle's CTR; a 16-row key
    cache for 64 keys forces evictions and refills, several streams force
    waits on another stream's key expansion, and a 48 MiB budget holds
    admission back."""
    nreq, pool_bytes = 3000, 32 << 20
    rs = wl.serving_inputs(nreq, 3e5, nkeys=64, median=4096, sigma=2.0, max_size=1 << 20,
                           seed=31 + nstreams)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=31)
    g = np.random.Generator(np.random.PCG64(32))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    st, res = serve.run_native(pool, rs.keys, reqs, nslots=16, nstreams=nstreams,
                               hbm_budget=48 << 20, max_batch_reqs=1024, realtime=realtime)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.rejected == 0
    assert st.key_misses > 0 and st.key_hits > 0 and st.key_hits + st.key_misses == nreq
    assert st.max_held <= 48 << 20 and 1 <= st.max_inflight <= nstreams
    assert np.all(np.isfinite(st.latency_s)) and np.all(st.latency_s > 0)
    got = [res[i].cpu().numpy() for i in range(nreq)]
    for i in range(nreq):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        ks = am.key_schedule(rs.keys[reqs.key_id[i]], DEV)
        alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
        assert np.array_equal(got[i], alone.cpu().numpy()), i

    def agrees(i):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        return np.array_equal(got[i], exp)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool_ex:
        bad = [i for i, ok in zip(range(nreq), pool_ex.map(agrees, range(nreq))) if not ok]
    assert not bad, bad[:10]


def test_native_rejects_oversize():
    """A request larger than the whole budget is rejected (no output, infinite
    latency); the others are served."""
    rs = wl.serving_inputs(200, 1e5, nkeys=8, median=4096, sigma=1.0, max_size=1 << 16, seed=5)
    reqs = serve.requests_from_stream(rs, 8 << 20, seed=5)
    reqs.size[7] = 6 << 20                                   # 6 MiB in + 6 MiB out > 8 MiB
    reqs.in_off[7] = 0
    pool = torch.zeros(8 << 20, dtype=torch.uint8, device=DEV)
    st, res = serve.run_native(pool, rs.keys, reqs, nslots=8, hbm_budget=8 << 20)
    torch.cuda.synchronize()
    assert st.rejected == 1 and st.completed == 199
    assert res[7] is None and np.isinf(st.latency_s[7])
    assert res[8] is not None and res[8].numel() == int(reqs.size[8])


@pytest.mark.parametrize("max_batch_mib,nreq,median_kib", [(4, 400, 128), (48, 400, 128),
                                                          (160, 700, 640)])
def test_native_batch_sizes_cover_every_tile(oracle, max_batch_mib, nreq, median_kib):
    """Backlogged requests cut into batches of about max_batch_mib MiB: the
    loop runs batches of up to 2,048 blocks per wave of its grid (128 MiB on
    256 CUs) with 256-block tiles and larger ones with 1,024-block tiles;
    every output equals the request run alone, and a sample equals the
    oracle."""
    pool_bytes = 64 << 20
    rs = wl.serving_inputs(nreq, 1e5, nkeys=24, median=median_kib << 10, sigma=1.0,
                           max_size=(2 if median_kib < 512 else 8) << 20,
                           seed=40 + max_batch_mib)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=41)
    g = np.random.Generator(np.random.PCG64(42))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    if max_batch_mib > 128:
        waves = 16 * am.device_cu_count()
        assert int(reqs.size.sum()) > 2 * (2048 * 16 * waves)   # batches above the threshold
    st, res = serve.run_native(pool, rs.keys, reqs, nslots=8, nstreams=2, hbm_budget=2 << 30,
                               max_batch_bytes=max_batch_mib << 20, realtime=False)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.rejected == 0
    assert st.batches >= int(reqs.size.sum()) // ((max_batch_mib + 2) << 20)
    # backlogged on two streams: a second batch was launched while the first ran
    assert st.max_inflight == 2
    for i in range(nreq):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        ks = am.key_schedule(rs.keys[reqs.key_id[i]], DEV)
        alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
        assert torch.equal(res[i], alone), i
    for i in range(0, nreq, 40):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        assert np.array_equal(res[i].cpu().numpy(), exp), i


def test_native_all_key_sizes(oracle):
    """Keys of 16, 24 and 32 bytes in one trace (the staging kernel expands
    each size into the cache); 8 rows for 30 keys so rows are refilled with
    keys of other sizes; every other request starts at a random counter."""
    nreq, pool_bytes = 1500, 16 << 20
    rs = wl.serving_inputs(nreq, 2e5, nkeys=30, median=2048, sigma=1.5, max_size=256 << 10,
                           seed=51)
    g = np.random.Generator(np.random.PCG64(52))
    rs.keys = [g.bytes((16, 24, 32)[i % 3]) for i in range(30)]
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=53)
    # half the requests start at a random counter (not group aligned), up to
    # the last one that still fits the request
    r = g.integers(0, (1 << 32) - (reqs.size + 15) // 16, dtype=np.int64)
    reqs.ctr0 = np.where(np.arange(nreq) % 2 == 1, r, 0).astype(np.uint32)
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    st, res = serve.run_native(pool, rs.keys, reqs, nslots=8, nstreams=2)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.key_misses > 30
    for i in range(nreq):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        ks = am.key_schedule(rs.keys[reqs.key_id[i]], DEV)
        alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
        assert torch.equal(res[i], alone), i
    for i in range(0, nreq, 50):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        assert np.array_equal(res[i].cpu().numpy(), exp), i


@pytest.mark.parametrize("realtime", [False, True])
def test_native_small_output_ring(oracle, realtime):
    """The output area is a quarter of the trace's output: batches take ranges
    of it and give them back when they retire, so later batches reuse the
    same bytes and admission waits for them.  A consumer copies each
    completed batch out before its range is reused; every collected result
    equals the request run alone and the oracle's CTR, two batches were in
    flight at once, and the ring never held more than its size."""
    nreq, pool_bytes = 2500, 32 << 20
    rs = wl.serving_inputs(nreq, 4e5, nkeys=48, median=8192, sigma=1.5, max_size=1 << 20,
                           seed=61 + realtime)
    reqs = serve.requests_from_stream(rs, pool_bytes, seed=62)
    g = np.random.Generator(np.random.PCG64(63))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    pad = (reqs.size + 15) // 16 * 16
    lin = np.concatenate([[0], np.cumsum(pad)])
    total = int(lin[-1])
    ring_bytes = (total // 4) // 16 * 16
    assert ring_bytes >= int(pad.max())
    out = torch.full((ring_bytes,), 0xEE, dtype=torch.uint8, device=DEV)
    collected = torch.zeros(total, dtype=torch.uint8, device=DEV)
    seen = np.zeros(nreq, bool)

    def consume(first, count, out_off):
        # the batch's outputs are contiguous in the ring, in request order
        o = int(out_off[first])
        n = int(lin[first + count] - lin[first])
        assert o + n <= ring_bytes
        assert not seen[first:first + count].any()
        seen[first:first + count] = True
        collected[int(lin[first]):int(lin[first]) + n].copy_(out[o:o + n])
        torch.cuda.synchronize()

    st, _ = serve.run_native(pool, rs.keys, reqs, nslots=16, nstreams=2, hbm_budget=1 << 30,
                             max_batch_bytes=ring_bytes // 6, realtime=realtime, out=out,
                             on_batch=consume)
    torch.cuda.synchronize()
    assert st.completed == nreq and st.rejected == 0 and seen.all()
    assert st.max_out_used <= ring_bytes and st.max_inflight == 2
    assert st.bytes == int(reqs.size.sum()) and total > 3 * ring_bytes
    col = collected.cpu().numpy()
    for i in range(nreq):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        ks = am.key_schedule(rs.keys[reqs.key_id[i]], DEV)
        alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
        assert np.array_equal(col[int(lin[i]):int(lin[i]) + n], alone.cpu().numpy()), i

    def agrees(i):
        a, n = int(reqs.in_off[i]), int(reqs.size[i])
        exp = oracle.ctr_xcrypt(rs.keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                int(reqs.ctr0[i]), pool_h[a:a + n])
        return np.array_equal(col[int(lin[i]):int(lin[i]) + n], exp)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool_ex:
        bad = [i for i, ok in zip(range(nreq), pool_ex.map(agrees, range(nreq))) if not ok]
    assert not bad, bad[:10]


def test_native_server_object_runs_twice(oracle):
    """aes_server_create once, two traces through aes_server_run: the key
    cache carries over (the second run hits keys the first one loaded), and
    in both runs every result equals the request run alone and sampled ones
    the oracle."""
    pool_bytes = 16 << 20
    g = np.random.Generator(np.random.PCG64(71))
    pool_h = np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()
    pool = torch.from_numpy(pool_h).to(DEV)
    rs1 = wl.serving_inputs(1200, 3e5, nkeys=40, median=4096, sigma=1.5, max_size=256 << 10,
                            seed=72)
    keys = rs1.keys
    reqs1 = serve.requests_from_stream(rs1, pool_bytes, seed=73)
    rs2 = wl.serving_inputs(900, 3e5, nkeys=40, median=4096, sigma=1.5, max_size=256 << 10,
                            seed=74)
    reqs2 = serve.requests_from_stream(rs2, pool_bytes, seed=75)
    srv = serve.NativeServer(keys, nslots=64, nstreams=2, max_batch_reqs=512)
    try:
        st1, res1 = srv.run(pool, reqs1)
        st2, res2 = srv.run(pool, reqs2)
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert st1.completed == len(reqs1) and st2.completed == len(reqs2)
    # misses count requests whose key was filled for their batch: every key
    # missed in the first run, none in the second
    assert st1.key_misses >= 40 and st2.key_misses == 0 and st2.key_hits == len(reqs2)
    for reqs, res, seed in ((reqs1, res1, 1), (reqs2, res2, 2)):
        for i in range(len(reqs)):
            a, n = int(reqs.in_off[i]), int(reqs.size[i])
            ks = am.key_schedule(keys[reqs.key_id[i]], DEV)
            alone = am.ctr_xcrypt(ks, reqs.nonce[i].tobytes(), int(reqs.ctr0[i]), pool[a:a + n])
            assert torch.equal(res[i], alone), (seed, i)
        for i in range(0, len(reqs), 60):
            a, n = int(reqs.in_off[i]), int(reqs.size[i])
            exp = oracle.ctr_xcrypt(keys[reqs.key_id[i]], reqs.nonce[i].tobytes(),
                                    int(reqs.ctr0[i]), pool_h[a:a + n])
            assert np.array_equal(res[i].cpu().numpy(), exp), (seed, i)

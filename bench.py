"""Benchmark: AES-128-CTR over a 4 GiB buffer resident in HBM on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--layout ttable|bitslice]

A step is one aes_ctr_xcrypt call over the whole 4 GiB plaintext (2^28 blocks):
counter-block generation, all rounds, the XOR with the plaintext and the HBM
reads and writes.  Inputs are generated and copied to the device before the
timed region.  Prints one JSON line.

Besides the throughput it reports
  * roofline: HBM-roofline position of the CTR kernel (algorithmic bytes = 16 B
    read + 16 B written per block, divided by the kernel's average duration
    from HIP events on the launch stream), plus the binding on-chip limits;
  * gcm: AES-128-GCM over the same buffer (encrypt, decrypt) and the GHASH
    passes alone, with their HBM and LDS fractions;
  * batched / serving: many-message launches and the request loop;
  * sweep: the paper's Fig. 3 workloads (CBC and CTR against message count
    and length);
  * dbcolumn: AES-256 ECB over the 2^26-row database column;
  * cpu_baseline: the CPU oracle (plain algebraic AES) timed on the host's
    cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 lanes x 2.4 GHz, 32-bit ops
LDS_PEAK_TREADS = 256 * 32 * 2.4e9 / 1e12  # 32 dword reads per clock per CU
WARM_MS = 150                  # default warm-up length (see --warmup)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=-1,
                   help="untimed steps before the timed ones; the default (-1) runs steps "
                        "until %d ms have passed (at least 3): after idle the chip takes "
                        "tens of milliseconds under load to reach its working clock"
                        % WARM_MS)
    p.add_argument("--nbytes", type=int, default=4 << 30)
    p.add_argument("--layout", choices=["auto", "ttable", "bitslice"], default="auto")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--op", choices=["ctr", "ecb-enc", "ecb-dec", "gcm-enc", "gcm-dec"],
                   default="ctr",
                   help="operation of the stream leg (the headline metric is ctr)")
    p.add_argument("--key-bytes", type=int, default=16, choices=[16, 24, 32])
    p.add_argument("--ctr-precompute", type=int, default=0, choices=[0, 1, 2],
                   help="CTR with the table layout: 0 = rounds 1-2 precomputed (default), "
                        "1 = round-1 nonce terms only, 2 = none (the measured baseline)")
    p.add_argument("--mode", choices=["aes", "copy"], default="aes",
                   help="copy: time a plain device copy of the same buffer instead "
                        "(reference for HBM counter calibration)")
    p.add_argument("--cpu-threads", type=int, default=0)
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-gcm", action="store_true")
    p.add_argument("--no-dbcolumn", action="store_true",
                   help="skip the AES-256 ECB database-column leg")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--serving-requests", type=int, default=100_000)
    p.add_argument("--sweep", action="store_true",
                   help="instead of the benchmark: the paper's Fig. 3 workloads (rate vs "
                        "number of 16-byte messages; rate vs length for 128 messages)")
    p.add_argument("--no-sweep", action="store_true",
                   help="leave the Fig. 3 workloads out of the benchmark line")
    p.add_argument("--plaintext", choices=["random", "zero"], default="random",
                   help="stream leg input: uniform random bytes (the workload) or all zero "
                        "(for data-dependence checks of the counters)")
    p.add_argument("--key-seed", type=int, default=None,
                   help="draw the stream leg's key and nonce from this seed instead of the "
                        "workload's (for key-dependence checks of the counters)")
    p.add_argument("--no-tune", action="store_true",
                   help="time the library's default launch shape instead of the autotuned one")
    p.add_argument("--no-probes", action="store_true",
                   help="leave out the on-chip ceiling microbenchmarks (LDS, rounds, VALU)")
    p.add_argument("--trace-summary", metavar="DIR",
                   help="instead of the benchmark: summarize the kernel trace that "
                        "rocprofv3 --kernel-trace --output-format csv wrote under DIR, over "
                        "the last --last dispatches of each kernel (the timed steps of a "
                        "bench run are its last dispatches of the stream kernel)")
    p.add_argument("--pmc-summary", metavar="DIR",
                   help="instead of the benchmark: average the counters rocprofv3 --pmc "
                        "--output-format csv wrote under DIR over the last --last dispatches "
                        "of each kernel")
    p.add_argument("--last", type=int, default=20)
    p.add_argument("--split-gap-ms", type=float, default=0.0,
                   help="with --trace-summary: also split the trace into runs at idle gaps "
                        "longer than this (every kernel idle) and summarize each run")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return p.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, threads):
    """Oracle CTR (as it stands) on a bounded prefix of the same plaintext:
    48 MiB per host thread, about 10 s of CPU work on the benchmark host."""
    import numpy as np
    from oracle import oracle as orc
    o = orc.default()
    sample = min(inp.nbytes, (48 << 20) * threads)
    g = next(inp.plaintext_chunks(chunk=sample))[1]
    t0 = time.perf_counter()
    o.ctr_xcrypt(inp.key, inp.nonce, inp.ctr0, g, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample / dt / 1e9, 6), "unit": "GB/s", "cores": threads,
            "kind": "oracle", "host": "%s, %d cpus" % (_cpu_model(), os.cpu_count() or 0),
            "sample": "first %d MiB of the 4 GiB AES-128-CTR plaintext, %d host threads, "
                      "%.2f s" % (sample >> 20, threads, dt)}


def batched_leg():
    """10,000 messages (log-uniform 1 B .. 1 MiB, own AES-128 key and nonce):
    one persistent launch (autotuned; replayed as a HIP graph, and called
    directly, each 20 times back to back) against a loop of one plain
    aes_ctr_xcrypt launch per message.  GBps_batched is the faster of the
    two forms, named in `form`."""
    import torch
    from paper_1506_08503_amd import autotune, batch, workloads as wl
    b = wl.batched_inputs()
    db = batch.DeviceBatch(b)
    tune, table = autotune.tune_batched(db, reps=3, cache_path=None)
    g = db.graph(tune)
    ms_single = autotune.time_launch(g.launch, 10)
    ms_default = autotune.time_launch(lambda: db.run(None), 5)
    # back-to-back replays: the rate when the stream is kept busy (as the
    # stream leg's K timed steps); the single-call figure adds launch latency
    reps = 20
    g.launch()
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.launch()
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    # the same launch without the graph, back to back
    db.run(tune)
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        db.run(tune)
    e.record()
    torch.cuda.synchronize()
    ms_direct = a.elapsed_time(e) / reps
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    db.run_plain_loop()
    e.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    loop_ms = a.elapsed_time(e)
    g.close()
    best, form = (ms, "graph") if ms <= ms_direct else (ms_direct, "direct")
    return {"workload": "10000 messages, log-uniform 1 B..1 MiB, own AES-128 key+nonce",
            "bytes": db.nbytes, "GBps_batched": round(db.nbytes / best / 1e6, 1),
            "form": form,
            "GBps_batched_graph": round(db.nbytes / ms / 1e6, 1),
            "GBps_batched_direct": round(db.nbytes / ms_direct / 1e6, 1),
            "ms_batched_graph": round(ms, 4), "ms_batched_direct": round(ms_direct, 4),
            "ms_batched_graph_single_call": round(ms_single, 4),
            "ms_batched_default_tune_single_call": round(ms_default, 4),
            "GBps_plain_loop": round(db.nbytes / loop_ms / 1e6, 2),
            "ms_plain_loop": round(loop_ms, 3), "ms_plain_loop_wall": round(wall, 3),
            "speedup": round(loop_ms / ms, 1), "tune": tune}


SERVING_WARMUP = 5000
# Batch limits of the C++ serving loop.  Measured with 1,024 key rows (five
# runs each on two boxes): a 64 / 128 / 256 MiB byte limit gave closed-loop
# capacities of 33.0-36.4 / 35.1-38.5 / 37.0-42.0 M requests/s with the same
# latency at a fixed offered load (p50 / p99 at 18-20 M requests/s:
# 0.054-0.060 / 0.090-0.125 ms for all three; at 32 M: 0.107-0.129 /
# 0.201-0.230 ms): under load batches stay well below the limit, and a
# backlog drains in fewer, larger launches.
SERVING_BATCH_BYTES = 256 << 20
SERVING_BATCH_REQS = 16384


def serving_leg(nreq):
    """Open-loop Poisson arrivals of AES-128/256 CTR requests (lognormal sizes,
    median 4 KiB, sigma 2, clipped to 16 MiB; 1,024 keys; 4 GiB HBM budget),
    payloads already in device memory, served by the library's request loop
    (aes_serve_run: admission, key cache, batching and launches in C++, two
    streams).  Capacity is measured closed-loop, then latency at 50% and 80%
    of it; key caches of 1,024 and 256 slots.  Each open-loop run serves
    SERVING_WARMUP requests more than nreq and its latency percentiles cover
    the last nreq (the run starts with an empty key cache and an idle loop);
    p99_ms_all is the 99th percentile over every request.  The same loop
    written in Python (serve.Server) is measured closed-loop beside it.  Every
    run follows a 50 ms GPU warm-up."""
    import numpy as np
    import torch
    from paper_1506_08503_amd import serve, workloads as wl
    pool_bytes = 256 << 20
    g = np.random.Generator(np.random.PCG64(wl.SEED_SERVING + 1))
    pool = torch.from_numpy(np.frombuffer(g.bytes(pool_bytes), np.uint8).copy()).cuda()
    out = [None]
    # each run starts after seconds of host-side trace generation with the
    # GPU idle: warm it up as before the stream measurement (50 ms of CTR on a
    # 64 MiB buffer; +6-8% closed-loop capacity with 1,024 key rows)
    import paper_1506_08503_amd as am
    wks = am.key_schedule(bytes(16))
    wbuf = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")

    def out_for(reqs):
        need = int(((reqs.size + 15) // 16 * 16).sum())
        if out[0] is None or out[0].numel() < need:
            out[0] = None
            out[0] = torch.empty(need, dtype=torch.uint8, device="cuda")
        return out[0]

    def run(rate, n, nslots, closed=False, python_loop=False):
        nwarm = 0 if closed else SERVING_WARMUP
        rs = wl.serving_inputs(n + nwarm, rate, nkeys=1024)
        reqs = serve.requests_from_stream(rs, pool_bytes)
        if closed:
            reqs.arrival[:] = 0.0
        ob = None if python_loop else out_for(reqs)
        warm(torch, lambda: am.ctr_xcrypt(wks, bytes(12), 0, wbuf, out=wbuf), ms=50)
        if python_loop:
            ex = serve.GpuExecutor(pool, rs.keys, nslots, nstreams=2, max_segs=8192,
                                   out_arena_bytes=4 << 30)
            srv = serve.Server(ex, serve.KeyCache(nslots, len(rs.keys)), hbm_budget=4 << 30,
                               max_batch_reqs=8192, window_s=25e-6)
            st, _ = srv.run(reqs)
        else:
            st, _ = serve.run_native(pool, rs.keys, reqs, nslots, nstreams=2,
                                     hbm_budget=4 << 30, max_batch_reqs=SERVING_BATCH_REQS,
                                     max_batch_bytes=SERVING_BATCH_BYTES, window_s=25e-6,
                                     out=ob)
        torch.cuda.synchronize()
        s = st.summary(skip=nwarm)
        if nwarm:
            s["warmup_requests"] = nwarm
            s["p99_ms_all"] = st.summary()["p99_ms"]
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}

    run(1e5, 5000, 1024, closed=True)            # warm-up
    res_all = {"workload": "%d requests, lognormal sizes median 4 KiB sigma 2 (<=16 MiB), "
                           "1024 keys (half AES-128, half AES-256), 4 GiB budget" % nreq,
               "loop": "aes_serve_run (C++), 2 streams, batches up to %d MiB / %d requests, "
                       "25 us window" % (SERVING_BATCH_BYTES >> 20, SERVING_BATCH_REQS),
               "python_loop": "serve.Server, batches up to 64 MiB / 8192 requests"}
    for nslots in (1024, 256):
        cap = run(1e5, nreq, nslots, closed=True)
        rate = cap["req_per_s"]
        res = {"capacity": cap}
        for rho in (0.5, 0.8):
            res["rho%.1f" % rho] = dict(run(rho * rate, nreq, nslots), offered_req_per_s=
                                        round(rho * rate))
        res_all["key_slots_%d" % nslots] = res
    run(1e5, 5000, 1024, closed=True, python_loop=True)
    res_all["python_loop_capacity_1024_slots"] = run(1e5, nreq, 1024, closed=True,
                                                     python_loop=True)["req_per_s"]
    return res_all


def sweep_fig3():
    """Rates of the paper's Fig. 3 workloads (sec. IV): AES-128 CBC encryption
    and decryption of N 16-byte messages for growing N, and of 128 messages of
    growing length; CTR of the same bytes beside them.  One JSON line."""
    import numpy as np
    import torch
    import paper_1506_08503_amd as am
    from paper_1506_08503_amd import autotune
    g = np.random.Generator(np.random.PCG64(0xF163))
    ks = am.key_schedule(g.bytes(16))
    rows = []

    def measure(nmsg, msg_bytes):
        n = nmsg * msg_bytes
        x = torch.from_numpy(np.frombuffer(g.bytes(n), np.uint8).copy()).cuda()
        iv = torch.from_numpy(np.frombuffer(g.bytes(16 * nmsg), np.uint8).copy()).cuda()
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        reps = 20 if n < (64 << 20) else 5
        enc = lambda: am.cbc_encrypt(ks, iv, x, nmsg, out=y)
        dec = lambda: am.cbc_decrypt(ks, iv, y, nmsg, out=z)
        ctr = lambda: am.ctr_xcrypt(ks, b"\0" * 12, 0, x, out=z)
        warm(torch, enc)
        t_enc = autotune.time_launch(enc, reps)
        warm(torch, dec)
        t_dec = autotune.time_launch(dec, reps)
        warm(torch, ctr)
        t_ctr = autotune.time_launch(ctr, reps)
        assert torch.equal(am.cbc_decrypt(ks, iv, y, nmsg), x)
        return {"messages": nmsg, "msg_bytes": msg_bytes, "total_bytes": n,
                "cbc_enc_GBps": round(n / t_enc / 1e6, 3), "cbc_dec_GBps": round(n / t_dec / 1e6, 3),
                "ctr_GBps": round(n / t_ctr / 1e6, 3), "cbc_enc_ms": round(t_enc, 4)}

    for e in range(4, 27, 2):                      # 16 .. 2^26 sixteen-byte messages
        rows.append(dict(measure(1 << e, 16), curve="16-byte messages"))
    for e in range(4, 21, 2):                      # 128 messages of 16 B .. 1 MiB
        rows.append(dict(measure(128, 1 << e), curve="128 messages"))
    return {"sweep": "paper Fig. 3 workloads, AES-128", "rows": rows}


# Measured on an MI355X (rocprofv3 --pmc SQ_INSTS_VALU, AES-128 CTR over 4 GiB):
# VALU lane operations per block of ctr_grouped_kernel.
CTR_VALU_PER_BLOCK = 207


def probes():
    """On-chip ceilings measured on this GPU (csrc/probe.hip): conflict-free
    random LDS reads, the T-table round function without HBM traffic, and
    three-input XOR chains; each with the shader clock it ran at."""
    import ctypes
    path = os.path.join(ROOT, "paper_1506_08503_amd", "libaesmi_probe.so")
    lib = ctypes.CDLL(path)
    f = lib.aesmi_probe_run
    f.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int] + [ctypes.POINTER(ctypes.c_double)] * 3
    f.restype = ctypes.c_int
    out = {}
    for kind, name, iters in ((0, "lds", 40000), (1, "rounds", 10000), (2, "valu", 20000)):
        ms, rate, clk = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = f(kind, iters, 5, ctypes.byref(ms), ctypes.byref(rate), ctypes.byref(clk))
        if rc:
            raise RuntimeError("probe %s failed with HIP error %d" % (name, rc))
        out[name] = {"rate_t_per_s": round(rate.value / 1e12, 3), "ms": round(ms.value, 3),
                     "sclk_ghz": round(clk.value, 3)}
    return out


def binding_roofline(lds_reads, nblocks, ms, pr):
    """The CTR kernel's on-chip position: its LDS reads and VALU operations
    per second against the probes' measured rates and against the unit peaks
    at the shader clock the probe held."""
    sec = ms * 1e-3
    lds = lds_reads / sec / 1e12
    valu = CTR_VALU_PER_BLOCK * nblocks / sec / 1e12
    res = {"lds_treads_per_s": round(lds, 3), "valu_tops_per_s": round(valu, 3),
           "valu_ops_per_block": CTR_VALU_PER_BLOCK,
           "valu_ops_per_block_source": "rocprofv3 --pmc SQ_INSTS_VALU x 64 / blocks, "
                                        "profiles/ctr_grouped_kernel_aes128_ctr_4GiB.md"}
    if pr:
        lds_clk, valu_clk = pr["lds"]["sclk_ghz"], pr["valu"]["sclk_ghz"]
        res.update({
            "lds_probe_treads_per_s": pr["lds"]["rate_t_per_s"],
            "lds_frac_of_probe": round(lds / pr["lds"]["rate_t_per_s"], 4),
            "round_probe_lookups_t_per_s": round(pr["rounds"]["rate_t_per_s"] * 16, 3),
            "lds_frac_of_round_probe": round(lds / (pr["rounds"]["rate_t_per_s"] * 16), 4),
            "lds_peak_at_probe_sclk_treads": round(256 * 32 * lds_clk / 1e3, 3),
            "lds_frac_at_probe_sclk": round(lds / (256 * 32 * lds_clk / 1e3), 4)
            if lds_clk else None,
            "valu_probe_tops_per_s": pr["valu"]["rate_t_per_s"],
            "valu_frac_of_probe": round(valu / pr["valu"]["rate_t_per_s"], 4),
            "valu_frac_at_probe_sclk": round(valu / (256 * 64 * valu_clk / 1e3), 4)
            if valu_clk else None,
            "probes": pr})
    return res


def trace_summary(root, last, split_gap_ms=0.0):
    """Per kernel: calls in the trace, and count / average / min / max
    duration (ms) of its last `last` dispatches, from rocprofv3's kernel
    trace CSV files under root.  With split_gap_ms > 0, also per run: the
    dispatches split where the GPU ran no kernel for longer than that."""
    import csv
    import glob
    rows, allk = {}, []
    for path in sorted(glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                ev = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                rows.setdefault(name, []).append(ev)
                allk.append(ev + (name,))

    def stats(ts):
        d = [(e - b) / 1e6 for b, e in ts]
        return {"calls": len(d), "avg_ms": round(sum(d) / len(d), 4),
                "min_ms": round(min(d), 4), "max_ms": round(max(d), 4)}
    out = {}
    for name, ts in rows.items():
        ts.sort()
        out[name] = dict(stats(ts[-last:]), calls=len(ts), last=len(ts[-last:]))
    if split_gap_ms > 0 and allk:
        allk.sort()
        runs, cur, busy_until = [], [], None
        for b, e, name in allk:
            if cur and b - busy_until > split_gap_ms * 1e6:
                runs.append(cur)
                cur = []
            cur.append((b, e, name))
            busy_until = e if busy_until is None or not cur[:-1] else max(busy_until, e)
        runs.append(cur)
        out["runs"] = []
        for run in runs:
            per = {}
            for b, e, name in run:
                per.setdefault(name, []).append((b, e))
            out["runs"].append({"span_ms": round((max(e for _, e, _ in run) - run[0][0]) / 1e6, 3),
                                "kernels": {n: stats(ts) for n, ts in per.items()}})
    return out


def pmc_summary(root, last):
    """Per kernel: the mean of each counter over its last `last` dispatches,
    from rocprofv3's counter collection CSV files under root, with the mean
    dispatch duration and, when GRBM_GUI_ACTIVE was collected, the shader
    clock it implies (the counter is summed over the GPU's XCDs, whose number
    the agent info file gives)."""
    import csv
    import glob
    per, dur, nxcc = {}, {}, 0
    for path in sorted(glob.glob(os.path.join(root, "**", "*agent_info.csv"), recursive=True)):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Agent_Type") == "GPU":
                    nxcc = int(r["Num_Xcc"])
    for path in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"),
                                 recursive=True)):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                i = int(r["Dispatch_Id"])
                d = per.setdefault(r["Kernel_Name"], {}).setdefault(i, {})
                d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                dur[i] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    out = {}
    for name, disp in per.items():
        ids = sorted(disp)[-last:]
        keys = sorted({k for i in ids for k in disp[i]})
        res = {"dispatches": len(disp), "last": len(ids),
               "duration_ms": round(sum(dur[i] for i in ids) / len(ids), 4),
               **{k: round(sum(disp[i].get(k, 0.0) for i in ids) / len(ids), 3) for k in keys}}
        if "GRBM_GUI_ACTIVE" in keys and nxcc:
            res["sclk_ghz"] = round(sum(disp[i]["GRBM_GUI_ACTIVE"] / nxcc / (dur[i] * 1e6)
                                        for i in ids) / len(ids), 3)
        out[name] = res
    return out


def warm(torch, fn, ms=WARM_MS):
    """Call fn until ms milliseconds have passed (at least three calls) and
    return the number of calls: after idle the chip takes tens of
    milliseconds under load to reach its working clock."""
    n = 0
    t0 = time.perf_counter()
    while n < 3 or (time.perf_counter() - t0) * 1e3 < ms:
        fn()
        torch.cuda.synchronize()
        n += 1
    return n


def _event_ms(torch, fn, steps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def gcm_leg(am, ks, iv, x, y, steps=10):
    """AES-GCM (SP 800-38D) over the same resident buffer: encryption,
    decryption, and GHASH alone.  The wide GHASH pass reads 16 B per block
    and, per 64 blocks (one wave step), issues 246 VALU ops per two blocks per
    lane (123 per block) and 16 ds_read_b128 + 14 ds_read_b32, which the gfx950
    LDS serves in 16 x 4 + 14 x 2 = 92 clocks per CU (measured: b128 at 16
    lanes per clock, b32 at 32)."""
    import torch
    n = x.numel()
    nblocks = n // 16
    ws = torch.empty(am.gcm_workspace_bytes(0, n), dtype=torch.uint8, device=x.device)
    tag = torch.empty(16, dtype=torch.uint8, device=x.device)
    enc = _event_ms(torch, lambda: am.gcm_encrypt(ks, iv, x, out=y, tag=tag, ws=ws), steps)
    dec = _event_ms(torch, lambda: am.gcm_decrypt(ks, iv, y, out=x, tag=tag, ws=ws), steps)
    gws = torch.empty(am.ghash_workspace_bytes(nblocks), dtype=torch.uint8, device=x.device)
    h = bytes(range(16))
    gh = _event_ms(torch, lambda: am.ghash(h, y, y=tag, ws=gws), steps)
    sec = gh * 1e-3
    valu = 123 * nblocks / (VALU_PEAK_TOPS * 1e12 * sec)
    lds = nblocks * 92 / 64 / (256 * 2.4e9 * sec)
    return {"workload": "aes128-gcm-%dMiB" % (n >> 20), "aad_bytes": 0,
            "enc_GBps": round(n / (enc * 1e-3) / 1e9, 1), "enc_ms": round(enc, 4),
            "dec_GBps": round(n / (dec * 1e-3) / 1e9, 1), "dec_ms": round(dec, 4),
            "ghash_ms": round(gh, 4), "ghash_GBps": round(n / sec / 1e9, 1),
            "ghash_hbm_frac": round(n / sec / 1e9 / HBM_PEAK_GBS, 4),
            "ghash_valu_frac_at_2p4ghz": round(valu, 4),
            "ghash_lds_frac_at_2p4ghz": round(lds, 4),
            "kernel": "ghash_pass_wide_kernel"}


def dbcolumn_leg(steps=20):
    """The database-column workload (sec. I: deterministic encryption for
    equality queries over encrypted data): 2^26 int64 values, Zipf s = 1.1
    over 2^20 distinct values, each zero-padded to a 16-byte block and
    encrypted with AES-256 ECB (1 GiB resident in HBM).  Encryption and
    decryption are timed after a warm-up each, and the round trip is checked
    on the device."""
    import torch
    import paper_1506_08503_amd as am
    from paper_1506_08503_amd import workloads as wl
    col = wl.dbcolumn_inputs()
    values = torch.from_numpy(col.values).cuda()
    ranks = torch.from_numpy(col.ranks).cuda()
    blocks = torch.zeros((ranks.numel(), 2), dtype=torch.int64, device="cuda")
    blocks[:, 0] = values[ranks]
    del values, ranks
    pt = blocks.view(torch.uint8).view(-1)
    ks = am.key_schedule(col.key)
    ct = torch.empty_like(pt)
    back = torch.empty_like(pt)
    enc = lambda: am.ecb_encrypt(ks, pt, out=ct)
    dec = lambda: am.ecb_decrypt(ks, ct, out=back)
    warm(torch, enc)
    t_enc = _event_ms(torch, enc, steps)
    warm(torch, dec)
    t_dec = _event_ms(torch, dec, steps)
    ok = bool(torch.equal(back, pt))
    n = pt.numel()
    return {"workload": "aes256-ecb-dbcolumn: 2^26 int64 (Zipf s=1.1 over 2^20 values), "
                        "zero-padded 16-B blocks, 1 GiB",
            "rows": n // 16,
            "enc_GBps": round(n / (t_enc * 1e-3) / 1e9, 1), "enc_ms": round(t_enc, 4),
            "dec_GBps": round(n / (t_dec * 1e-3) / 1e9, 1), "dec_ms": round(t_dec, 4),
            "rows_per_s_enc": round((n // 16) / (t_enc * 1e-3)),
            "round_trip_equal": ok}


def load_traffic(path, kernel):
    try:
        with open(path) as f:
            data = json.load(f)
        return data.get(kernel)
    except (OSError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the AES path needs no cross-GPU exchange; "
              "a multi-GPU run is one independent process per GPU over its own block "
              "range (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.last, args.split_gap_ms)),
              flush=True)
        return
    if args.pmc_summary:
        print(json.dumps(pmc_summary(args.pmc_summary, args.last)), flush=True)
        return
    import torch
    import paper_1506_08503_amd as am
    from paper_1506_08503_amd import workloads as wl

    if args.sweep:
        print(json.dumps(sweep_fig3()), flush=True)
        return
    if args.op.startswith("gcm") and args.layout == "bitslice":
        print("GCM runs on the table kernels (--layout auto|ttable)", file=sys.stderr)
        sys.exit(2)
    layout = {"auto": am.LAYOUT_AUTO, "ttable": am.LAYOUT_TTABLE,
              "bitslice": am.LAYOUT_BITSLICE}[args.layout]
    inp = wl.stream_inputs(wl.SEED_STREAM, args.nbytes, key_bytes=args.key_bytes)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x = torch.empty(inp.nbytes, dtype=torch.uint8, device=dev)
    if args.plaintext == "zero":
        x.zero_()
    else:
        for off, piece in inp.plaintext_chunks():
            x[off:off + piece.size].copy_(torch.from_numpy(piece))
    if args.key_seed is not None:
        kin = wl.stream_inputs(args.key_seed, args.nbytes, key_bytes=args.key_bytes)
        inp.key, inp.nonce = kin.key, kin.nonce
    y = torch.empty_like(x)
    ks = am.key_schedule(inp.key, dev)
    kw = {} if layout == am.LAYOUT_AUTO else {"layout": layout}
    if args.ctr_precompute:
        kw["ctr_precompute"] = args.ctr_precompute
    if args.op.startswith("gcm"):
        gws = torch.empty(am.gcm_workspace_bytes(0, inp.nbytes), dtype=torch.uint8, device=dev)
        gtag = torch.empty(16, dtype=torch.uint8, device=dev)

    def step():
        if args.mode == "copy":
            y.copy_(x)
        elif args.op == "ecb-enc":
            am.ecb_encrypt(ks, x, out=y, **kw)
        elif args.op == "ecb-dec":
            am.ecb_decrypt(ks, x, out=y, **kw)
        elif args.op == "gcm-enc":
            am.gcm_encrypt(ks, inp.nonce, x, out=y, tag=gtag, ws=gws)
        elif args.op == "gcm-dec":
            am.gcm_decrypt(ks, inp.nonce, x, out=y, tag=gtag, ws=gws)
        else:
            am.ctr_xcrypt(ks, inp.nonce, inp.ctr0, x, out=y, **kw)

    tuned = None
    if (not args.no_tune and args.mode == "aes" and args.layout == "auto"
            and not args.ctr_precompute and args.op in ("ctr", "ecb-enc", "ecb-dec")):
        # autotuned launch shape (after a warm-up, so that the candidates are
        # timed at the working clock); the timed steps use the winner
        from paper_1506_08503_amd import autotune
        warm(torch, step)
        best, table = autotune.tune_plain(args.op, inp.nbytes, args.key_bytes, cache_path=None,
                                          x=x, y=y)
        default_ms = next(ms for cand, ms in table if not cand)
        tuned = {"chosen": best, "chosen_ms": round(table[0][1], 4),
                 "library_default_ms": round(default_ms, 4), "candidates": len(table)}
        kw.update(best)
    if args.warmup >= 0:
        for _ in range(args.warmup):
            step()
    else:
        args.warmup = warm(torch, step)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    avg_ms = sum(kernel_ms) / len(kernel_ms)
    ms_per_step = wall * 1e3 / args.steps

    nblocks = (inp.nbytes + 15) // 16
    value = inp.nbytes / (ms_per_step * 1e-3) / 1e9
    alg_bytes = 32 * nblocks
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    bitslice = args.layout == "bitslice" or kw.get("layout") == am.LAYOUT_BITSLICE
    kernel_name = {("ctr", False): "ctr_grouped_kernel", ("ctr", True): "ctr_bitslice_kernel",
                   ("ecb-enc", False): "ecb_ttable_kernel<false, 0>",
                   ("ecb-enc", True): "ecb_bitslice_kernel<false>",
                   ("ecb-dec", False): "ecb_ttable_kernel<true, 0>",
                   ("ecb-dec", True): "ecb_bitslice_kernel<true>",
                   ("gcm-enc", False): "gcm step (ctr_grouped_kernel + ghash passes)",
                   ("gcm-dec", False): "gcm step (ghash passes + ctr_grouped_kernel)"}[
                       (args.op, bitslice)]
    bpl = kw.get("blocks_per_lane", 0) or 4
    if args.op == "ctr" and not bitslice and (args.ctr_precompute or bpl != 4):
        kernel_name = "ctr_ttable_kernel<%d, %s>" % (bpl, "false" if args.ctr_precompute == 2
                                                     else "true")
    default_cfg = (args.op, args.key_bytes, args.nbytes, args.layout,
                   args.ctr_precompute) == ("ctr", 16, 4 << 30, "auto", 0)
    # counters were taken for the default workload only (AES-128 CTR, 4 GiB)
    traffic = load_traffic(args.traffic_json, kernel_name) \
        if default_cfg and kernel_name == "ctr_grouped_kernel" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_source": ("not measured in this run: FETCH_SIZE + WRITE_SIZE per "
                                   "dispatch from two rocprofv3 --pmc runs of this command, "
                                   "scaled by a plain copy's counters (profiles/traffic.json)")
                if traffic else None,
                "kernel": kernel_name,
                "kernel_ms_avg": round(avg_ms, 4), "kernel_ms_min": round(min(kernel_ms), 4)}
    pr = None
    if not args.no_probes and args.mode == "aes":
        pr = probes()
    if not bitslice and not args.op.startswith("gcm"):
        # On-chip limit of the table kernels: LDS reads per block -- CTR:
        # 16 (Nr - 2) (rounds 1-2 come from per-thread and per-256-counter
        # group precomputation); ECB: 16 Nr -- against 32 reads/clk/CU.
        nr = {16: 10, 24: 12, 32: 14}[args.key_bytes]
        pre = args.ctr_precompute if bpl == 4 else max(args.ctr_precompute, 1)
        per_block = {0: 16 * (nr - 2), 1: 16 * nr - 12, 2: 16 * nr}[pre] \
            if args.op == "ctr" else 16 * nr
        lds_reads = per_block * nblocks
        roofline["lds_treads_per_s"] = round(lds_reads / (avg_ms * 1e-3) / 1e12, 3)
        roofline["lds_frac_at_2p4ghz"] = round(lds_reads / (avg_ms * 1e-3) / 1e12
                                               / LDS_PEAK_TREADS, 4)
        if kernel_name == "ctr_grouped_kernel" and args.key_bytes == 16:
            roofline["binding"] = binding_roofline(lds_reads, nblocks, avg_ms, pr)
    if args.mode == "copy":
        print(json.dumps({"mode": "copy", "nbytes": inp.nbytes, "ms_avg": round(avg_ms, 4),
                          "GBps_read_plus_write": round(2 * inp.nbytes / (avg_ms * 1e-3) / 1e9,
                                                        1)}), flush=True)
        return
    metric = "AES-128-CTR GB/s at 4 GiB"
    if args.op != "ctr" or args.key_bytes != 16 or args.nbytes != 4 << 30:
        metric = "AES-%d-%s GB/s at %d MiB" % (8 * args.key_bytes, args.op.upper(),
                                               args.nbytes >> 20)
    out = {"metric": metric, "value": round(value, 2), "unit": "GB/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u8",
           "data": "synthetic (PCG64 seed 0xAE502 uniform bytes)",
           "config": {"workload": "aes%d-%s-%dMiB" % (8 * args.key_bytes, args.op,
                                                         args.nbytes >> 20),
                      "nbytes": inp.nbytes,
                      "blocks": nblocks, "layout": args.layout, "in_place": False,
                      "ctr_precompute": args.ctr_precompute, "launch": dict(kw)},
           "roofline": roofline}
    if tuned:
        out["tune"] = tuned
    if not args.no_gcm and default_cfg:
        out["gcm"] = gcm_leg(am, ks, inp.nonce, x, y)
    del x, y
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_leg()
    if not args.no_serving:
        out["serving"] = serving_leg(args.serving_requests)
    if not args.no_sweep and default_cfg:
        out["sweep"] = sweep_fig3()
    if not args.no_dbcolumn and default_cfg:
        out["dbcolumn"] = dbcolumn_leg()
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(inp, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

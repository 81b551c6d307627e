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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--nbytes", type=int, default=4 << 30)
    p.add_argument("--layout", choices=["auto", "ttable", "bitslice"], default="auto")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--mode", choices=["aes", "copy"], default="aes",
                   help="copy: time a plain device copy of the same buffer instead "
                        "(reference for HBM counter calibration)")
    p.add_argument("--cpu-threads", type=int, default=0)
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return p.parse_args()


def cpu_baseline(inp, threads):
    """Oracle CTR (as it stands) on a bounded prefix of the same plaintext."""
    import numpy as np
    from oracle import oracle as orc
    o = orc.default()
    sample = min(inp.nbytes, (2 << 20) * threads)
    g = next(inp.plaintext_chunks(chunk=sample))[1]
    t0 = time.perf_counter()
    o.ctr_xcrypt(inp.key, inp.nonce, inp.ctr0, g, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample / dt / 1e9, 6), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d MiB of the 4 GiB AES-128-CTR plaintext, %d host threads, "
                      "%.2f s" % (sample >> 20, threads, dt)}


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
        print("bench.py measures one GPU only: the AES path needs no cross-GPU exchange "
              "and this build runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1506_08503_amd as am
    from paper_1506_08503_amd import workloads as wl

    layout = {"auto": am.LAYOUT_AUTO, "ttable": am.LAYOUT_TTABLE,
              "bitslice": am.LAYOUT_BITSLICE}[args.layout]
    inp = wl.stream_inputs(wl.SEED_STREAM, args.nbytes)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x = torch.empty(inp.nbytes, dtype=torch.uint8, device=dev)
    for off, piece in inp.plaintext_chunks():
        x[off:off + piece.size].copy_(torch.from_numpy(piece))
    y = torch.empty_like(x)
    ks = am.key_schedule(inp.key, dev)
    kw = {} if layout == am.LAYOUT_AUTO else {"layout": layout}

    def step():
        if args.mode == "copy":
            y.copy_(x)
        else:
            am.ctr_xcrypt(ks, inp.nonce, inp.ctr0, x, out=y, **kw)

    for _ in range(args.warmup):
        step()
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
    kernel_name = "ctr_ttable_kernel" if args.layout != "bitslice" else "ctr_bitslice_kernel"
    traffic = load_traffic(args.traffic_json, kernel_name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": kernel_name,
                "kernel_ms_avg": round(avg_ms, 4), "kernel_ms_min": round(min(kernel_ms), 4)}
    if args.layout != "bitslice":
        # On-chip limits of the table kernel: 148 LDS reads per AES-128 block
        # (4 in round 1, 16 in each of rounds 2..10) against 32 reads/clk/CU.
        lds_reads = 148 * nblocks
        roofline["lds_treads_per_s"] = round(lds_reads / (avg_ms * 1e-3) / 1e12, 3)
        roofline["lds_frac_at_2p4ghz"] = round(lds_reads / (avg_ms * 1e-3) / 1e12
                                               / LDS_PEAK_TREADS, 4)
    if args.mode == "copy":
        print(json.dumps({"mode": "copy", "nbytes": inp.nbytes, "ms_avg": round(avg_ms, 4),
                          "GBps_read_plus_write": round(2 * inp.nbytes / (avg_ms * 1e-3) / 1e9,
                                                        1)}), flush=True)
        return
    out = {"metric": "AES-128-CTR GB/s at 4 GiB", "value": round(value, 2), "unit": "GB/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u8",
           "data": "synthetic (PCG64 seed 0xAE502 uniform bytes)",
           "config": {"workload": "aes128-ctr-4GiB", "nbytes": inp.nbytes,
                      "blocks": nblocks, "layout": args.layout, "in_place": False},
           "roofline": roofline}
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(inp, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

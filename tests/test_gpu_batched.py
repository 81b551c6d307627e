"""GPU parity of the batched persistent kernel (aes_ctr_xcrypt_batched).

Every segment must equal the CPU oracle's CTR of that message alone, with its
own key, nonce and counter (tolerance 0), for both round-function layouts and
several tile sizes; invalid segments are reported and left untouched; graph
replays equal eager runs; the full 10,000-message workload equals a loop of
plain per-message launches and the oracle on every byte.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import paper_1506_08503_amd as am
from paper_1506_08503_amd import batch as bt
from paper_1506_08503_amd import autotune
from paper_1506_08503_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"

TUNES = [None,
         {"layout": am.LAYOUT_TTABLE, "tile_blocks": 64, "wg_size": 256, "grid_per_cu": 2},
         {"layout": am.LAYOUT_TTABLE, "tile_blocks": 256, "wg_size": 1024, "grid_per_cu": 1},
         {"layout": am.LAYOUT_TTABLE, "tile_blocks": 4096, "wg_size": 512, "grid_per_cu": 1},
         {"layout": am.LAYOUT_TTABLE, "tile_blocks": 1024, "wg_size": 1024, "grid_per_cu": 1,
          "blocks_per_lane": 2},
         {"layout": am.LAYOUT_TTABLE, "tile_blocks": 512, "wg_size": 256, "grid_per_cu": 4,
          "blocks_per_lane": 1},
         {"layout": am.LAYOUT_BITSLICE, "tile_blocks": 2048, "wg_size": 256, "grid_per_cu": 2},
         {"layout": am.LAYOUT_BITSLICE, "tile_blocks": 4096, "wg_size": 64, "grid_per_cu": 4},
         # library default tile and shape of each layout
         {"layout": am.LAYOUT_TTABLE},
         {"layout": am.LAYOUT_BITSLICE}]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def mixed_case(seed=77, nrandom=300):
    """Messages of edge-case and random lengths, 128/192/256-bit keys, counters
    aligned and unaligned to 256, some close to the 2^32 limit."""
    g = _rng(seed)
    edge = [0, 1, 15, 16, 17, 31, 32, 33, 16 * 255, 16 * 256, 16 * 256 + 1, 16 * 2048,
            16 * 2049 + 7, 16 * 4096 * 3 + 5]
    lengths = np.array(edge + wl.log_uniform_lengths(g, nrandom, 1 << 18).tolist(), np.int64)
    n = lengths.size
    key_bytes = g.choice([16, 24, 32], size=n)
    keys = [g.bytes(int(k)) for k in key_bytes]
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    ctr0 = np.where(g.random(n) < 0.5, 0, g.integers(0, 2 ** 31, size=n)).astype(np.uint64)
    ctr0[:4] = [2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 1, 2 ** 32 - 2]   # 0/1/1/2 blocks
    ctr0[5] = 2 ** 32 - 2                                            # 17 bytes: 2 blocks
    nblk = (lengths + 15) // 16
    assert np.all(ctr0 + nblk <= 2 ** 32)
    in_off, total = wl.pack_offsets(lengths)
    # outputs land in a different order with gaps, to catch offset mix-ups
    perm = g.permutation(n)
    out_off = np.zeros(n, np.int64)
    pos = 0
    for i in perm:
        out_off[i] = pos
        pos += (int(lengths[i]) + 15) // 16 * 16 + 16 * int(g.integers(0, 3))
    pt = np.frombuffer(g.bytes(total), np.uint8).copy()
    return dict(lengths=lengths, keys=keys, nonces=nonces, ctr0=ctr0.astype(np.uint32),
                in_off=in_off, out_off=out_off, pt=pt, out_total=pos)


def key_table(keys, device=DEV):
    return torch.stack([am.key_schedule(k, device) for k in keys])


def oracle_all(oracle, case):
    def one(i):
        a, n = int(case["in_off"][i]), int(case["lengths"][i])
        return oracle.ctr_xcrypt(case["keys"][i], case["nonces"][i].tobytes(),
                                 int(case["ctr0"][i]), case["pt"][a:a + n])
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(one, range(case["lengths"].size)))


@pytest.fixture(scope="module")
def mixed(oracle):
    case = mixed_case()
    case["expected"] = oracle_all(oracle, case)
    return case


def run_case(case, tune, in_place=False):
    n = case["lengths"].size
    segs_h = bt.segment_table(case["in_off"], case["in_off"] if in_place else case["out_off"],
                              case["lengths"], np.arange(n, dtype=np.uint32), case["ctr0"],
                              case["nonces"])
    segs = torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV)
    kt = key_table(case["keys"])
    x = torch.from_numpy(case["pt"]).to(DEV)
    out = x if in_place else torch.full((case["out_total"] + 16,), 0xA5, dtype=torch.uint8,
                                        device=DEV)
    ws = bt.workspace(n, DEV)
    am.ctr_xcrypt_batched(segs, kt, x, out, ws, tune)
    assert am.batched_read_status(ws) == 0
    return out.cpu().numpy(), ws


def _tune_id(t):
    if t is None:
        return "default"
    return "%s-t%d-w%d-g%d-b%d" % ("bs" if t["layout"] == 2 else "tt", t.get("tile_blocks", 0),
                                  t.get("wg_size", 0), t.get("grid_per_cu", 0),
                                  t.get("blocks_per_lane", 0))


@pytest.mark.parametrize("tune", TUNES, ids=_tune_id)
def test_batched_mixed_matches_oracle(mixed, tune):
    out, _ = run_case(mixed, tune)
    off = mixed["out_off"]
    for i, exp in enumerate(mixed["expected"]):
        got = out[int(off[i]):int(off[i]) + exp.size]
        assert np.array_equal(got, exp), (i, int(mixed["lengths"][i]), int(mixed["ctr0"][i]))
    # bytes outside every segment stay untouched
    mask = np.ones(out.size, bool)
    for i, exp in enumerate(mixed["expected"]):
        mask[int(off[i]):int(off[i]) + exp.size] = False
    assert np.all(out[mask] == 0xA5)


def test_batched_in_place(mixed):
    out, _ = run_case(mixed, None, in_place=True)
    for i, exp in enumerate(mixed["expected"]):
        a = int(mixed["in_off"][i])
        assert np.array_equal(out[a:a + exp.size], exp), i


def test_batched_invalid_segments(oracle):
    g = _rng(9)
    n = 8
    lengths = np.full(n, 16 * 300 + 3, np.int64)
    in_off, total = wl.pack_offsets(lengths)
    keys = [g.bytes(16) for _ in range(4)]
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    slots = np.array([0, 1, 4, 2, 3, 0, 1, 2], np.uint32)       # slot 4 does not exist
    ctr0 = np.zeros(n, np.uint32)
    ctr0[6] = 2 ** 32 - 10                                       # counter overflow
    segs_h = bt.segment_table(in_off, in_off, lengths, slots, ctr0, nonces)
    segs_h["in_off"][4] += 8                                     # misaligned
    segs_h["reserved"][5] = 1                                    # reserved must be 0
    pt = np.frombuffer(g.bytes(total + 16), np.uint8).copy()
    x = torch.from_numpy(pt).to(DEV)
    out = torch.full_like(x, 0x5A)
    ws = bt.workspace(n, DEV)
    am.ctr_xcrypt_batched(torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV),
                          key_table(keys), x, out, ws)
    assert am.batched_read_status(ws) == -7          # AES_ERR_SEGMENT
    o = out.cpu().numpy()
    for i in range(n):
        a, ln = int(in_off[i]), int(lengths[i])
        if i in (2, 4, 5, 6):
            assert np.all(o[a:a + ln] == 0x5A), i
        else:
            exp = oracle.ctr_xcrypt(keys[slots[i]], nonces[i].tobytes(), 0, pt[a:a + ln])
            assert np.array_equal(o[a:a + ln], exp), i


BITSLICE_TUNE = next(t for t in TUNES if t and t["layout"] == am.LAYOUT_BITSLICE)


@pytest.mark.parametrize("tune", [None, BITSLICE_TUNE], ids=["ttable", "bitslice"])
def test_batched_invalid_key_schedule(oracle, tune):
    """A key slot whose schedule has no valid round count: its segments are
    left untouched and the status says AES_ERR_SEGMENT; the others are right."""
    g = _rng(10)
    n = 6
    lengths = np.array([16 * 4096 + 5, 100, 16 * 5000, 33, 16 * 2048, 7], np.int64)
    in_off, total = wl.pack_offsets(lengths)
    keys = [g.bytes(16) for _ in range(3)]
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    slots = np.array([0, 1, 2, 1, 0, 2], np.uint32)
    segs_h = bt.segment_table(in_off, in_off, lengths, slots, np.zeros(n, np.uint32), nonces)
    pt = np.frombuffer(g.bytes(total + 16), np.uint8).copy()
    x = torch.from_numpy(pt).to(DEV)
    out = torch.full_like(x, 0x5A)
    table = key_table(keys)
    table[1, 0:4] = torch.tensor([9, 0, 0, 0], dtype=torch.uint8)   # nr = 9
    ws = bt.workspace(n, DEV)
    am.ctr_xcrypt_batched(torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV), table, x,
                          out, ws, tune)
    assert am.batched_read_status(ws) == -7
    o = out.cpu().numpy()
    for i in range(n):
        a, ln = int(in_off[i]), int(lengths[i])
        if slots[i] == 1:
            assert np.all(o[a:a + ln] == 0x5A), i
        else:
            exp = oracle.ctr_xcrypt(keys[slots[i]], nonces[i].tobytes(), 0, pt[a:a + ln])
            assert np.array_equal(o[a:a + ln], exp), i


@pytest.mark.parametrize("nsegs,pattern", [(9, "empties"), (20000, "many")])
def test_batched_empty_runs_and_large_tables(oracle, nsegs, pattern):
    """Runs of empty segments (at the start, inside and at the end of the
    table: they share their tile start with the next segment), and a table
    larger than the prepare kernel keeps in LDS (tile counts then go through
    global memory)."""
    g = _rng(11 + nsegs)
    if pattern == "empties":
        lengths = np.array([0, 0, 100, 0, 0, 16 * 5000 + 3, 0, 0, 0], np.int64)
    else:
        lengths = g.integers(0, 600, size=nsegs).astype(np.int64)
        lengths[::7] = 0
        lengths[-50:] = 0
    n = lengths.size
    in_off, total = wl.pack_offsets(lengths)
    keys = [g.bytes(16) for _ in range(4)]
    slots = g.integers(0, 4, size=n).astype(np.uint32)
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    ctr0 = g.integers(0, 2 ** 20, size=n).astype(np.uint32)
    segs_h = bt.segment_table(in_off, in_off, lengths, slots, ctr0, nonces)
    pt = np.frombuffer(g.bytes(total + 16), np.uint8).copy()
    x = torch.from_numpy(pt).to(DEV)
    out = torch.full_like(x, 0x5A)
    ws = bt.workspace(n, DEV)
    am.ctr_xcrypt_batched(torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV),
                          key_table(keys), x, out, ws)
    assert am.batched_read_status(ws) == 0
    o = out.cpu().numpy()
    exp = np.full_like(pt, 0x5A)
    for i in range(n):
        a, ln = int(in_off[i]), int(lengths[i])
        if ln:
            exp[a:a + ln] = oracle.ctr_xcrypt(keys[slots[i]], nonces[i].tobytes(), int(ctr0[i]),
                                              pt[a:a + ln])
    assert np.array_equal(o, exp)


@pytest.mark.parametrize("tile,bpl", [(256, 4), (1024, 4), (1024, 2), (320, 4)])
def test_batched_tile_remainders(oracle, tile, bpl):
    """The last pass of a tile: every remainder of 1 to 256 blocks after the
    whole four-block passes (one, two, three or four blocks per lane), with
    and without a partial last block in each of its slots, counters aligned
    and not aligned to 256-counter groups; outputs land in a buffer whose
    other bytes must stay untouched."""
    g = _rng(12 + tile + bpl)
    rest = np.concatenate([np.arange(1, 257), g.integers(1, 257, size=60)])
    whole = g.integers(0, 3, size=rest.size) * 256
    tails = g.integers(0, 16, size=rest.size)
    lengths = ((whole + rest - (tails > 0)) * 16 + tails).astype(np.int64)
    n = lengths.size
    in_off, total = wl.pack_offsets(lengths)
    out_off = in_off + 16 * np.arange(n)              # a 16-byte gap after every message
    keys = [g.bytes(16), g.bytes(32)]
    slots = (np.arange(n) % 2).astype(np.uint32)
    nonces = np.frombuffer(g.bytes(12 * n), np.uint8).reshape(n, 12)
    ctr0 = np.where(np.arange(n) % 3 == 0, 0, g.integers(0, 2 ** 24, size=n)).astype(np.uint32)
    segs_h = bt.segment_table(in_off, out_off, lengths, slots, ctr0, nonces)
    pt = np.frombuffer(g.bytes(total + 16), np.uint8).copy()
    x = torch.from_numpy(pt).to(DEV)
    out = torch.full((total + 16 * n + 16,), 0xA5, dtype=torch.uint8, device=DEV)
    ws = bt.workspace(n, DEV)
    am.ctr_xcrypt_batched(torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV),
                          key_table(keys), x, out, ws,
                          {"layout": am.LAYOUT_TTABLE, "tile_blocks": tile, "blocks_per_lane": bpl})
    assert am.batched_read_status(ws) == 0
    o = out.cpu().numpy()
    exp = np.full(o.size, 0xA5, np.uint8)
    for i in range(n):
        a, b, ln = int(in_off[i]), int(out_off[i]), int(lengths[i])
        exp[b:b + ln] = oracle.ctr_xcrypt(keys[slots[i]], nonces[i].tobytes(), int(ctr0[i]),
                                          pt[a:a + ln])
    bad = np.flatnonzero(o != exp)
    assert bad.size == 0, (bad[:8], lengths[np.searchsorted(out_off, bad[0], "right") - 1])


def test_batched_graph_replays(mixed):
    """A captured graph replayed three times, the input rewritten in place with
    eager work and synchronizations in between; every replay equals an eager
    batched run on the same data."""
    n = mixed["lengths"].size
    segs_h = bt.segment_table(mixed["in_off"], mixed["out_off"], mixed["lengths"],
                              np.arange(n, dtype=np.uint32), mixed["ctr0"], mixed["nonces"])
    segs = torch.from_numpy(segs_h.view(np.uint8).copy()).to(DEV)
    kt = key_table(mixed["keys"])
    x = torch.from_numpy(mixed["pt"]).to(DEV)
    out = torch.zeros(mixed["out_total"] + 16, dtype=torch.uint8, device=DEV)
    ws = bt.workspace(n, DEV)
    graph = am.BatchedGraph(segs, kt, x, out, ws)
    ref_out = torch.zeros_like(out)
    ws2 = bt.workspace(n, DEV)
    try:
        for rep in range(3):
            x.add_(rep + 1)                       # new data in the same buffer (eager)
            torch.cuda.synchronize()
            graph.launch()
            torch.cuda.synchronize()
            am.ctr_xcrypt_batched(segs, kt, x, ref_out, ws2)
            torch.cuda.synchronize()
            assert torch.equal(out, ref_out), rep
            assert am.batched_read_status(ws) == 0
    finally:
        graph.close()


def test_autotune_small():
    """The tuner times every candidate on the caller's batch and its pick gives
    the same bytes as the default launch and as one plain launch per message."""
    db = bt.DeviceBatch(wl.batched_inputs(nmsg=300, max_len=1 << 18, seed=5), DEV)
    best, table = autotune.tune_batched(db, reps=1, cache_path=None)
    assert table and best == table[0][0]
    ref = db.run(None).clone()
    assert torch.equal(db.run(best), ref)
    db.out.zero_()
    assert torch.equal(db.run_plain_loop(), ref)


@pytest.mark.slow
def test_batched_full_workload(oracle):
    """10,000 messages, log-uniform 1 B .. 1 MiB, own AES-128 keys and nonces
    (0.68 GiB): one persistent launch equals 10,000 plain launches byte for
    byte, so does every launch shape the benchmark's autotuner tries (it
    times whichever wins on the box), and the oracle agrees on every byte of
    every message (about 10 s on 16 host threads)."""
    b = wl.batched_inputs()
    db = bt.DeviceBatch(b, DEV)
    got = db.run().clone()
    assert db.status() == 0
    db.out.zero_()
    loop = db.run_plain_loop().clone()
    assert torch.equal(got, loop)
    for cand in autotune.candidates():
        db.out.zero_()
        db.run(cand)
        assert db.status() == 0, cand
        assert torch.equal(db.out, got), cand
    pt = db.x.cpu().numpy()
    out = got.cpu().numpy()

    def check(i):
        a, n = int(b.offsets[i]), int(b.lengths[i])
        exp = oracle.ctr_xcrypt(b.keys[i].tobytes(), b.nonces[i].tobytes(), 0, pt[a:a + n])
        return np.array_equal(out[a:a + n], exp)
    # largest messages first so that the threads finish together
    order = np.argsort(-b.lengths, kind="stable").tolist()
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        bad = [i for i, ok in zip(order, ex.map(check, order)) if not ok]
    assert not bad, bad[:10]

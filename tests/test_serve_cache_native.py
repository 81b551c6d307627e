"""The serving loop's C++ key cache (csrc/serve_cache.hpp, built here with
g++, no GPU) against the Python model serve.KeyCache: random sequences of
batch takes and releases give the same prefix length, the same rows filled
for the same keys, the same hit and miss counts and the same final mapping;
with a row cap the C++ cache never takes more rows than the cap."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1506_08503_amd import serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1506_08503_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = tmp_path_factory.mktemp("cache") / "serve_cache_driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC,
                    os.path.join(ROOT, "tests", "serve_cache_driver.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


def _script(seed, nkeys, nslots, steps, cap, max_inflight=3):
    """Commands and the Python model's expected output lines."""
    g = np.random.Generator(np.random.PCG64(seed))
    kc = serve.KeyCache(nslots, nkeys)
    cmds, expect, inflight = ["%d %d" % (nkeys, nslots)], [], []
    ntake = 0
    # skewed key popularity: a few hot keys, a long tail
    p = 1.0 / np.arange(1, nkeys + 1) ** 0.8
    p /= p.sum()
    for _ in range(steps):
        if inflight and (len(inflight) >= max_inflight or g.random() < 0.4):
            b, slots = inflight.pop(0)
            cmds.append("R %d" % b)
            kc.release(slots)
            continue
        ids = g.choice(nkeys, size=int(g.integers(1, 120)), p=p)
        cmds.append("T %d %d %s" % (cap, ids.size, " ".join(map(str, ids))))
        k, res = kc.take(ids)
        fills = res[2] if res is not None else []
        expect.append("T %d %d %d %d%s" % (k, kc.hits, kc.misses, len(fills),
                                           "".join(" %d %d" % f for f in fills)))
        if k:
            inflight.append((ntake, res[1]))
        ntake += 1
    cmds.append("S")
    expect.append(" ".join(str(int(x)) for x in kc.slot_of))
    return "\n".join(cmds) + "\n", expect


@pytest.mark.parametrize("seed,nkeys,nslots", [(1, 8, 4), (2, 50, 16), (3, 300, 64),
                                               (4, 1024, 256), (5, 40, 40), (6, 20, 64)])
def test_native_cache_equals_python_model(driver, seed, nkeys, nslots):
    script, expect = _script(seed, nkeys, nslots, steps=400, cap=nslots)
    out = subprocess.run([driver], input=script, capture_output=True, text=True, check=True)
    got = [l.strip() for l in out.stdout.splitlines()]
    assert len(got) == len(expect)
    for i, (a, b) in enumerate(zip(got, expect)):
        assert a == b.strip(), (i, a[:200], b[:200])


def test_native_cache_row_cap(driver):
    """With a cap of 5 rows per take: every take pins at most 5 rows that
    were unpinned (misses plus hits on unpinned rows), and no row holds two
    keys."""
    g = np.random.Generator(np.random.PCG64(9))
    nkeys, nslots, cap = 60, 16, 5
    cmds, takes = ["%d %d" % (nkeys, nslots)], []
    for t in range(60):
        ids = g.integers(0, nkeys, size=int(g.integers(1, 80)))
        cmds.append("T %d %d %s" % (cap, ids.size, " ".join(map(str, ids))))
        takes.append(ids)
        if t % 2:
            cmds.append("R %d" % (t - 1))
            cmds.append("R %d" % t)
        cmds.append("S")
    out = subprocess.run([driver], input="\n".join(cmds) + "\n", capture_output=True,
                         text=True, check=True).stdout.splitlines()
    pinned = set()              # rows pinned by the take before (odd takes release both)
    rows_before = None
    for t, ids in enumerate(takes):
        tl, sl = out[2 * t].split(), out[2 * t + 1].split()
        k = int(tl[1])
        slot_of = np.array([int(x) for x in sl])
        assert k >= 1                                  # the first request always fits a free cap
        assert len(set(slot_of[slot_of >= 0].tolist())) == int((slot_of >= 0).sum())
        distinct = set(ids[:k].tolist())
        rows = {int(slot_of[key]) for key in distinct}
        assert all(r >= 0 for r in rows)
        assert len(rows - pinned) <= cap
        if k < ids.size:                               # the next distinct key would need a row
            nxt = int(ids[k])
            assert nxt not in distinct
        pinned = set() if t % 2 else rows
        rows_before = slot_of
    assert rows_before is not None

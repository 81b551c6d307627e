"""The C-ABI library on the host: symbols, host key expansion, argument checks.

No GPU needed: every call here either is pure host code (aes_expand_key,
aes_status_string, aes_batched_workspace_bytes) or fails argument validation,
which the library does before any HIP call.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_1506_08503_amd as am

L = am.lib()
VP = ctypes.c_void_p


def test_every_header_function_is_exported():
    names = am.header_functions()
    assert "aes_ctr_xcrypt" in names and len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", am.aesmi.LIB_PATH],
                         stdout=subprocess.PIPE, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)


def _words_to_bytes(words, n):
    return np.array(words[:n], dtype="<u4").view(np.uint8)


@pytest.mark.parametrize("key_bytes", [16, 24, 32])
def test_host_key_schedule_matches_oracle(oracle, key_bytes):
    g = np.random.Generator(np.random.PCG64(key_bytes))
    keys = [g.bytes(key_bytes) for _ in range(20)] + [b"\xff" * key_bytes,
                                                     b"\x00" * key_bytes]
    for key in keys:
        ks = am.expand_key(key)
        nr, rk = oracle.expand_key(key)
        assert ks.nr == nr and ks.key_bytes == key_bytes
        enc = _words_to_bytes(list(ks.rk_enc), 4 * (nr + 1))
        assert np.array_equal(enc, rk)
        # equivalent inverse cipher keys: reversed, InvMixColumns on inner keys
        dec = _words_to_bytes(list(ks.rk_dec), 4 * (nr + 1)).reshape(nr + 1, 16)
        rkr = rk.reshape(nr + 1, 16)
        assert np.array_equal(dec[0], rkr[nr]) and np.array_equal(dec[nr], rkr[0])
        for r in range(1, nr):
            assert np.array_equal(dec[r], oracle.inv_mix_columns(rkr[nr - r]))
        assert all(w == 0 for w in list(ks.rk_enc)[4 * (nr + 1):])


def _status(fn, *args):
    return fn(*args)


def test_expand_key_errors():
    ks = am.KeySchedule()
    assert L.aes_expand_key(None, 16, ctypes.byref(ks)) == -1
    buf = ctypes.create_string_buffer(32)
    for bad in (0, 8, 15, 17, 20, 31, 33, 64):
        assert L.aes_expand_key(buf, bad, ctypes.byref(ks)) == -2
    with pytest.raises(am.AesError, match="AES_ERR_KEYLEN"):
        am.expand_key(b"x" * 15)
    assert L.aes_expand_keys_device(VP(0x1000), 17, 4, VP(0x2000), None) == -2
    assert L.aes_expand_keys_device(VP(0x1000), 16, 0, None, None) == 0
    assert L.aes_expand_keys_device(None, 16, 3, VP(0x2000), None) == -1


def test_ecb_validation():
    ks, a, b = VP(0x10000), VP(0x20000), VP(0x40000)
    for fn in (L.aes_ecb_encrypt, L.aes_ecb_decrypt):
        assert fn(None, None, None, 0, None) == 0              # empty: no-op
        assert fn(None, a, b, 16, None) == -1
        assert fn(ks, None, b, 16, None) == -1
        assert fn(ks, a, None, 16, None) == -1
        assert fn(ks, a, b, 17, None) == -3
        assert fn(ks, VP(0x20008), b, 32, None) == -4
        assert fn(ks, a, VP(0x40004), 32, None) == -4
        assert fn(ks, a, VP(0x20010), 64, None) == -5            # partial overlap
        assert fn(ks, VP(0x20010), a, 64, None) == -5
    bad = am.Launch(0, 100, 0, 0)
    assert L.aes_ecb_encrypt_ex(ks, a, b, 32, ctypes.byref(bad), None) == -9
    bad = am.Launch(7, 0, 0, 0)
    assert L.aes_ecb_decrypt_ex(ks, a, b, 32, ctypes.byref(bad), None) == -9
    bad = am.Launch(1, 256, 0, 3)
    assert L.aes_ecb_encrypt_ex(ks, a, b, 32, ctypes.byref(bad), None) == -9
    bad = am.Launch(2, 512, 0, 0)                       # bitsliced: at most 256 threads
    assert L.aes_ecb_encrypt_ex(ks, a, b, 32, ctypes.byref(bad), None) == -9


def test_ctr_validation():
    ks, a, b = VP(0x10000), VP(0x20000), VP(0x40000)
    nonce = ctypes.create_string_buffer(12)
    f = L.aes_ctr_xcrypt
    assert f(None, None, 0, None, None, 0, None) == 0
    assert f(ks, None, 0, a, b, 5, None) == -1
    assert f(None, nonce, 0, a, b, 5, None) == -1
    assert f(ks, nonce, 0, VP(0x20001), b, 5, None) == -4
    assert f(ks, nonce, 0, a, VP(0x20008), 64, None) == -4
    assert f(ks, nonce, 0, a, VP(0x20010), 64, None) == -5
    # counter space: ctr0 + ceil(n / 16) must stay <= 2^32
    assert f(ks, nonce, 2 ** 32 - 1, a, b, 17, None) == -6
    assert f(ks, nonce, 2 ** 32 - 2, a, b, 33, None) == -6
    bad = am.Launch(0, 2048, 0, 0)
    assert L.aes_ctr_xcrypt_ex(ks, nonce, 0, a, b, 16, ctypes.byref(bad), None) == -9
    bad = am.Launch(1, 0, 0, 4, 3)                      # ctr_precompute is 0, 1 or 2
    assert L.aes_ctr_xcrypt_ex(ks, nonce, 0, a, b, 16, ctypes.byref(bad), None) == -9
    # status strings
    for code, name in am.STATUS.items():
        assert L.aes_status_string(code)
    assert L.aes_status_string(12345) == b"unknown status"


def test_cbc_validation():
    ks, iv, a, b = VP(0x10000), VP(0x30000), VP(0x20000), VP(0x40000)
    for f in (L.aes_cbc_encrypt, L.aes_cbc_decrypt):
        assert f(None, None, 16, None, None, 0, 32, None) == 0
        assert f(None, None, 16, None, None, 5, 0, None) == 0
        assert f(None, iv, 16, a, b, 4, 32, None) == -1
        assert f(ks, None, 16, a, b, 4, 32, None) == -1
        assert f(ks, iv, 16, a, b, 4, 24, None) == -3
        assert f(ks, iv, 8, a, b, 4, 32, None) == -9
        assert f(ks, VP(0x30008), 16, a, b, 4, 32, None) == -4
        assert f(ks, iv, 0, a, VP(0x20010), 4, 32, None) == -5
    assert L.aes_cbc_decrypt(ks, iv, 16, a, a, 4, 32, None) == -5   # no in-place decrypt


def test_batched_validation():
    segs, kt, a, b, ws = VP(0x10000), VP(0x20000), VP(0x40000), VP(0x80000), VP(0x100000)
    f = L.aes_ctr_xcrypt_batched
    need = L.aes_batched_workspace_bytes(10)
    assert need >= 256 and L.aes_batched_workspace_bytes(1000) > need
    assert f(None, 0, None, 0, None, None, None, None, 0, None) == 0
    assert f(None, 10, kt, 4, a, b, None, ws, need, None) == -1
    assert f(segs, 10, kt, 0, a, b, None, ws, need, None) == -7
    assert f(segs, 10, kt, 4, a, b, None, VP(0x100010), need, None) == -4
    assert f(segs, 10, kt, 4, a, b, None, ws, need - 1, None) == -9
    bad = am.BatchTune(0, 0, 0, 100)
    assert f(segs, 10, kt, 4, a, b, ctypes.byref(bad), ws, need, None) == -9
    for bpl in (3, 8):
        bad = am.BatchTune(am.LAYOUT_TTABLE, 0, 0, 0, bpl)
        assert f(segs, 10, kt, 4, a, b, ctypes.byref(bad), ws, need, None) == -9
    # the bitsliced layout: at most 256 threads, tiles of whole 2048-block batches
    for bad in (am.BatchTune(am.LAYOUT_BITSLICE, 512, 0, 0),
                am.BatchTune(am.LAYOUT_BITSLICE, 0, 0, 1024)):
        assert f(segs, 10, kt, 4, a, b, ctypes.byref(bad), ws, need, None) == -9
    st = ctypes.c_int32(0)
    assert L.aes_batched_read_status(None, None, ctypes.byref(st)) == -1
    g = VP()
    assert L.aes_batched_graph_create(segs, 10, kt, 4, a, b, None, ws, 1, None, None) == -1
    assert L.aes_batched_graph_destroy(None) == 0
    assert L.aes_batched_graph_launch(None, None) == -1


def test_server_validation():
    """aes_server_create / _run / _destroy check keys, parameters and the
    trace before any HIP call."""
    keys32 = np.zeros((2, 32), np.uint8)
    klen = np.array([16, 32], np.uint8)
    prm = am.ServeParams(16, 2, 1024, 1, 1 << 30, 1 << 26, 50e-6)
    h = VP(123)
    assert L.aes_server_create(keys32.ctypes.data, klen.ctypes.data, 2, ctypes.byref(prm),
                               None) == -1
    assert L.aes_server_create(None, klen.ctypes.data, 2, ctypes.byref(prm),
                               ctypes.byref(h)) == -1 and not h.value
    bad = am.ServeParams(16, 0, 1024, 1, 1 << 30, 1 << 26, 50e-6)
    assert L.aes_server_create(keys32.ctypes.data, klen.ctypes.data, 2, ctypes.byref(bad),
                               ctypes.byref(h)) == -9
    k2 = np.array([16, 17], np.uint8)
    assert L.aes_server_create(keys32.ctypes.data, k2.ctypes.data, 2, ctypes.byref(prm),
                               ctypes.byref(h)) == -2
    st = am.ServeStats()
    reqs = np.zeros(1, dtype=am.serve_request_dtype())
    reqs["nbytes"] = 16
    lat, off = np.zeros(1), np.zeros(1, np.uint64)
    assert L.aes_server_run(None, reqs.ctypes.data, 1, VP(0x100000), 1 << 20, VP(0x400000),
                            1 << 20, lat.ctypes.data, off.ctypes.data, ctypes.byref(st)) == -1
    assert L.aes_server_destroy(None) == 0


def test_batched_noalloc_validation():
    """The allocation-free batched call checks its arguments before any HIP
    call: more segments than its static workspace holds, a bad tune or a
    misaligned status pointer are refused."""
    segs, kt, a, b, stp = VP(0x10000), VP(0x20000), VP(0x40000), VP(0x80000), VP(0x100000)
    f = L.aes_ctr_xcrypt_batched_noalloc
    assert am.NOALLOC_MAX_SEGS == 65536
    assert f(None, 0, None, 0, None, None, None, None, None) == 0
    assert f(None, 10, kt, 4, a, b, None, stp, None) == -1
    assert f(segs, 10, kt, 0, a, b, None, stp, None) == -7
    assert f(segs, 10, kt, 4, VP(0x40008), b, None, stp, None) == -4
    assert f(segs, 10, kt, 4, a, b, None, VP(0x100002), None) == -4
    assert f(segs, 65537, kt, 4, a, b, None, stp, None) == -9
    bad = am.BatchTune(am.LAYOUT_TTABLE, 0, 0, 0, 3)
    assert f(segs, 10, kt, 4, a, b, ctypes.byref(bad), stp, None) == -9


def test_binding_rejects_cpu_tensors():
    import torch
    x = torch.zeros(32, dtype=torch.uint8)
    with pytest.raises(TypeError):
        am.ctr_xcrypt(x, b"n" * 12, 0, x)
    with pytest.raises(TypeError):
        am.ecb_encrypt(x, x)


def test_gcm_and_ghash_validation():
    ks, iv, a, b = VP(0x10000), ctypes.create_string_buffer(12), VP(0x20000), VP(0x40000)
    tag, ws, aad = VP(0x60000), VP(0x100000), VP(0x70000)
    need = L.aes_gcm_workspace_bytes(0, 64)
    assert need >= 256 and L.aes_gcm_workspace_bytes(16, 1 << 30) > need
    for f in (L.aes_gcm_encrypt, L.aes_gcm_decrypt):
        assert f(None, iv, None, 0, a, b, 64, tag, ws, need, None) == -1
        assert f(ks, None, None, 0, a, b, 64, tag, ws, need, None) == -1
        assert f(ks, iv, None, 0, a, b, 64, None, ws, need, None) == -1
        assert f(ks, iv, None, 0, a, b, 64, tag, None, need, None) == -1
        assert f(ks, iv, None, 16, a, b, 64, tag, ws, need, None) == -1     # aad missing
        assert f(ks, iv, None, 0, None, b, 64, tag, ws, need, None) == -1
        assert f(ks, iv, None, 0, VP(0x20004), b, 64, tag, ws, need, None) == -4
        assert f(ks, iv, VP(0x70001), 3, a, b, 64, tag, ws, need, None) == -4
        assert f(ks, iv, None, 0, a, b, 64, VP(0x60008), ws, need, None) == -4
        assert f(ks, iv, None, 0, a, b, 64, tag, VP(0x100080), need, None) == -4
        assert f(ks, iv, None, 0, a, VP(0x20010), 64, tag, ws, need, None) == -5
        assert f(ks, iv, None, 0, a, b, 64, tag, ws, need - 1, None) == -9
        assert f(ks, iv, aad, 1 << 61, a, b, 64, tag, ws, need, None) == -3
        # at most 2^32 - 2 blocks (counters 2 .. 2^32 - 1)
        big = (2 ** 32 - 1) * 16
        assert f(ks, iv, None, 0, VP(1 << 44), VP(1 << 45), big, tag, ws, 1 << 40, None) == -6
    h = ctypes.create_string_buffer(16)
    gneed = L.aes_ghash_workspace_bytes(100)
    assert L.aes_ghash(None, a, 100, tag, ws, gneed, None) == -1
    assert L.aes_ghash(h, None, 100, tag, ws, gneed, None) == -1
    assert L.aes_ghash(h, VP(0x20008), 100, tag, ws, gneed, None) == -4
    assert L.aes_ghash(h, a, 100, tag, ws, gneed - 1, None) == -9


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message, before
    it touches torch or the GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_locals_do_not_shadow_its_functions():
    """bench.py's GPU legs cannot run here; at least no function (or a
    function nested in it) assigns a name that shadows a module-level function
    it also calls, the mistake that would only surface on the GPU."""
    import ast
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    tree = ast.parse(open(os.path.join(root, "bench.py")).read())
    module_funcs = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    bad = []
    for fn in ast.walk(tree):
        if not isinstance(fn, ast.FunctionDef):
            continue
        stored = {n.id for n in ast.walk(fn) if isinstance(n, ast.Name)
                  and isinstance(n.ctx, ast.Store)}
        stored |= {a.arg for a in fn.args.args}
        called = {n.func.id for n in ast.walk(fn) if isinstance(n, ast.Call)
                  and isinstance(n.func, ast.Name)}
        bad += [(fn.name, x) for x in stored & called & module_funcs]
    assert not bad, bad


def test_serve_run_validation():
    """aes_serve_run checks every request and parameter before it sets
    anything up (no GPU is touched for these cases)."""
    f = L.aes_serve_run
    dt = am.serve_request_dtype()
    reqs = np.zeros(3, dtype=dt)
    reqs["arrival_s"] = [0.0, 1e-6, 2e-6]
    reqs["in_off"] = [0, 16, 4096]
    reqs["nbytes"] = [5, 100, 4096]
    reqs["key_id"] = [0, 1, 0]
    keys32 = np.zeros((2, 32), np.uint8)
    klen = np.array([16, 32], np.uint8)
    lat = np.zeros(3, np.float64)
    off = np.zeros(3, np.uint64)
    pool, pool_bytes = VP(0x100000), 1 << 20
    out, out_bytes = VP(0x400000), 1 << 20
    prm = am.ServeParams(16, 2, 1024, 1, 1 << 30, 1 << 26, 50e-6)

    def call(r=reqs, k=klen, p=pool, pb=pool_bytes, o=out, ob=out_bytes, pr=prm, n=None):
        return f(r.ctypes.data, len(r) if n is None else n, keys32.ctypes.data, k.ctypes.data,
                 len(k), p, pb, o, ob, ctypes.byref(pr), lat.ctypes.data, off.ctypes.data, None)
    assert call(n=0) == 0
    assert f(None, 3, keys32.ctypes.data, klen.ctypes.data, 2, pool, pool_bytes, out,
             out_bytes, ctypes.byref(prm), lat.ctypes.data, off.ctypes.data, None) == -1
    for bad in (am.ServeParams(0, 2, 1024, 1, 1 << 30, 1 << 26, 50e-6),
                am.ServeParams(16, 9, 1024, 1, 1 << 30, 1 << 26, 50e-6),
                am.ServeParams(16, 2, 0, 1, 1 << 30, 1 << 26, 50e-6),
                am.ServeParams(16, 2, 1024, 1, 0, 1 << 26, 50e-6),
                am.ServeParams(16, 2, 1024, 1, 1 << 30, 1 << 26, -1.0)):
        assert call(pr=bad) == -9
    assert call(k=np.array([16, 20], np.uint8)) == -2
    assert call(p=VP(0x100008)) == -4
    assert call(o=VP(0x100000 + 4096)) == -5                 # output inside the pool
    cases = [("in_off", 1, 8, -4), ("in_off", 2, pool_bytes - 16, -7),
             ("key_id", 1, 2, -7), ("nbytes", 0, 0, -7), ("reserved", 2, 1, -7),
             ("arrival_s", 2, 0.0, -7)]
    for field, i, value, code in cases:
        r = reqs.copy()
        r[field][i] = value
        assert call(r=r) == code, (field, value)
    r = reqs.copy()
    r["ctr0"][2] = 2 ** 32 - 10                             # 256 blocks from 2^32 - 10
    assert call(r=r) == -7
    # the output area is a ring: any size from 16 bytes up is accepted (a
    # request whose output is larger than the whole area is rejected in the run)
    assert call(ob=15) == -9


def test_bench_trace_summary(tmp_path):
    """bench.py --trace-summary: per kernel, the last N dispatches of the
    rocprofv3 kernel trace (the timed steps of a bench run come last)."""
    import json
    import subprocess
    import sys
    d = tmp_path / "prof" / "host"
    d.mkdir(parents=True)
    rows = ["Kind,Kernel_Name,Start_Timestamp,End_Timestamp"]
    for i, ns in enumerate([9_000_000, 5_000_000, 2_000_000, 2_500_000, 3_000_000]):
        rows.append("KERNEL_DISPATCH,ctr_grouped_kernel,%d,%d" % (10**9 * (i + 1), 10**9 * (i + 1) + ns))
    rows.append("KERNEL_DISPATCH,other,5,10")
    (d / "run_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--trace-summary",
                          str(tmp_path / "prof"), "--last", "3"], capture_output=True, text=True,
                         check=True).stdout
    s = json.loads(out)
    assert s["ctr_grouped_kernel"] == {"calls": 5, "last": 3, "avg_ms": 2.5, "min_ms": 2.0,
                                       "max_ms": 3.0}
    assert s["other"]["calls"] == 1
    # split into runs at idle gaps longer than 500 ms: the dispatches are 1 s
    # apart and the first ("other", at 5 ns) is 1 s before the next
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--trace-summary",
                          str(tmp_path / "prof"), "--last", "3", "--split-gap-ms", "500"],
                         capture_output=True, text=True, check=True).stdout
    runs = json.loads(out)["runs"]
    assert len(runs) == 6 and runs[0]["kernels"]["other"]["calls"] == 1
    assert runs[1]["kernels"]["ctr_grouped_kernel"]["avg_ms"] == 9.0

"""Python binding of libaesmi (ctypes).

Argument marshalling only: every step of the cipher runs in the library's HIP
kernels.  PyTorch supplies device memory (uint8 CUDA tensors) and the current
HIP stream.  If ``libaesmi.so`` is missing the first call raises: there is no
fallback path.

The C entry points keep their names: ``aes_expand_key`` is ``expand_key``,
``aes_ctr_xcrypt`` is ``ctr_xcrypt`` and so on.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaesmi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "aesmi.h")

AES_OK = 0
STATUS = {0: "AES_OK", -1: "AES_ERR_NULL", -2: "AES_ERR_KEYLEN", -3: "AES_ERR_LENGTH",
          -4: "AES_ERR_ALIGN", -5: "AES_ERR_OVERLAP", -6: "AES_ERR_COUNTER",
          -7: "AES_ERR_SEGMENT", -8: "AES_ERR_HIP", -9: "AES_ERR_CONFIG",
          -10: "AES_ERR_DEVICE"}
LAYOUT_AUTO, LAYOUT_TTABLE, LAYOUT_BITSLICE = 0, 1, 2
SCHEDULE_BYTES = 488
SEGMENT_BYTES = 48


class AesError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        name = STATUS.get(status, str(status))
        text = _lib.aes_status_string(status).decode() if _lib is not None else name
        super().__init__("%s%s: %s" % (what + ": " if what else "", name, text))


class KeySchedule(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_uint32), ("key_bytes", ctypes.c_uint32),
                ("rk_enc", ctypes.c_uint32 * 60), ("rk_dec", ctypes.c_uint32 * 60)]

    def to_bytes(self) -> bytes:
        return ctypes.string_at(ctypes.addressof(self), ctypes.sizeof(self))


class Launch(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_uint32), ("wg_size", ctypes.c_uint32),
                ("grid_per_cu", ctypes.c_uint32), ("blocks_per_lane", ctypes.c_uint32),
                ("ctr_precompute", ctypes.c_uint32)]


class Segment(ctypes.Structure):
    _fields_ = [("in_off", ctypes.c_uint64), ("out_off", ctypes.c_uint64),
                ("nbytes", ctypes.c_uint64), ("key_slot", ctypes.c_uint32),
                ("ctr0", ctypes.c_uint32), ("nonce", ctypes.c_uint8 * 12),
                ("reserved", ctypes.c_uint32)]


class BatchTune(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_uint32), ("wg_size", ctypes.c_uint32),
                ("grid_per_cu", ctypes.c_uint32), ("tile_blocks", ctypes.c_uint32),
                ("blocks_per_lane", ctypes.c_uint32)]


# void (*)(void *user, uint64_t first, uint64_t count)
SERVE_BATCH_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)


class ServeParams(ctypes.Structure):
    _fields_ = [("nslots", ctypes.c_uint32), ("nstreams", ctypes.c_uint32),
                ("max_batch_reqs", ctypes.c_uint32), ("realtime", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64),
                ("window_s", ctypes.c_double), ("on_batch", SERVE_BATCH_FN),
                ("user", ctypes.c_void_p)]


class ServeStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("key_hits", ctypes.c_uint64), ("key_misses", ctypes.c_uint64),
                ("max_held", ctypes.c_uint64), ("max_out_used", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("elapsed_s", ctypes.c_double)]


SERVE_REQUEST_BYTES = 48


def serve_request_dtype():
    """numpy dtype with the byte layout of aes_serve_request_t (48 bytes)."""
    import numpy as np
    dt = np.dtype([("arrival_s", "<f8"), ("in_off", "<u8"), ("nbytes", "<u8"),
                   ("key_id", "<u4"), ("ctr0", "<u4"), ("nonce", "u1", (12,)),
                   ("reserved", "<u4")])
    assert dt.itemsize == SERVE_REQUEST_BYTES
    return dt


assert ctypes.sizeof(ServeParams) == 56 and ctypes.sizeof(ServeStats) == 80
assert ctypes.sizeof(KeySchedule) == SCHEDULE_BYTES
assert ctypes.sizeof(Segment) == SEGMENT_BYTES

_lib = None


def header_functions(path: str = HEADER) -> list[str]:
    """Names of every function the C header declares."""
    with open(path) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    return sorted(set(re.findall(r"\b(aes_\w+)\s*\(", text)))


def lib():
    """The loaded libaesmi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libaesmi.so is not built (python -m paper_1506_08503_amd.build); "
                               "there is no fallback implementation")
        l = ctypes.CDLL(LIB_PATH)
        vp, sz, u32, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int32
        st = ctypes.c_int
        sig = {
            "aes_expand_key": ([vp, sz, ctypes.POINTER(KeySchedule)], st),
            "aes_expand_keys_device": ([vp, sz, sz, vp, vp], st),
            "aes_ecb_encrypt": ([vp, vp, vp, sz, vp], st),
            "aes_ecb_decrypt": ([vp, vp, vp, sz, vp], st),
            "aes_ecb_encrypt_ex": ([vp, vp, vp, sz, ctypes.POINTER(Launch), vp], st),
            "aes_ecb_decrypt_ex": ([vp, vp, vp, sz, ctypes.POINTER(Launch), vp], st),
            "aes_ctr_xcrypt": ([vp, vp, u32, vp, vp, sz, vp], st),
            "aes_ctr_xcrypt_ex": ([vp, vp, u32, vp, vp, sz, ctypes.POINTER(Launch), vp], st),
            "aes_cbc_encrypt": ([vp, vp, sz, vp, vp, sz, sz, vp], st),
            "aes_cbc_decrypt": ([vp, vp, sz, vp, vp, sz, sz, vp], st),
            "aes_gcm_workspace_bytes": ([sz, sz], sz),
            "aes_gcm_encrypt": ([vp, vp, vp, sz, vp, vp, sz, vp, vp, sz, vp], st),
            "aes_gcm_decrypt": ([vp, vp, vp, sz, vp, vp, sz, vp, vp, sz, vp], st),
            "aes_ghash_workspace_bytes": ([sz], sz),
            "aes_ghash": ([vp, vp, sz, vp, vp, sz, vp], st),
            "aes_batched_workspace_bytes": ([u32], sz),
            "aes_ctr_xcrypt_batched": ([vp, u32, vp, u32, vp, vp, ctypes.POINTER(BatchTune),
                                        vp, sz, vp], st),
            "aes_batched_read_status": ([vp, vp, ctypes.POINTER(i32)], st),
            "aes_ctr_xcrypt_batched_noalloc": ([vp, u32, vp, u32, vp, vp,
                                                ctypes.POINTER(BatchTune), vp, vp], st),
            "aes_batched_graph_create": ([vp, u32, vp, u32, vp, vp, ctypes.POINTER(BatchTune),
                                          vp, sz, vp, ctypes.POINTER(vp)], st),
            "aes_batched_graph_launch": ([vp, vp], st),
            "aes_batched_graph_destroy": ([vp], st),
            "aes_serve_run": ([vp, sz, vp, vp, sz, vp, sz, vp, sz, ctypes.POINTER(ServeParams),
                               vp, vp, ctypes.POINTER(ServeStats)], st),
            "aes_server_create": ([vp, vp, sz, ctypes.POINTER(ServeParams), ctypes.POINTER(vp)],
                                  st),
            "aes_server_run": ([vp, vp, sz, vp, sz, vp, sz, vp, vp, ctypes.POINTER(ServeStats)],
                               st),
            "aes_server_destroy": ([vp], st),
            "aes_status_string": ([st], ctypes.c_char_p),
            "aes_version": ([], ctypes.c_char_p),
            "aes_device_cu_count": ([], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def _check(status: int, what: str):
    if status != AES_OK:
        raise AesError(status, what)


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev_u8(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError("%s must be a uint8 CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------- key schedule
def expand_key(key: bytes) -> KeySchedule:
    """aes_expand_key: host key expansion (16, 24 or 32-byte key)."""
    key = bytes(key)
    ks = KeySchedule()
    buf = ctypes.create_string_buffer(key, len(key))
    _check(lib().aes_expand_key(buf, len(key), ctypes.byref(ks)), "aes_expand_key")
    return ks


def schedule_to_device(ks: KeySchedule, device="cuda") -> torch.Tensor:
    """Copy a host schedule into a 488-byte device tensor."""
    host = torch.frombuffer(bytearray(ks.to_bytes()), dtype=torch.uint8)
    return host.to(device)


def key_schedule(key: bytes, device="cuda") -> torch.Tensor:
    return schedule_to_device(expand_key(key), device)


def expand_keys_device(keys: torch.Tensor) -> torch.Tensor:
    """aes_expand_keys_device: keys is an (n, key_bytes) uint8 CUDA tensor;
    returns an (n, 488) uint8 CUDA tensor of schedules."""
    _dev_u8(keys, "keys")
    if keys.dim() != 2:
        raise ValueError("keys must be (n, key_bytes)")
    n, kb = keys.shape
    out = torch.empty((n, SCHEDULE_BYTES), dtype=torch.uint8, device=keys.device)
    with torch.cuda.device(keys.device):
        _check(lib().aes_expand_keys_device(_ptr(keys), kb, n, _ptr(out), _stream(keys)),
               "aes_expand_keys_device")
    return out


def _launch(layout=None, wg_size=0, grid_per_cu=0, blocks_per_lane=0, ctr_precompute=0):
    if layout is None and not (wg_size or grid_per_cu or blocks_per_lane or ctr_precompute):
        return None
    return Launch(layout or 0, wg_size, grid_per_cu, blocks_per_lane, ctr_precompute)


def _ks_arg(ks: torch.Tensor):
    _dev_u8(ks, "key schedule")
    if ks.numel() != SCHEDULE_BYTES:
        raise ValueError("key schedule tensor must hold exactly one 488-byte schedule")
    return _ptr(ks)


def _out_like(x, out):
    if out is None:
        out = torch.empty_like(x)
    _dev_u8(out, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many bytes as the input")
    return out


# ---------------------------------------------------------------------- ECB
def _ecb(fname, ks, x, out, launch):
    _dev_u8(x, "input")
    out = _out_like(x, out)
    l = lib()
    with torch.cuda.device(x.device):
        if launch is None:
            st = getattr(l, fname)(_ks_arg(ks), _ptr(x), _ptr(out), x.numel(), _stream(x))
        else:
            st = getattr(l, fname + "_ex")(_ks_arg(ks), _ptr(x), _ptr(out), x.numel(),
                                           ctypes.byref(launch), _stream(x))
    _check(st, fname)
    return out


def ecb_encrypt(ks: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None,
                **launch) -> torch.Tensor:
    """aes_ecb_encrypt: every 16-byte block of x enciphered independently."""
    return _ecb("aes_ecb_encrypt", ks, x, out, _launch(**launch))


def ecb_decrypt(ks: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None,
                **launch) -> torch.Tensor:
    """aes_ecb_decrypt: every 16-byte block of x deciphered independently."""
    return _ecb("aes_ecb_decrypt", ks, x, out, _launch(**launch))


# ---------------------------------------------------------------------- CTR
def ctr_xcrypt(ks: torch.Tensor, nonce: bytes, ctr0: int, x: torch.Tensor,
               out: torch.Tensor | None = None, **launch) -> torch.Tensor:
    """aes_ctr_xcrypt: out = x XOR E(nonce || BE32(ctr0 + i)) block by block."""
    _dev_u8(x, "input")
    nonce = bytes(nonce)
    if len(nonce) != 12:
        raise ValueError("nonce must be 12 bytes")
    out = _out_like(x, out)
    nb = ctypes.create_string_buffer(nonce, 12)
    lc = _launch(**launch)
    l = lib()
    with torch.cuda.device(x.device):
        if lc is None:
            st = l.aes_ctr_xcrypt(_ks_arg(ks), nb, ctr0, _ptr(x), _ptr(out), x.numel(),
                                  _stream(x))
        else:
            st = l.aes_ctr_xcrypt_ex(_ks_arg(ks), nb, ctr0, _ptr(x), _ptr(out), x.numel(),
                                     ctypes.byref(lc), _stream(x))
    _check(st, "aes_ctr_xcrypt")
    return out


# ---------------------------------------------------------------------- CBC
def _cbc(fname, ks, iv, x, nmsg, out):
    _dev_u8(x, "input")
    _dev_u8(iv, "iv")
    if x.numel() % max(nmsg, 1):
        raise ValueError("input must hold nmsg rows of equal length")
    msg_bytes = x.numel() // nmsg if nmsg else 0
    if iv.numel() == 16:
        stride = 0
    elif iv.numel() == 16 * nmsg:
        stride = 16
    else:
        raise ValueError("iv must be 16 bytes or 16 bytes per row")
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        st = getattr(lib(), fname)(_ks_arg(ks), _ptr(iv), stride, _ptr(x), _ptr(out), nmsg,
                                   msg_bytes, _stream(x))
    _check(st, fname)
    return out


def cbc_encrypt(ks: torch.Tensor, iv: torch.Tensor, x: torch.Tensor, nmsg: int = 1,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """aes_cbc_encrypt: x holds nmsg rows of equal, 16-byte multiple length;
    iv is one 16-byte IV or one per row."""
    return _cbc("aes_cbc_encrypt", ks, iv, x, nmsg, out)


def cbc_decrypt(ks: torch.Tensor, iv: torch.Tensor, x: torch.Tensor, nmsg: int = 1,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """aes_cbc_decrypt (out of place)."""
    return _cbc("aes_cbc_decrypt", ks, iv, x, nmsg, out)


# ---------------------------------------------------------------------- GCM
def gcm_workspace_bytes(aad_len: int, nbytes: int) -> int:
    return int(lib().aes_gcm_workspace_bytes(aad_len, nbytes))


def ghash_workspace_bytes(nblocks: int) -> int:
    return int(lib().aes_ghash_workspace_bytes(nblocks))


def _workspace(nbytes: int, device, ws):
    if ws is None:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    _dev_u8(ws, "workspace")
    if ws.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    return ws


def _small_out(t, device, name):
    if t is None:
        t = torch.empty(16, dtype=torch.uint8, device=device)
    _dev_u8(t, name)
    if t.numel() != 16:
        raise ValueError("%s must hold 16 bytes" % name)
    return t


def _gcm(fname, ks, iv, x, aad, out, tag, ws):
    _dev_u8(x, "input")
    iv = bytes(iv)
    if len(iv) != 12:
        raise ValueError("iv must be 12 bytes")
    if aad is None:
        aad = torch.empty(0, dtype=torch.uint8, device=x.device)
    elif not isinstance(aad, torch.Tensor):
        aad = torch.frombuffer(bytearray(bytes(aad)), dtype=torch.uint8).to(x.device) \
            if len(aad) else torch.empty(0, dtype=torch.uint8, device=x.device)
    _dev_u8(aad, "aad")
    out = _out_like(x, out)
    tag = _small_out(tag, x.device, "tag")
    need = gcm_workspace_bytes(aad.numel(), x.numel())
    ws = _workspace(need, x.device, ws)
    ivb = ctypes.create_string_buffer(iv, 12)
    with torch.cuda.device(x.device):
        st = getattr(lib(), fname)(_ks_arg(ks), ivb, _ptr(aad) if aad.numel() else None,
                                   aad.numel(), _ptr(x), _ptr(out), x.numel(), _ptr(tag),
                                   _ptr(ws), ws.numel(), _stream(x))
    _check(st, fname)
    return out, tag


def gcm_encrypt(ks: torch.Tensor, iv: bytes, x: torch.Tensor, aad=None,
                out: torch.Tensor | None = None, tag: torch.Tensor | None = None,
                ws: torch.Tensor | None = None):
    """aes_gcm_encrypt: returns (ciphertext, 16-byte tag), both on the device.
    aad is a uint8 device tensor or bytes (copied to the device)."""
    return _gcm("aes_gcm_encrypt", ks, iv, x, aad, out, tag, ws)


def gcm_decrypt(ks: torch.Tensor, iv: bytes, x: torch.Tensor, aad=None,
                out: torch.Tensor | None = None, tag: torch.Tensor | None = None,
                ws: torch.Tensor | None = None):
    """aes_gcm_decrypt: returns (plaintext, tag computed over x).  The caller
    compares the tag with the received one before using the plaintext."""
    return _gcm("aes_gcm_decrypt", ks, iv, x, aad, out, tag, ws)


def ghash(h: bytes, x: torch.Tensor, y: torch.Tensor | None = None,
          ws: torch.Tensor | None = None) -> torch.Tensor:
    """aes_ghash: GHASH_H over the 16-byte blocks of x."""
    _dev_u8(x, "input")
    h = bytes(h)
    if len(h) != 16:
        raise ValueError("h must be 16 bytes")
    if x.numel() % 16:
        raise ValueError("input must be whole 16-byte blocks")
    nblocks = x.numel() // 16
    y = _small_out(y, x.device, "y")
    ws = _workspace(ghash_workspace_bytes(nblocks), x.device, ws)
    hb = ctypes.create_string_buffer(h, 16)
    with torch.cuda.device(x.device):
        st = lib().aes_ghash(hb, _ptr(x) if nblocks else None, nblocks, _ptr(y), _ptr(ws),
                             ws.numel(), _stream(x))
    _check(st, "aes_ghash")
    return y


# ------------------------------------------------------------------- batched
SEGMENT_DTYPE = None


def segment_dtype():
    """numpy dtype with the byte layout of aes_segment_t (48 bytes)."""
    import numpy as np
    global SEGMENT_DTYPE
    if SEGMENT_DTYPE is None:
        SEGMENT_DTYPE = np.dtype([("in_off", "<u8"), ("out_off", "<u8"), ("nbytes", "<u8"),
                                  ("key_slot", "<u4"), ("ctr0", "<u4"), ("nonce", "u1", (12,)),
                                  ("reserved", "<u4")])
        assert SEGMENT_DTYPE.itemsize == SEGMENT_BYTES
    return SEGMENT_DTYPE


def batched_workspace_bytes(nsegs: int) -> int:
    return int(lib().aes_batched_workspace_bytes(nsegs))


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, BatchTune):
        return tune
    return BatchTune(tune.get("layout", 0), tune.get("wg_size", 0), tune.get("grid_per_cu", 0),
                     tune.get("tile_blocks", 0), tune.get("blocks_per_lane", 0))


def ctr_xcrypt_batched(segs: torch.Tensor, ks_table: torch.Tensor, x: torch.Tensor,
                       out: torch.Tensor, ws: torch.Tensor, tune=None) -> torch.Tensor:
    """aes_ctr_xcrypt_batched: segs is a uint8 CUDA tensor holding nsegs
    aes_segment_t records, ks_table an (nkeys, 488) uint8 CUDA tensor, x / out
    the packed input / output buffers, ws a workspace of
    batched_workspace_bytes(nsegs) bytes (256-byte aligned)."""
    for t, n in ((segs, "segments"), (ks_table, "key table"), (x, "input"), (out, "output"),
                 (ws, "workspace")):
        _dev_u8(t, n)
    if segs.numel() % SEGMENT_BYTES or ks_table.numel() % SCHEDULE_BYTES:
        raise ValueError("segment / key table sizes must be whole records")
    nsegs = segs.numel() // SEGMENT_BYTES
    nkeys = ks_table.numel() // SCHEDULE_BYTES
    tn = _tune(tune)
    with torch.cuda.device(x.device):
        st = lib().aes_ctr_xcrypt_batched(_ptr(segs), nsegs, _ptr(ks_table), nkeys, _ptr(x),
                                          _ptr(out), ctypes.byref(tn) if tn else None, _ptr(ws),
                                          ws.numel(), _stream(x))
    _check(st, "aes_ctr_xcrypt_batched")
    return out


NOALLOC_MAX_SEGS = 65536


def ctr_xcrypt_batched_noalloc(segs: torch.Tensor, ks_table: torch.Tensor, x: torch.Tensor,
                               out: torch.Tensor, tune=None,
                               status: torch.Tensor | None = None) -> torch.Tensor:
    """aes_ctr_xcrypt_batched_noalloc: the batched call on the library's static
    device workspace (at most NOALLOC_MAX_SEGS segments); `status`, an int32
    CUDA tensor of one element, receives the segment status word."""
    for t, n in ((segs, "segments"), (ks_table, "key table"), (x, "input"), (out, "output")):
        _dev_u8(t, n)
    if status is not None and (not status.is_cuda or status.dtype != torch.int32
                               or status.numel() < 1):
        raise ValueError("status must be an int32 CUDA tensor")
    if segs.numel() % SEGMENT_BYTES or ks_table.numel() % SCHEDULE_BYTES:
        raise ValueError("segment / key table sizes must be whole records")
    tn = _tune(tune)
    with torch.cuda.device(x.device):
        st = lib().aes_ctr_xcrypt_batched_noalloc(
            _ptr(segs), segs.numel() // SEGMENT_BYTES, _ptr(ks_table),
            ks_table.numel() // SCHEDULE_BYTES, _ptr(x), _ptr(out),
            ctypes.byref(tn) if tn else None,
            ctypes.c_void_p(status.data_ptr()) if status is not None else None, _stream(x))
    _check(st, "aes_ctr_xcrypt_batched_noalloc")
    return out


def batched_read_status(ws: torch.Tensor) -> int:
    """Device status word of the last batched call (0 or AES_ERR_SEGMENT)."""
    v = ctypes.c_int32(0)
    with torch.cuda.device(ws.device):
        _check(lib().aes_batched_read_status(_ptr(ws), _stream(ws), ctypes.byref(v)),
               "aes_batched_read_status")
    return int(v.value)


class BatchedGraph:
    """aes_batched_graph_create / _launch / _destroy: the batched call captured
    with fixed pointers; rewrite the tensors' contents in place between launches."""

    def __init__(self, segs, ks_table, x, out, ws, tune=None):
        for t, n in ((segs, "segments"), (ks_table, "key table"), (x, "input"),
                     (out, "output"), (ws, "workspace")):
            _dev_u8(t, n)
        self._keep = (segs, ks_table, x, out, ws)
        self.device = x.device
        tn = _tune(tune)
        h = ctypes.c_void_p()
        with torch.cuda.device(x.device):
            st = lib().aes_batched_graph_create(
                _ptr(segs), segs.numel() // SEGMENT_BYTES, _ptr(ks_table),
                ks_table.numel() // SCHEDULE_BYTES, _ptr(x), _ptr(out),
                ctypes.byref(tn) if tn else None, _ptr(ws), ws.numel(), _stream(x),
                ctypes.byref(h))
        _check(st, "aes_batched_graph_create")
        self._h = h

    def launch(self):
        with torch.cuda.device(self.device):
            _check(lib().aes_batched_graph_launch(self._h, _stream(self._keep[2])),
                   "aes_batched_graph_launch")

    def close(self):
        if self._h:
            _check(lib().aes_batched_graph_destroy(self._h), "aes_batched_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_cu_count() -> int:
    return int(lib().aes_device_cu_count())

"""The Python binding's record layouts equal the C header's: a small C
program compiled against include/aesmi.h prints sizeof and offsetof of every
struct the binding mirrors (ctypes structures and numpy dtypes), and each
must match."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1506_08503_amd as am
from paper_1506_08503_amd import aesmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C type name -> (ctypes structure) for the structures the binding passes by pointer
CTYPES = {
    "aes_key_schedule_t": aesmi.KeySchedule,
    "aes_launch_t": aesmi.Launch,
    "aes_segment_t": aesmi.Segment,
    "aes_batch_tune_t": aesmi.BatchTune,
    "aes_serve_params_t": aesmi.ServeParams,
    "aes_serve_stats_t": aesmi.ServeStats,
}
# C type name -> numpy dtype of host tables handed over as raw bytes
DTYPES = {
    "aes_segment_t": aesmi.segment_dtype,
    "aes_serve_request_t": aesmi.serve_request_dtype,
}


def _c_layout(tmp_path):
    fields = {}
    for name, st in CTYPES.items():
        fields.setdefault(name, set()).update(f[0] for f in st._fields_)
    for name, fn in DTYPES.items():
        fields.setdefault(name, set()).update(fn().names)
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "aesmi.h"', "int main(void) {"]
    for name, fs in sorted(fields.items()):
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in sorted(fs):
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        t, f, v = line.split()
        got[(t, f)] = int(v)
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_binding_layouts_match_header(tmp_path):
    c = _c_layout(tmp_path)
    for name, st in CTYPES.items():
        assert ctypes.sizeof(st) == c[(name, "size")], name
        for f in st._fields_:
            assert getattr(st, f[0]).offset == c[(name, f[0])], (name, f[0])
    for name, fn in DTYPES.items():
        dt = fn()
        assert dt.itemsize == c[(name, "size")], name
        for f in dt.names:
            assert dt.fields[f][1] == c[(name, f)], (name, f)
    assert c[("aes_segment_t", "size")] == am.aesmi.SEGMENT_BYTES == 48
    assert c[("aes_serve_request_t", "size")] == aesmi.SERVE_REQUEST_BYTES == 48
    assert c[("aes_key_schedule_t", "size")] == am.aesmi.SCHEDULE_BYTES == 488

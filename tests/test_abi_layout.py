"""The ctypes mirrors of the C-ABI structs match the header, field by field.

A small C program, compiled here with the host C compiler against
include/hashwave.h, prints each struct's size and every field's offset; the
binding's ctypes.Structure must agree on both (a field added to the header
but not to the binding, or in another order, shifts everything after it).
Host-only: nothing is loaded from the GPU library."""
import os
import shutil
import subprocess
import tempfile

import pytest

import paper_2509_16407_amd as hw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("hwave_config", hw._Config), ("hwave_item", hw._Item), ("hwave_tune_result", hw._Tune),
         ("hwave_probe_stats", hw._Probe), ("hwave_request", hw._Request),
         ("hwave_server_config", hw._ServerCfg), ("hwave_serve_stats", hw._ServeStats),
         ("hwave_raw_view", hw._Raw)]


@pytest.fixture(scope="module")
def c_layout():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hashwave.h"', "int main(void) {"]
    for cname, py in PAIRS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("  return 0;\n}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines) + "\n")
        r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.splitlines():
        a, b, v = line.split()
        res[(a, b)] = int(v)
    return res


@pytest.mark.parametrize("cname,py", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_struct_matches_header(c_layout, cname, py):
    import ctypes
    assert ctypes.sizeof(py) == c_layout[(cname, "size")]
    for f, _ in py._fields_:
        assert getattr(py, f).offset == c_layout[(cname, f)], (cname, f)

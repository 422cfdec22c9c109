"""Builds libhashwave.so for gfx950 in-tree: each source compiled by hipcc in
parallel, then linked into one shared library next to this file.  Also builds
libhashwave_instr.so, the same sources with -DHW_INSTRUMENT (query probe
counters, hwave_probe_counters), used by tests that count lines per query."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhashwave.so")
OUT_INSTR = os.path.join(HERE, "libhashwave_instr.so")
OBJ = os.path.join(HERE, "_build")
OBJ_INSTR = os.path.join(HERE, "_build_instr")

SOURCES = ["capi.hip", "inst_u64_double.hip", "inst_u64_p2.hip", "inst_u64_iceberg.hip", "inst_u64_chain.hip", "inst_u64_cuckoo.hip", "inst_u32_double.hip",
           "inst_u32_p2.hip", "inst_u32_iceberg.hip", "inst_u64_bsp.hip", "inst_multi.hip", "inst_multi_solo.hip", "autotune.hip",
           "server.hip"]
HEADERS = ["hw_device.hpp", "hw_ops.hpp", "hw_launch.hpp", "hw_multi.hpp"]

ARCH = os.environ.get("HWAVE_ARCH", "gfx950")
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(src: str, extra, obj_dir: str = OBJ) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(extra_flags=(), out: str = OUT, jobs: int | None = None, instrumented: bool = True) -> str:
    """Compiles every source (always) and links `out`; with `instrumented`, also
    the instrumented library.  Returns the path of `out`."""
    if instrumented:
        _link(list(extra_flags) + ["-DHW_INSTRUMENT"], OUT_INSTR, OBJ_INSTR, jobs)
    return _link(list(extra_flags), out, OBJ, jobs)


def _link(extra_flags, out: str, obj_dir: str, jobs) -> str:
    os.makedirs(obj_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra_flags), obj_dir), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-lpthread", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build(extra))

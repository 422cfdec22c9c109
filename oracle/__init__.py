"""HashWave CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package.  The GPU library (`paper_2509_16407_amd`) never imports
it and shares no code with it; the two meet only through the seeded input
generators in `paper_2509_16407_amd.workloads`, which hold no table arithmetic.

Contents:
  * `OracleMap`  -- the plain map the paper's API defines (Section 5.1), batches
    applied one operation at a time in input order (Section 4.1's serialisability);
  * `layout_check` -- design invariants and probe counts of a raw table image;
  * `sim_insert` -- sequential placement simulator (Section 2.2 placement rules);
  * `brute` -- a pure-Python linear-scan twin of `OracleMap` for tiny inputs.

Parity status per function (see the test files for the pins):
  OracleMap        pinned: brute-force twin, closed forms (v = 3k+1, absent keys
                   miss), sum invariants, sentinel/capacity special cases.
  layout_check     pinned: hand-built images with planted violations; probe model
                   pinned through sim_insert against Table 1 and against the
                   uniform-probing closed form.
  sim_insert       pinned: Table 1 load probes (double hashing 1.22 / 2.05, power of
                   two choice 2.83 / 2.13, iceberg 2.97 / 2.16) and Knuth's
                   uniform-probing formulas; iceberg placement also pinned by its
                   front-yard-first invariant on brute-force small images.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hw_oracle.cpp")
LIB = os.path.join(HERE, "libhw_oracle.so")

QUERY, INSERT, UPSERT, ERASE = 0, 1, 2, 3
SUM, KEEP, REPLACE, MIN, MAX = 0, 1, 2, 3, 4
MISS, DONE, EXISTED, FULL, INVALID = 0, 1, 2, 3, 4
DOUBLE, DOUBLE_M, P2, P2_M, ICEBERG, ICEBERG_M, CHAINING, CUCKOO = 0, 1, 2, 3, 4, 5, 6, 7


def build(force: bool = False, extra_flags=(), out: str | None = None) -> str:
    """Compile the oracle with the host C++ compiler; returns the library path."""
    out = out or LIB
    if force or out != LIB or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", *extra_flags, SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class _Report(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "live", "tombs", "empties", "reserved", "duplicate_keys", "misplaced",
        "tag_mismatch", "locks_held", "in_alternate")] + [
        ("pos_probe_sum", ctypes.c_double), ("neg_probe_sum", ctypes.c_double),
        ("neg_count", ctypes.c_uint64), ("max_seq_index", ctypes.c_uint64),
        ("front_room", ctypes.c_uint64)]


_lib = None


def load(path: str | None = None):
    """The oracle library.  HW_ORACLE_LIB names an alternative build (used only by
    the mutation test, which plants known mistakes in copies of the oracle)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        alt = os.environ.get("HW_ORACLE_LIB")
        _lib = _bind(ctypes.CDLL(alt if alt else build()))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    U64 = ctypes.c_uint64
    lib.orc_map_new.restype = P
    lib.orc_map_new.argtypes = [ctypes.c_int, U64]
    lib.orc_map_free.argtypes = [P]
    lib.orc_map_size.restype = U64
    lib.orc_map_size.argtypes = [P]
    lib.orc_map_apply.restype = ctypes.c_int
    lib.orc_map_apply.argtypes = [P, U64, P, ctypes.c_int, P, P, ctypes.c_int, P, P]
    lib.orc_map_dump.argtypes = [P, P, P]
    lib.orc_map_digest.argtypes = [P, P, P]
    lib.orc_tag.restype = ctypes.c_uint16
    lib.orc_tag.argtypes = [U64]
    for f in ("orc_primary_bucket", "orc_p2_alternate"):
        getattr(lib, f).restype = U64
        getattr(lib, f).argtypes = [U64, U64]
    lib.orc_double_probe.restype = U64
    lib.orc_double_probe.argtypes = [U64, U64, U64]
    lib.orc_iceberg_front_buckets.restype = U64
    lib.orc_iceberg_front_buckets.argtypes = [U64]
    lib.orc_iceberg_buckets.argtypes = [U64, U64, ctypes.POINTER(U64)]
    lib.orc_layout_check.restype = U64
    lib.orc_layout_check.argtypes = [ctypes.c_int, ctypes.c_int, U64, U64, P, P, P, U64, P, U64,
                                     U64, ctypes.POINTER(_Report)]
    lib.orc_image_pairs.restype = U64
    lib.orc_image_pairs.argtypes = [ctypes.c_int, U64, P, P, P]
    lib.orc_sim_insert.restype = U64
    lib.orc_sim_insert.argtypes = [ctypes.c_int, ctypes.c_int, U64, U64, P, P, P, P, U64,
                                   ctypes.c_int, ctypes.c_int, P]
    lib.orc_chain_bucket.restype = U64
    lib.orc_chain_bucket.argtypes = [U64, U64]
    lib.orc_chain_check.restype = U64
    lib.orc_chain_check.argtypes = [U64, U64, P, P, U64, P, U64, ctypes.POINTER(_Report)]
    lib.orc_sim_chain_insert.restype = U64
    lib.orc_sim_chain_insert.argtypes = [U64, U64, P, P, U64, ctypes.c_int]
    lib.orc_cuckoo_buckets.argtypes = [U64, U64, ctypes.POINTER(U64)]
    lib.orc_sim_cuckoo_insert.restype = U64
    lib.orc_sim_cuckoo_insert.argtypes = [U64, U64, P, P, U64, U64, U64, ctypes.c_int]
    lib.orc_sim_aging.restype = ctypes.c_int
    lib.orc_sim_aging.argtypes = [ctypes.c_int, U64, U64, U64, U64, P, U64, U64, U64, P, P, U64, P]
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint64)


class OracleMap:
    """The semantic map: a batch is applied one operation at a time in input order."""

    def __init__(self, key_bits: int = 64, capacity: int = 0, lib=None):
        self.lib = lib or load()
        self.key_bits = key_bits
        self.h = self.lib.orc_map_new(key_bits, capacity)
        if not self.h:
            raise ValueError("bad key width")

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_map_free(self.h)
            self.h = None

    def apply(self, keys, vals=None, ops=None, default_op=QUERY, combine=SUM):
        keys = _u64(keys)
        n = len(keys)
        vals = _u64(vals)
        ops = None if ops is None else np.ascontiguousarray(ops, dtype=np.uint8)
        status = np.zeros(n, dtype=np.uint8)
        out = np.zeros(n, dtype=np.uint64)
        rc = self.lib.orc_map_apply(self.h, n, _ptr(ops), default_op, _ptr(keys), _ptr(vals),
                                    combine, _ptr(status), _ptr(out))
        if rc != 0:
            raise ValueError("oracle apply failed")
        return status, out

    def insert(self, keys, vals):
        return self.apply(keys, vals, default_op=INSERT)[0]

    def upsert(self, keys, vals, combine=SUM):
        return self.apply(keys, vals, default_op=UPSERT, combine=combine)[0]

    def query(self, keys):
        st, out = self.apply(keys, default_op=QUERY)
        return st, out

    def erase(self, keys):
        return self.apply(keys, default_op=ERASE)[0]

    def size(self) -> int:
        return int(self.lib.orc_map_size(self.h))

    def dump(self):
        n = self.size()
        k = np.zeros(n, dtype=np.uint64)
        v = np.zeros(n, dtype=np.uint64)
        if n:
            self.lib.orc_map_dump(self.h, _ptr(k), _ptr(v))
        return k, v

    def digest(self):
        s = ctypes.c_uint64()
        x = ctypes.c_uint64()
        self.lib.orc_map_digest(self.h, ctypes.byref(s), ctypes.byref(x))
        return s.value, x.value


def layout_check(design, key_bits, nb, bucket_slots, slots, tags=None, locks=None,
                 neg_keys=None, tile_bytes=128, lib=None):
    """Invariant violations and probe statistics of a raw table image (numpy arrays).

    `slots` is the raw slot array (any dtype, bucket-major, 16 B or 8 B per slot).
    Returns (violations, report dict)."""
    lib = lib or load()
    rep = _Report()
    slots = np.ascontiguousarray(slots)
    tags = None if tags is None else np.ascontiguousarray(tags, dtype=np.uint16)
    locks = None if locks is None else np.ascontiguousarray(locks, dtype=np.uint64)
    neg = _u64(neg_keys)
    nv = lib.orc_layout_check(design, key_bits, nb, bucket_slots, _ptr(slots), _ptr(tags),
                              _ptr(locks), 0 if locks is None else len(locks), _ptr(neg),
                              0 if neg is None else len(neg), tile_bytes, ctypes.byref(rep))
    d = {name: getattr(rep, name) for name, _ in _Report._fields_}
    return int(nv), d


def image_pairs(key_bits, slots):
    lib = load()
    slots = np.ascontiguousarray(slots)
    nslots = slots.nbytes // (16 if key_bits == 64 else 8)
    k = np.zeros(nslots, dtype=np.uint64)
    v = np.zeros(nslots, dtype=np.uint64)
    c = lib.orc_image_pairs(key_bits, nslots, _ptr(slots), _ptr(k), _ptr(v))
    return k[:c], v[:c]


def sim_insert(design, key_bits, nb, bucket_slots, keys, vals=None, shortcut=True,
               slots=None, tags=None, visits=False):
    """Sequential placement of `keys` (Section 2.2 rules) into a fresh image.

    Returns (slots uint8 array, tags uint16 array or None, n_failed), and with
    visits=True also each insert's bucket visits (uint32 array)."""
    lib = load()
    sb = 16 if key_bits == 64 else 8
    init = slots is None
    if slots is None:
        slots = np.empty(nb * bucket_slots * sb, dtype=np.uint8)
        if design in (DOUBLE_M, P2_M, ICEBERG_M):
            tags = np.empty(nb * bucket_slots, dtype=np.uint16)
    keys = _u64(keys)
    vals = _u64(vals)
    vis = np.zeros(len(keys), dtype=np.uint32) if visits else None
    failed = lib.orc_sim_insert(design, key_bits, nb, bucket_slots, _ptr(slots), _ptr(tags),
                                _ptr(keys), _ptr(vals), len(keys), int(bool(shortcut)), int(init), _ptr(vis))
    if visits:
        return slots, tags, int(failed), vis
    return slots, tags, int(failed)


# Table 1's insert and delete columns, as accesses (reading 13): every access
# to a cache line counts, the lock's acquire and release included.
LOCK_ACCESSES = 2       # acquire and release of the primary bucket's lock
INSERT_WRITES = 2       # the claim (compare-and-swap) and the key-value publish


def insert_probes_tags(visits):
    """Mean insert probes of a tag design from its inserts' bucket visits: one tag
    line per visit, the lock's two accesses and the two writes of the placement."""
    return float(np.mean(visits)) + LOCK_ACCESSES + INSERT_WRITES


def delete_probes(design, query_probes):
    """Mean delete probes from the positive-query probes of the same keys: the
    search reads what a query reads, then the lock's two accesses and the
    removal's writes (the key; in the tag designs the tag too)."""
    writes = 2 if design in (DOUBLE_M, P2_M, ICEBERG_M) else 1
    return query_probes + LOCK_ACCESSES + writes


def tag_of(key: int) -> int:
    return int(load().orc_tag(key))


def primary_bucket(key: int, nb: int) -> int:
    return int(load().orc_primary_bucket(key, nb))


def double_probe(key: int, nb: int, i: int) -> int:
    return int(load().orc_double_probe(key, nb, i))


def p2_alternate(key: int, nb: int) -> int:
    return int(load().orc_p2_alternate(key, nb))


def iceberg_front_buckets(nb: int) -> int:
    return int(load().orc_iceberg_front_buckets(nb))


def iceberg_buckets(key: int, nb: int):
    """(front bucket, first backyard choice, second backyard choice)."""
    out = (ctypes.c_uint64 * 3)()
    load().orc_iceberg_buckets(key, nb, out)
    return int(out[0]), int(out[1]), int(out[2])


def sim_aging(design, nb, bucket_slots, plan, tile_bytes=128, probe_cap=0, from_iter=0):
    """Sequential aging run (Section 6.5) over `plan` (workloads.aging_plan):
    returns (mean positive probes, mean negative probes, failed inserts), probes
    counted from iteration `from_iter` on."""
    lib = load()
    keys = _u64(plan["keys"])
    negs = _u64(plan["negs"])
    ps = np.ascontiguousarray(plan["pos_start"], dtype=np.uint64)
    out = np.zeros(3, dtype=np.float64)
    rc = lib.orc_sim_aging(design, nb, bucket_slots, tile_bytes, probe_cap, _ptr(keys), plan["n0"], plan["s"],
                           plan["iters"], _ptr(ps), _ptr(negs), from_iter, _ptr(out))
    if rc != 0:
        raise ValueError("bad aging arguments")
    return float(out[0]), float(out[1]), int(out[2])


def chain_bucket(key: int, nb: int) -> int:
    return int(load().orc_chain_bucket(key, nb))


def chain_check(nb, nodes, locks=None, neg_keys=None, lib=None):
    """Invariants and probes of a chaining image: `nodes` is the raw node array
    (128 bytes per node, nb bucket nodes first).  Returns (violations, report)."""
    lib = lib or load()
    rep = _Report()
    nodes = np.ascontiguousarray(nodes).view(np.uint64)
    locks = None if locks is None else np.ascontiguousarray(locks, dtype=np.uint64)
    neg = _u64(neg_keys)
    nv = lib.orc_chain_check(nb, len(nodes) // 16, _ptr(nodes), _ptr(locks), 0 if locks is None else len(locks),
                             _ptr(neg), 0 if neg is None else len(neg), ctypes.byref(rep))
    return int(nv), {name: getattr(rep, name) for name, _ in _Report._fields_}


def sim_chain_insert(nb, n_nodes, keys, nodes=None):
    """Sequential chaining inserts (first empty slot along the chain, else a new
    tail node).  Returns (nodes uint64 array, n_failed)."""
    lib = load()
    init = nodes is None
    if nodes is None:
        nodes = np.empty(n_nodes * 16, dtype=np.uint64)
    keys = _u64(keys)
    failed = lib.orc_sim_chain_insert(nb, n_nodes, _ptr(nodes), _ptr(keys), len(keys), int(init))
    return nodes, int(failed)


def cuckoo_buckets(key: int, nb: int):
    """The three candidate buckets of a key in hash order (possibly repeated)."""
    out = (ctypes.c_uint64 * 3)()
    load().orc_cuckoo_buckets(key, nb, out)
    return int(out[0]), int(out[1]), int(out[2])


def sim_cuckoo_insert(nb, bucket_slots, keys, max_kicks=500, seed=1, slots=None):
    """Sequential three-way cuckoo inserts; returns (slots uint8 array, n_failed)."""
    lib = load()
    init = slots is None
    if slots is None:
        slots = np.empty(nb * bucket_slots * 16, dtype=np.uint8)
    keys = _u64(keys)
    failed = lib.orc_sim_cuckoo_insert(nb, bucket_slots, _ptr(slots), _ptr(keys), len(keys), max_kicks, seed,
                                       int(init))
    return slots, int(failed)

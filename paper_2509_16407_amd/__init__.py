"""HashWave: concurrent GPU hash tables for MI355X (gfx950).

Thin ctypes binding over `libhashwave.so` (C-ABI in include/hashwave.h).  It
only marshals arguments: every table operation runs in the library's HIP
kernels.  PyTorch provides device memory (tables are created inside a torch
uint8 buffer with `hwave_create_in`) and the current stream.  Keys and values
travel as int64 / int32 tensors holding the unsigned bit patterns.

There is no fallback: if the shared library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Table", "Multi", "Server", "lib", "autotune", "multi_upsert_tables", "DESIGNS", "COMBINES", "OPS",
           "HashWaveError"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhashwave.so")
LIB_INSTR_PATH = os.path.join(HERE, "libhashwave_instr.so")

DESIGNS = {"DOUBLE": 0, "DOUBLE_M": 1, "P2": 2, "P2_M": 3, "ICEBERG": 4, "ICEBERG_M": 5, "CHAINING": 6, "CUCKOO": 7}
COMBINES = {"sum": 0, "keep": 1, "replace": 2, "min": 3, "max": 4}
OPS = {"query": 0, "insert": 1, "upsert": 2, "erase": 3}
ST_MISS, ST_DONE, ST_EXISTED, ST_FULL, ST_INVALID, ST_TIMEOUT = 0, 1, 2, 3, 4, 5
F_NO_SHORTCUT = 1
F_NO_ERASE = 2
F_BSP = 4
F_AGGREGATE = 8
F_MERGE_MIXED = 16


class HashWaveError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [("kv_bits", ctypes.c_uint32), ("bucket_slots", ctypes.c_uint32),
                ("tile", ctypes.c_uint32), ("probe_cap", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("lock_timeout_us", ctypes.c_uint32)]


class _Item(ctypes.Structure):
    _fields_ = [("table", ctypes.c_uint32), ("op", ctypes.c_uint32), ("begin", ctypes.c_uint64),
                ("end", ctypes.c_uint64)]


class _Tune(ctypes.Structure):
    _fields_ = [("design", ctypes.c_uint32), ("bucket_slots", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("kv_bits", ctypes.c_uint32), ("gops", ctypes.c_double), ("full_ops", ctypes.c_uint64),
                ("load", ctypes.c_double), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _Probe(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("bucket_lines", ctypes.c_uint64), ("slot_lines", ctypes.c_uint64),
                ("writes", ctypes.c_uint64), ("write_visits", ctypes.c_uint64)]


class _Request(ctypes.Structure):
    _fields_ = [("table", ctypes.c_uint32), ("op", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("h_keys", ctypes.c_void_p), ("h_vals", ctypes.c_void_p), ("h_vals_out", ctypes.c_void_p),
                ("h_status", ctypes.c_void_p)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("slot_ops", ctypes.c_uint64),
                ("max_requests", ctypes.c_uint32), ("device", ctypes.c_int32)]


class _ServeStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("ops", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("mean_requests_per_batch", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("runtime_copied", ctypes.c_uint64)]


class _Raw(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_void_p), ("tags", ctypes.c_void_p), ("locks", ctypes.c_void_p),
                ("n_lock_words", ctypes.c_uint64), ("lock_queues", ctypes.c_void_p),
                ("n_lock_queues", ctypes.c_uint64), ("num_buckets", ctypes.c_uint64),
                ("bucket_slots", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("kv_bits", ctypes.c_uint32), ("design", ctypes.c_uint32), ("slot_bytes", ctypes.c_uint64),
                ("lock_stride", ctypes.c_uint32)]


_lib = None
_lib_instr = None


def lib(instrumented: bool = False):
    """The loaded C library (raises if it has not been built); `instrumented`:
    the build that keeps query probe counters (hwave_probe_counters)."""
    global _lib, _lib_instr
    path = LIB_INSTR_PATH if instrumented else LIB_PATH
    if (_lib_instr if instrumented else _lib) is None:
        if not os.path.exists(path):
            raise HashWaveError("%s is missing: build it with __graft_entry__.build() "
                                "(no CPU fallback exists)" % path)
        L = _bind(ctypes.CDLL(path))
        if instrumented:
            _lib_instr = L
        else:
            _lib = L
    return _lib_instr if instrumented else _lib


def _bind(L):
    P, U64, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    sig = {
        "hwave_config_default": (I, [I, ctypes.POINTER(_Config)]),
        "hwave_table_bytes": (I, [U64, I, ctypes.POINTER(_Config), ctypes.POINTER(U64)]),
        "hwave_create": (I, [ctypes.POINTER(P), U64, I, ctypes.POINTER(_Config), P]),
        "hwave_create_in": (I, [ctypes.POINTER(P), P, U64, U64, I, ctypes.POINTER(_Config), P]),
        "hwave_destroy": (I, [P]),
        "hwave_clear": (I, [P, P]),
        "hwave_insert": (I, [P, P, P, U64, P, P]),
        "hwave_upsert": (I, [P, P, P, U64, I, P, P]),
        "hwave_query": (I, [P, P, U64, P, P, P]),
        "hwave_erase": (I, [P, P, U64, P, P]),
        "hwave_mixed": (I, [P, P, P, P, U64, I, P, P, P]),
        "hwave_mixed_noalloc": (I, [P, P, P, P, U64, I, P, P, P]),
        "hwave_size": (I, [P, P, P]),
        "hwave_export": (I, [P, P, P, P, P]),
        "hwave_num_buckets": (U64, [P]),
        "hwave_capacity": (U64, [P]),
        "hwave_primary_bucket": (I, [P, P, U64, P, P]),
        "hwave_candidate_buckets": (I, [P, P, U64, P, P]),
        "hwave_raw": (I, [P, ctypes.POINTER(_Raw)]),
        "hwave_strerror": (ctypes.c_char_p, [I]),
        "hwave_last_hip_error": (I, []),
        "hwave_stream_sync": (I, [P]),
        "hwave_multi_supported": (I, [ctypes.c_uint32, I, ctypes.c_uint32, ctypes.c_uint32]),
        "hwave_multi_create": (I, [ctypes.POINTER(P), P, ctypes.c_uint32, P]),
        "hwave_multi_destroy": (I, [P]),
        "hwave_multi_kernel": (I, [P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
        "hwave_multi_run": (I, [P, P, ctypes.c_uint32, P, P, P, P, P]),
        "hwave_multi_clear": (I, [P, P]),
        "hwave_multi_upsert": (I, [P, P, P, P, I, P, P]),
        "hwave_multi_upsert_tables": (I, [P, ctypes.c_uint32, P, P, P, I, P, P]),
        "hwave_server_create": (I, [ctypes.POINTER(P), P, ctypes.c_uint32, ctypes.POINTER(_ServerCfg)]),
        "hwave_server_submit": (I, [P, ctypes.POINTER(_Request), ctypes.c_double, ctypes.POINTER(U64)]),
        "hwave_server_poll": (I, [P, U64, ctypes.POINTER(I)]),
        "hwave_server_drain": (I, [P]),
        "hwave_server_replay": (I, [P, P, P, U64, ctypes.POINTER(ctypes.c_double)]),
        "hwave_server_stats": (I, [P, ctypes.POINTER(_ServeStats)]),
        "hwave_server_destroy": (I, [P]),
        "hwave_now": (ctypes.c_double, []),
        "hwave_autotune": (I, [ctypes.c_uint32, U64, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32,
                               ctypes.c_uint32, ctypes.POINTER(_Tune), ctypes.c_uint32,
                               ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_Tune), P]),
        "hwave_probe_counters": (I, [P, ctypes.POINTER(_Probe), I, P]),
        "hwave_tune_save": (I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_Tune),
                                ctypes.c_uint32]),
        "hwave_tune_load": (I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_Tune),
                                ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _check(rc):
    if rc != 0:
        L = lib()
        raise HashWaveError("%s (code %d, hip error %d)" % (
            L.hwave_strerror(rc).decode(), rc, L.hwave_last_hip_error()))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Table:
    """One hash table in device memory.

    design: "DOUBLE" | "DOUBLE_M" | "P2" | "P2_M" | "ICEBERG" | "ICEBERG_M" | "CHAINING" | "CUCKOO"; kv_bits 64 or 32; bucket/tile 0 =
    the design default (Section 5 configurations).  Keys/values are int64 tensors
    (kv_bits=64) or int32 tensors (kv_bits=32) on the table's device.
    """

    def __init__(self, capacity: int, design: str = "P2_M", kv_bits: int = 64, bucket: int = 0,
                 tile: int = 0, probe_cap: int = 0, flags: int = 0, device=None, stream=None,
                 instrumented: bool = False, lock_timeout_us: int = 0):
        import torch
        L = lib(instrumented)
        self._L = L
        self.design = design
        self.design_id = DESIGNS[design]
        self.cfg = _Config(kv_bits, bucket, tile, probe_cap, flags, lock_timeout_us)
        nbytes = ctypes.c_uint64()
        _check(L.hwave_table_bytes(capacity, self.design_id, ctypes.byref(self.cfg),
                                   ctypes.byref(nbytes)))
        dv = torch.device(device if device is not None else "cuda")
        if dv.index is None:
            dv = torch.device("cuda", torch.cuda.current_device())
        self.device = dv
        self.buffer = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.hwave_create_in(ctypes.byref(h), _ptr(self.buffer), nbytes.value, capacity,
                                     self.design_id, ctypes.byref(self.cfg), _stream(stream)))
        self.h = h
        self.kv_bits = kv_bits
        self.dtype = torch.int64 if kv_bits == 64 else torch.int32
        raw = _Raw()
        _check(L.hwave_raw(self.h, ctypes.byref(raw)))
        self._raw = raw
        self.capacity = int(L.hwave_capacity(self.h))
        self.num_buckets = int(L.hwave_num_buckets(self.h))
        self.bucket_slots = int(raw.bucket_slots)
        self.tile = int(raw.tile)

    # -- lifetime
    def close(self):
        if getattr(self, "h", None):
            self._L.hwave_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def _empty(self, n, dtype=None):
        import torch
        return torch.empty(n, dtype=dtype or self.dtype, device=self.device)

    def _u8(self, n):
        import torch
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def _keys(self, t):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
            raise HashWaveError("keys/values must be contiguous %s tensors on %s" % (self.dtype, self.device))
        return t

    # -- operations (asynchronous on the current or given stream)
    def clear(self, stream=None):
        _check(self._L.hwave_clear(self.h, _stream(stream)))

    def insert(self, keys, vals, status=None, stream=None):
        n = keys.numel()
        status = self._u8(n) if status is None else status
        _check(self._L.hwave_insert(self.h, _ptr(self._keys(keys)), _ptr(self._keys(vals)), n,
                                  _ptr(status), _stream(stream)))
        return status

    def upsert(self, keys, vals, combine="sum", status=None, stream=None):
        n = keys.numel()
        status = self._u8(n) if status is None else status
        _check(self._L.hwave_upsert(self.h, _ptr(self._keys(keys)), _ptr(self._keys(vals)), n,
                                  COMBINES[combine], _ptr(status), _stream(stream)))
        return status

    def query(self, keys, out=None, found=None, stream=None):
        n = keys.numel()
        out = self._empty(n) if out is None else out
        found = self._u8(n) if found is None else found
        _check(self._L.hwave_query(self.h, _ptr(self._keys(keys)), n, _ptr(out), _ptr(found),
                                 _stream(stream)))
        return found, out

    def erase(self, keys, found=None, stream=None):
        n = keys.numel()
        found = self._u8(n) if found is None else found
        _check(self._L.hwave_erase(self.h, _ptr(self._keys(keys)), n, _ptr(found), _stream(stream)))
        return found

    def mixed(self, ops, keys, vals, combine="sum", out=None, status=None, stream=None):
        n = keys.numel()
        out = self._empty(n) if out is None else out
        status = self._u8(n) if status is None else status
        _check(self._L.hwave_mixed(self.h, _ptr(ops), _ptr(self._keys(keys)),
                                 None if vals is None else _ptr(self._keys(vals)), n,
                                 COMBINES[combine], _ptr(out), _ptr(status), _stream(stream)))
        return status, out

    def mixed_noalloc(self, ops, keys, vals, combine="sum", out=None, status=None, stream=None):
        """hwave_mixed_noalloc: a mixed call with upserts merged by key in the
        library's fixed device workspace (at most 2^18 operations)."""
        n = keys.numel()
        out = self._empty(n) if out is None else out
        status = self._u8(n) if status is None else status
        _check(self._L.hwave_mixed_noalloc(self.h, _ptr(ops), _ptr(self._keys(keys)),
                                         None if vals is None else _ptr(self._keys(vals)), n,
                                         COMBINES[combine], _ptr(out), _ptr(status), _stream(stream)))
        return status, out

    def size(self, stream=None) -> int:
        import torch
        c = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self._L.hwave_size(self.h, _ptr(c), _stream(stream)))
        return int(c.item())

    def export(self, stream=None):
        """(keys, vals) of every live pair, unordered."""
        import torch
        k = self._empty(self.capacity)
        v = self._empty(self.capacity)
        c = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self._L.hwave_export(self.h, _ptr(k), _ptr(v), _ptr(c), _stream(stream)))
        n = int(c.item())
        return k[:n], v[:n]

    def primary_bucket(self, keys, stream=None):
        n = keys.numel()
        out = self._empty(n, dtype=__import__("torch").int64)
        _check(self._L.hwave_primary_bucket(self.h, _ptr(self._keys(keys)), n, _ptr(out),
                                          _stream(stream)))
        return out

    def candidate_buckets(self, keys, stream=None):
        """(n, 3) int64 tensor: the buckets each key may occupy (C-ABI
        hwave_candidate_buckets; unused entries -1)."""
        n = keys.numel()
        out = self._empty(3 * n, dtype=__import__("torch").int64)
        _check(self._L.hwave_candidate_buckets(self.h, _ptr(self._keys(keys)), n, _ptr(out),
                                             _stream(stream)))
        return out.view(n, 3)

    def probe_counters(self, reset: bool = False, stream=None) -> dict:
        """Probe counters (instrumented tables only, C-ABI hwave_probe_counters): queries and the
        lines they read, and the locked upserts and the buckets their searches looked at."""
        c = _Probe()
        _check(self._L.hwave_probe_counters(self.h, ctypes.byref(c), int(bool(reset)), _stream(stream)))
        return {"queries": c.queries, "bucket_lines": c.bucket_lines, "slot_lines": c.slot_lines,
                "writes": c.writes, "write_visits": c.write_visits}

    def raw(self):
        """Views of the raw device image: dict(slots=uint8, tags=int16 or None, locks=int32 words of
        lock bytes, lock_queues=int64 ticket words)."""
        import torch
        base = self.buffer.data_ptr()
        r = self._raw
        slot_bytes = int(r.slot_bytes)
        out = {"slots": self.buffer[r.slots - base: r.slots - base + slot_bytes]}
        if r.tags:
            off = r.tags - base
            out["tags"] = self.buffer[off: off + 2 * self.capacity].view(torch.int16)
        else:
            out["tags"] = None
        off = r.locks - base
        out["locks"] = self.buffer[off: off + 4 * r.n_lock_words].view(torch.int32)
        out["lock_stride"] = int(r.lock_stride)
        off = r.lock_queues - base
        out["lock_queues"] = self.buffer[off: off + 8 * r.n_lock_queues].view(torch.int64)
        return out


class Multi:
    """A group of tables (one key width) served by one persistent kernel per call."""

    def __init__(self, tables, stream=None):
        self.tables = list(tables)
        if not self.tables:
            raise HashWaveError("empty table group")
        self.kv_bits = self.tables[0].kv_bits
        arr = (ctypes.c_void_p * len(self.tables))(*[t.h.value for t in self.tables])
        h = ctypes.c_void_p()
        _check(lib().hwave_multi_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p),
                                        len(self.tables), _stream(stream)))
        self.h = h

    def kernel(self):
        """(kind, waves per SIMD) of the kernel the group runs on; kind is 'menu',
        'extended' or 'solo' (every table on one configuration)."""
        k, wv = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().hwave_multi_kernel(self.h, ctypes.byref(k), ctypes.byref(wv)))
        return ("menu", "extended", "solo")[k.value], wv.value

    def close(self):
        if getattr(self, "h", None):
            lib().hwave_multi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        _check(lib().hwave_multi_clear(self.h, _stream(stream)))

    def run(self, items, keys, vals=None, out=None, status=None, stream=None):
        """items: sequence of (table, op, begin, end) with op an int (OPS value |
        combine << 8).  Returns (status, out) tensors."""
        import torch
        n = keys.numel()
        dt = keys.dtype
        out = torch.empty(n, dtype=dt, device=keys.device) if out is None else out
        status = torch.empty(n, dtype=torch.uint8, device=keys.device) if status is None else status
        arr = (_Item * len(items))(*[_Item(int(a), int(b), int(c), int(d)) for a, b, c, d in items])
        _check(lib().hwave_multi_run(self.h, ctypes.cast(arr, ctypes.c_void_p), len(items), _ptr(keys),
                                     _ptr(vals), _ptr(out), _ptr(status), _stream(stream)))
        return status, out

    def upsert(self, offsets, keys, vals, combine="sum", status=None, stream=None):
        import torch
        n = keys.numel()
        status = torch.empty(n, dtype=torch.uint8, device=keys.device) if status is None else status
        offs = (ctypes.c_uint64 * len(offsets))(*[int(x) for x in offsets])
        _check(lib().hwave_multi_upsert(self.h, ctypes.cast(offs, ctypes.c_void_p), _ptr(keys), _ptr(vals),
                                        COMBINES[combine], _ptr(status), _stream(stream)))
        return status


def multi_upsert_tables(tables, d_offsets, keys, vals, combine="sum", status=None, stream=None):
    """hwave_multi_upsert_tables: table i receives ops [d_offsets[i], d_offsets[i+1])
    of the shared arrays as one upsert, in one persistent launch; d_offsets is an
    int64 device tensor of len(tables) + 1 entries."""
    import torch
    n = keys.numel()
    status = torch.empty(n, dtype=torch.uint8, device=keys.device) if status is None else status
    arr = (ctypes.c_void_p * len(tables))(*[t.h.value for t in tables])
    _check(lib().hwave_multi_upsert_tables(ctypes.cast(arr, ctypes.c_void_p), len(tables), _ptr(d_offsets),
                                           _ptr(keys), _ptr(vals), COMBINES[combine], _ptr(status),
                                           _stream(stream)))
    return status


class Server:
    """Request loop over resident tables (C-ABI hwave_server_*).

    mode "batched": continuous batching into persistent multi-table launches;
    mode "plain": one request at a time with single-table launches (baseline).
    Request arrays are pinned CPU tensors (torch pin_memory) the caller keeps
    alive until drain()."""

    def __init__(self, tables, mode="batched", slots=3, slot_ops=1 << 22, max_requests=0, device=0):
        self.tables = list(tables)
        arr = (ctypes.c_void_p * len(self.tables))(*[t.h.value for t in self.tables])
        cfg = _ServerCfg(0 if mode == "batched" else 1, slots, slot_ops, max_requests, device)
        h = ctypes.c_void_p()
        _check(lib().hwave_server_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p),
                                         len(self.tables), ctypes.byref(cfg)))
        self.h = h
        self._keep = []

    @staticmethod
    def request(table, op, keys, vals=None, out=None, status=None):
        n = keys.numel()
        return _Request(int(table), int(op), n, keys.data_ptr(), 0 if vals is None else vals.data_ptr(),
                        0 if out is None else out.data_ptr(), 0 if status is None else status.data_ptr())

    def submit(self, table, op, keys, vals=None, out=None, status=None, arrival=0.0):
        r = self.request(table, op, keys, vals, out, status)
        t = ctypes.c_uint64()
        _check(lib().hwave_server_submit(self.h, ctypes.byref(r), arrival, ctypes.byref(t)))
        self._keep.append((keys, vals, out, status))
        return t.value

    def replay(self, requests, offsets_s):
        """requests: list of _Request (see request()); offsets_s: arrival times (s)."""
        arr = (_Request * len(requests))(*requests)
        offs = (ctypes.c_double * len(offsets_s))(*[float(x) for x in offsets_s])
        t0 = ctypes.c_double()
        _check(lib().hwave_server_replay(self.h, ctypes.cast(arr, ctypes.c_void_p),
                                         ctypes.cast(offs, ctypes.c_void_p), len(requests), ctypes.byref(t0)))
        return t0.value

    def drain(self):
        _check(lib().hwave_server_drain(self.h))

    def stats(self):
        st = _ServeStats()
        _check(lib().hwave_server_stats(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _ServeStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().hwave_server_destroy(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def multi_supported(kv_bits, design, bucket, tile) -> bool:
    return bool(lib().hwave_multi_supported(kv_bits, DESIGNS[design], bucket, tile))


def autotune(kv_bits: int, capacity: int, designs=("DOUBLE", "DOUBLE_M", "P2", "P2_M"), load=0.85,
             reps=3, flags=0, stream=None):
    """Times every multi-table menu configuration of `designs` for tables of
    `capacity` slots (C-ABI hwave_autotune).  Returns (best, all) as dicts."""
    mask = 0
    for d in designs:
        mask |= 1 << DESIGNS[d]
    res = (_Tune * 64)()
    n = ctypes.c_uint32()
    best = _Tune()
    _check(lib().hwave_autotune(kv_bits, capacity, mask, load, reps, flags, res, 64, ctypes.byref(n),
                                ctypes.byref(best), _stream(stream)))
    return _tune_dict(best), [_tune_dict(res[i]) for i in range(min(n.value, 64))]


def _tune_dict(r):
    names = {v: k for k, v in DESIGNS.items()}
    return {"design": names[r.design], "bucket": r.bucket_slots, "tile": r.tile, "kv_bits": r.kv_bits,
            "gops": r.gops, "full_ops": r.full_ops, "load": r.load, "flags": r.flags}


def tune_classes(kv_bits: int, exponents, path=None, **kw):
    """Autotunes each capacity class 2^e at one load and set of flags (keyword
    arguments of `autotune`); returns {e: best} and, with `path`, saves it (C-ABI
    hwave_tune_save).  Each entry records the load and flags it was tuned for."""
    table = {}
    for e in exponents:
        best, _ = autotune(kv_bits, 1 << e, **kw)
        table[int(e)] = best
    if path:
        save_tuning(path, table)
    return table


def save_tuning(path, table):
    """Writes {log2 capacity: best-configuration dict} (C-ABI hwave_tune_save)."""
    es = sorted(table)
    arr = (_Tune * max(1, len(es)))()
    caps = (ctypes.c_uint32 * max(1, len(es)))()
    for i, e in enumerate(es):
        v = table[e]
        arr[i] = _Tune(DESIGNS[v["design"]], v["bucket"], v["tile"], v["kv_bits"], v["gops"], v.get("full_ops", 0),
                       v["load"], v.get("flags", 0), 0)
        caps[i] = int(e)
    _check(lib().hwave_tune_save(os.fsencode(path), caps, arr, len(es)))


def load_tuning(path, cap=64):
    """Reads what save_tuning wrote (C-ABI hwave_tune_load): {log2 capacity: dict}."""
    arr = (_Tune * cap)()
    caps = (ctypes.c_uint32 * cap)()
    n = ctypes.c_uint32()
    _check(lib().hwave_tune_load(os.fsencode(path), caps, arr, cap, ctypes.byref(n)))
    return {int(caps[i]): _tune_dict(arr[i]) for i in range(n.value)}

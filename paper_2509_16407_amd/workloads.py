"""Seeded synthetic input generators shared by the tests, the benchmark and the oracle runs.

This module holds no hash-table arithmetic: it only draws numbers.  Every
random quantity a workload needs (keys, values, shuffles, Zipf ranks, arrival
times) is produced here from named, published generators and handed to both
sides as plain arrays.

* splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state advances by the odd constant
  0x9E3779B97F4A7C15 and each output is a bijective mix of the state, so the
  outputs of one stream at distinct counters are distinct.  A stream is fully
  described by its 64-bit seed; element i of the stream is the output after
  i+1 advances.
* Zipf(theta) ranks by the closed-form inversion of Gray, Sundaresan,
  Englert, Baclawski and Weinberger, "Quickly generating billion-record
  synthetic databases", SIGMOD 1994 (the method the YCSB client uses).
* Fisher-Yates shuffles driven by a splitmix64 stream.

The workload recipes (which stream feeds which array) follow the evaluation
setups of the paper's load benchmark (Section 6.3) and mixed-operation aging
benchmark (Section 6.5); they are documented with each function below.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)

U64_MAX = (1 << 64) - 1

# Largest chunk materialised at once, to bound host memory on 2^28-key workloads.
_CHUNK = 1 << 24


def stream_seed(config: int, purpose: int) -> int:
    """Seed of the splitmix64 stream for (workload config id, purpose id)."""
    return ((config & 0xFFFFFFFF) << 32) | (purpose & 0xFFFFFFFF)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Elements [start, start+count) of the splitmix64 stream with the given seed (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    if count >= 4096:
        _helper().sm64_fill(_c_u64(seed & U64_MAX), _c_u64(start), _c_u64(count), _cptr(out))
        return out
    s0 = np.uint64(seed & U64_MAX)
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = s0 + ctr * GAMMA
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
        out[:] = z ^ (z >> _S31)
    return out


def distinct_keys(seed: int, count: int, key_bits: int = 64, n_reserved: int = 3,
                  skip: int = 0) -> np.ndarray:
    """`count` distinct keys: a splitmix64 stream with the top `n_reserved` values of the
    key range removed (those are the table's reserved key patterns).

    Keys are taken in stream order after dropping the first `skip` accepted keys, so
    `distinct_keys(s, a)` followed by `distinct_keys(s, b, skip=a)` continues the same
    stream: the two arrays are disjoint (splitmix64 is a bijection of its counter).
    For key_bits=32 the stream output is truncated to its low 32 bits and duplicates
    are removed by keeping first occurrences (in stream order).
    """
    if key_bits == 64:
        limit = U64_MAX - n_reserved  # keys must be <= limit
        need = skip + count
        # reserved values appear with probability ~3/2^64: draw, filter, top up.
        raw = splitmix64(seed, 0, need)
        ok = raw <= np.uint64(limit)
        pos = need
        while int(ok.sum()) < need:
            extra = splitmix64(seed, pos, need - int(ok.sum()))
            pos += len(extra)
            raw = np.concatenate([raw[ok], extra])
            ok = raw <= np.uint64(limit)
        return raw[ok][skip:need].copy()
    if key_bits == 32:
        limit = (1 << 32) - 1 - n_reserved
        need = skip + count
        got = np.empty(0, dtype=np.uint64)
        pos = 0
        while len(got) < need:
            batch = splitmix64(seed, pos, max(need - len(got), 1024) + (need >> 4))
            pos += len(batch)
            cand = batch & np.uint64(0xFFFFFFFF)
            cand = cand[cand <= np.uint64(limit)]
            allk = np.concatenate([got, cand])
            _, first = np.unique(allk, return_index=True)
            first.sort()
            got = allk[first]
        return got[skip:need].copy()
    raise ValueError("key_bits must be 32 or 64")


def uniform_below(seed: int, start: int, count: int, bound: int) -> np.ndarray:
    """`count` integers uniform in [0, bound) from a splitmix64 stream (multiply-shift
    reduction of the high 32 bits; bound < 2^32)."""
    assert 0 < bound < (1 << 32)
    r = splitmix64(seed, start, count) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return ((r * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)


def unit_float(seed: int, start: int, count: int) -> np.ndarray:
    """`count` doubles uniform in [0, 1): top 53 bits of a splitmix64 stream."""
    r = splitmix64(seed, start, count) >> np.uint64(11)
    return r.astype(np.float64) * (1.0 / (1 << 53))


def permutation(seed: int, n: int) -> np.ndarray:
    """Fisher-Yates permutation of range(n) driven by a splitmix64 stream.

    Step i (from n-1 down to 1) swaps position i with j = floor(u_i * (i+1)), u_i the
    i-th stream double.  Vectorised draws, sequential swaps in chunks for big n.
    """
    p = np.arange(n, dtype=np.int64)
    if n <= 1:
        return p
    u = unit_float(seed, 0, n - 1)  # u[k] drives step i = n-1-k
    idx = np.arange(n - 1, 0, -1, dtype=np.int64)
    j = np.minimum((u * (idx + 1)).astype(np.int64), idx)
    _swap_loop(p, idx, j)
    return p


def _swap_loop(p, idx, j):
    """Sequential Fisher-Yates swaps (numpy has no vectorised form); a compiled
    loop takes over for large n."""
    n = len(idx)
    if n > 200000:
        _swap_loop_fast(p, idx, j)
        return
    for k in range(n):
        a = idx[k]
        b = j[k]
        p[a], p[b] = p[b], p[a]


_lib = None


def _c_u64(x):
    import ctypes
    return ctypes.c_uint64(int(x))


def _cptr(a):
    import ctypes
    return a.ctypes.data_as(ctypes.c_void_p)


def _swap_loop_fast(p, idx, j):
    import ctypes
    _helper().fy_swaps(_cptr(p), _cptr(idx), _cptr(j), ctypes.c_int64(len(idx)))


_HELPER_SRC = r"""
#include <stdint.h>
static inline uint64_t sm64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
void sm64_fill(uint64_t seed, uint64_t start, uint64_t count, uint64_t* out) {
  for (uint64_t i = 0; i < count; i++) out[i] = sm64_at(seed, start + i);
}
void sm64_gather(uint64_t seed, const int64_t* idx, uint64_t count, uint64_t* out) {
  for (uint64_t i = 0; i < count; i++) out[i] = sm64_at(seed, (uint64_t)idx[i]);
}
uint64_t select_s(uint64_t seed, uint64_t n, uint64_t k, int64_t* out) {
  uint64_t got = 0;
  for (uint64_t i = 0; i < n && got < k; i++) {
    double u = (double)(sm64_at(seed, i) >> 11) * (1.0 / 9007199254740992.0);
    if ((double)(n - i) * u < (double)(k - got)) out[got++] = (int64_t)i;
  }
  return got;
}
/* 4-round Feistel permutation of 32-bit values (Luby-Rackoff), round function
   = low 16 bits of splitmix64 keyed by (key, round): distinct x give distinct y. */
static inline uint32_t feistel32(uint64_t key, uint32_t x) {
  uint32_t L = x >> 16, R = x & 0xFFFFu;
  for (int r = 0; r < 4; r++) {
    uint32_t F = (uint32_t)(sm64_at(key ^ ((uint64_t)r << 56), R) & 0xFFFFu);
    uint32_t nl = R;
    R = L ^ F;
    L = nl;
  }
  return (L << 16) | R;
}
/* Group-by batch of one table: D distinct 32-bit keys (top two patterns skipped)
   at even positions, each followed by a uniform repeat of one of them; values
   from a second stream.  keys/vals hold 2D entries. */
void groupby_fill(uint64_t seed, uint64_t D, uint32_t* keys, uint32_t* vals) {
  uint64_t got = 0;
  uint32_t x = 0;
  while (got < D) {
    uint32_t k = feistel32(seed, x++);
    if (k >= 0xFFFFFFFEu) continue;
    keys[2 * got] = k;
    got++;
  }
  for (uint64_t i = 0; i < D; i++) keys[2 * i + 1] = keys[2 * (sm64_at(seed ^ 0x5bd1e9955bd1e995ull, i) % D)];
  for (uint64_t j = 0; j < 2 * D; j++) vals[j] = (uint32_t)sm64_at(seed ^ 0x6c62272e07bb0142ull, j);
}
void fy_swaps(int64_t* p, const int64_t* idx, const int64_t* j, int64_t n) {
  for (int64_t k = 0; k < n; k++) { int64_t a = idx[k], b = j[k];
    int64_t t = p[a]; p[a] = p[b]; p[b] = t; }
}
"""


def _helper():
    """The generators' inner loops compiled once with the host C compiler."""
    global _lib
    if _lib is None:
        import ctypes
        import hashlib
        import os
        import subprocess
        import tempfile
        tag = hashlib.sha1(_HELPER_SRC.encode()).hexdigest()[:12]
        d = os.path.join(tempfile.gettempdir(), "hw_workloads_%d" % os.getuid())
        os.makedirs(d, exist_ok=True)
        so = os.path.join(d, "gen_%s.so" % tag)
        if not os.path.exists(so):
            c = os.path.join(d, "gen_%s.c" % tag)
            with open(c, "w") as f:
                f.write(_HELPER_SRC)
            tmp = so + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", c, "-o", tmp])
            os.replace(tmp, so)
        lib = ctypes.CDLL(so)
        P, U = ctypes.c_void_p, ctypes.c_uint64
        lib.sm64_fill.argtypes = [U, U, U, P]
        lib.sm64_fill.restype = None
        lib.sm64_gather.argtypes = [U, P, U, P]
        lib.sm64_gather.restype = None
        lib.select_s.argtypes = [U, U, U, P]
        lib.select_s.restype = U
        lib.fy_swaps.argtypes = [P, P, P, ctypes.c_int64]
        lib.fy_swaps.restype = None
        lib.groupby_fill.argtypes = [U, U, P, P]
        lib.groupby_fill.restype = None
        _lib = lib
    return _lib


class Zipf:
    """Zipf(theta) ranks in [0, n) by the Gray et al. (1994) inversion.

    zeta(n) = sum_{i=1..n} i^-theta; alpha = 1/(1-theta);
    eta = (1 - (2/n)^(1-theta)) / (1 - zeta(2)/zeta(n)).
    For u uniform in [0,1): uz = u*zeta(n); rank 0 if uz < 1, rank 1 if uz < 1 + 0.5^theta,
    else floor(n * (eta*u - eta + 1)^alpha).
    """

    def __init__(self, n: int, theta: float = 0.99):
        assert n >= 2 and 0 < theta < 1
        self.n = int(n)
        self.theta = float(theta)
        zn = 0.0
        for c0 in range(1, n + 1, _CHUNK):
            c1 = min(n + 1, c0 + _CHUNK)
            zn += float(np.sum(np.arange(c0, c1, dtype=np.float64) ** (-theta)))
        self.zetan = zn
        zeta2 = 1.0 + 0.5 ** theta
        self.alpha = 1.0 / (1.0 - theta)
        self.eta = (1.0 - (2.0 / n) ** (1.0 - theta)) / (1.0 - zeta2 / zn)
        self.half_pow = 0.5 ** theta

    def ranks(self, seed: int, start: int, count: int) -> np.ndarray:
        u = unit_float(seed, start, count)
        uz = u * self.zetan
        r = np.floor(self.n * np.power(self.eta * u - self.eta + 1.0, self.alpha))
        r = np.minimum(r, self.n - 1).astype(np.int64)
        r = np.where(uz < 1.0 + self.half_pow, 1, r)
        r = np.where(uz < 1.0, 0, r)
        return r


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns plain numpy arrays; nothing here knows how the
# table stores or finds keys.
# ---------------------------------------------------------------------------

def value_of(keys: np.ndarray, key_bits: int = 64) -> np.ndarray:
    """Value convention of the load benchmarks: v = 3k + 1 (wrapping)."""
    with np.errstate(over="ignore"):
        v = keys * np.uint64(3) + np.uint64(1)
    if key_bits == 32:
        v &= np.uint64(0xFFFFFFFF)
    return v


def load_then_query(capacity: int, load: float, workload_id: int = 1):
    """Insert floor(load*capacity) distinct keys (v = 3k+1), then query them plus the
    same number of absent keys (continuation of the key stream), shuffled.

    Returns dict(keys, vals, qkeys, expect_found) where expect_found marks the
    positive queries.  Absent keys are guaranteed distinct from inserted ones.
    """
    n = int(load * capacity)
    s_keys = stream_seed(workload_id, 1)
    keys = distinct_keys(s_keys, n)
    absent = distinct_keys(s_keys, n, skip=n)
    q = np.concatenate([keys, absent])
    perm = permutation(stream_seed(workload_id, 2), len(q))
    qkeys = q[perm]
    expect_found = perm < n
    return dict(keys=keys, vals=value_of(keys), qkeys=qkeys, expect_found=expect_found)


def load_phases(capacity: int, fractions=(0.5, 0.75, 0.9), workload_id: int = 2):
    """Distinct-key insert phases filling a table to each fraction of `capacity`.

    Phase p inserts keys [floor(f_{p-1} * cap), floor(f_p * cap)) of one stream.
    Returns (all_keys, bounds) with bounds[p] = cumulative count after phase p.
    """
    bounds = [int(f * capacity) for f in fractions]
    keys = distinct_keys(stream_seed(workload_id, 1), bounds[-1])
    return keys, bounds


def mixed_batches(universe: int, batch: int, n_batches: int, theta: float = 0.99,
                  frac_upsert: float = 0.3, frac_erase: float = 0.2, workload_id: int = 3,
                  ukeys: np.ndarray | None = None):
    """Generator of deterministic mixed batches over a Zipf-distributed key universe.

    The universe is `universe` distinct keys (stream (config,1), or the given `ukeys`);
    Zipf ranks index it.  Per batch of `batch` ops (n_up = floor(frac_upsert*batch)
    upserts, n_er = floor(frac_erase*batch) erases, the rest queries), draws are
    interleaved: a stream of candidates, each a kind (query / upsert / erase in
    those proportions) and a Zipf rank, is read in order; the first candidate that
    names a rank makes that kind the rank's owner for the batch, and a candidate is
    kept only if its kind owns its rank (erases: only the first, so erase keys are
    distinct), until every kind has its count.  So every kind draws from the whole
    distribution -- a hot rank is as likely to become an upsert key (repeated many
    times) as its kind's share -- and the three key sets stay disjoint.
    Upsert values: a splitmix64 stream; op order shuffled.
    Because erase and upsert keys are disjoint and queries avoid both, every output is
    the same under any serialisation of the batch.
    Yields dict(ops, keys, vals, ranks) with ops coded 0 query, 2 upsert, 3 erase.
    """
    if ukeys is None:
        ukeys = distinct_keys(stream_seed(workload_id, 1), universe)
    assert len(ukeys) == universe
    z = Zipf(universe, theta)
    n_up = int(frac_upsert * batch)
    n_er = int(frac_erase * batch)
    n_q = batch - n_up - n_er
    want = np.array([n_q, n_up, n_er], dtype=np.int64)
    cum = np.cumsum(want / batch)
    zs = stream_seed(workload_id, 3)
    ks = stream_seed(workload_id, 5)
    zpos = 0
    owner = np.full(universe, -1, dtype=np.int8)   # rank -> owning kind this batch
    etaken = np.zeros(universe, dtype=bool)        # rank already erased this batch
    for b in range(n_batches):
        got = [[], [], []]
        have = np.zeros(3, dtype=np.int64)
        touched = []
        rate = np.ones(3)  # kept / drawn per kind in the last chunk
        drawn = 0
        while (have < want).any():
            if drawn > 64 * batch:
                raise ValueError("mixed_batches: a %d-key universe is too small for %d distinct erase keys "
                                 "per batch" % (universe, n_er))
            # enough candidates for the slowest kind at its last acceptance rate
            need = (want - have) / (want / batch) / np.maximum(rate, 0.02)
            m = int(1.1 * need.max()) + 4096
            r = z.ranks(zs, zpos, m)
            kind = np.searchsorted(cum, unit_float(ks, zpos, m), side="right").clip(0, 2).astype(np.int8)
            zpos += m
            drawn += m
            # a rank's owner is the kind of its first candidate (earlier chunks first)
            uniq, first = np.unique(r, return_index=True)
            fresh = owner[uniq] < 0
            owner[uniq[fresh]] = kind[first[fresh]]
            touched.append(uniq[fresh])
            ok = owner[r] == kind
            # erases: the first candidate of each rank only, across chunks too
            idx = np.flatnonzero(ok & (kind == 2))
            if len(idx):
                _, fi = np.unique(r[idx], return_index=True)
                keep = np.zeros(len(idx), dtype=bool)
                keep[fi] = ~etaken[r[idx[fi]]]
                etaken[r[idx[keep]]] = True
                ok[idx[~keep]] = False
            for k in range(3):
                offered = kind == k
                kept = r[ok & offered]
                rate[k] = len(kept) / max(1, int(offered.sum()))
                sel = kept[: int(want[k] - have[k])]
                got[k].append(sel)
                have[k] += len(sel)
        for u in touched:
            owner[u] = -1
            etaken[u] = False
        qr, up, er = (np.concatenate(g) for g in got)
        ops = np.concatenate([np.zeros(n_q, np.uint8), np.full(n_up, 2, np.uint8),
                              np.full(n_er, 3, np.uint8)])
        ranks = np.concatenate([qr, up, er])
        vals = np.zeros(batch, dtype=np.uint64)
        vals[n_q:n_q + n_up] = splitmix64(stream_seed(workload_id, 4), b * batch, n_up)
        perm = permutation(stream_seed(workload_id, 1000 + b), batch)
        yield dict(ops=ops[perm], keys=ukeys[ranks[perm]], vals=vals[perm], ranks=ranks[perm])


def hottest_upsert_share(batch: dict) -> float:
    """Share of a mixed batch's upserts that go to its most frequent upsert key."""
    u = batch["ops"] == 2
    if not u.any():
        return 0.0
    _, c = np.unique(batch["ranks"][u], return_counts=True)
    return float(c.max()) / float(u.sum())


def sample_without_replacement(seed: int, n: int, k: int) -> np.ndarray:
    """k distinct indices of range(n), uniform without replacement, increasing.

    Selection sampling (Knuth, TAOCP vol. 2, 3.4.2, Algorithm S; Fan, Muller and
    Rezucha 1962): index i is taken when (n - i) * u_i < k - (taken so far), u_i the
    i-th double of the splitmix64 stream `seed`."""
    assert 0 <= k <= n
    out = np.empty(k, dtype=np.int64)
    if k:
        got = _helper().select_s(_c_u64(seed & U64_MAX), _c_u64(n), _c_u64(k), _cptr(out))
        assert got == k
    return out


def universe_keys(universe: int, workload_id: int = 3) -> np.ndarray:
    """The key universe used by `mixed_batches` (same stream)."""
    return distinct_keys(stream_seed(workload_id, 1), universe)


def groupby_tables(exponents, load: float = 0.85, workload_id: int = 4):
    """Group-by aggregation batches for tables of capacity 2^e (e in `exponents`):
    table t gets D_t = floor(load * 2^e) distinct uint32 keys, each followed by a
    uniform repeat of one of them, with uint32 values.  Returns (offsets, keys,
    vals): table t's ops are [offsets[t], offsets[t+1]) of the uint32 arrays."""
    ds = [int(load * (1 << int(e))) for e in exponents]
    offsets = np.zeros(len(ds) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([2 * d for d in ds])
    keys = np.empty(int(offsets[-1]), dtype=np.uint32)
    vals = np.empty(int(offsets[-1]), dtype=np.uint32)
    h = _helper()

    def fill(t):
        a, d = int(offsets[t]), ds[t]
        h.groupby_fill(_c_u64(stream_seed(workload_id, 1 << 20 | t)), _c_u64(d),
                       _cptr(keys[a: a + 2 * d]), _cptr(vals[a: a + 2 * d]))

    import concurrent.futures as cf
    import os
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(len(ds))))
    return offsets, keys, vals


def table_exponents(n_tables: int, e_min: int, e_max: int, workload_id: int = 4) -> np.ndarray:
    """Capacity exponents uniform in [e_min, e_max] (log-uniform capacities)."""
    return uniform_below(stream_seed(workload_id, 2), 0, n_tables, e_max - e_min + 1) + e_min


def splitmix64_at(seed: int, idx: np.ndarray) -> np.ndarray:
    """Elements idx[i] of the splitmix64 stream `seed` (uint64)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.uint64)
    if len(idx):
        _helper().sm64_gather(_c_u64(seed & U64_MAX), _cptr(idx), _c_u64(len(idx)), _cptr(out))
    return out


def served_requests(n_tables: int, universe: int, n_req: int, rate_per_s: float, log2_min: float = 8,
                    log2_max: float = 20, theta: float = 0.99, mix=(0.5, 0.3, 0.2), workload_id: int = 5):
    """Request stream of the served form: Poisson arrivals at `rate_per_s` (exponential
    gaps), table uniform over n_tables, kind query / upsert / insert with
    probabilities `mix`, size floor(2^U) with U uniform in [log2_min, log2_max], keys
    Zipf(theta) ranks over a per-table universe whose rank-r key is element r of
    stream (config, 100 + table).  Yields dicts (t_offset, table, kind, keys, vals);
    insert values are 3k+1, upsert values a separate stream."""
    u = unit_float(stream_seed(workload_id, 1), 0, 4 * n_req)
    z = Zipf(universe, theta)
    t = 0.0
    zpos = 0
    for i in range(n_req):
        t += -np.log(1.0 - u[4 * i]) / rate_per_s
        table = min(int(u[4 * i + 1] * n_tables), n_tables - 1)
        r = u[4 * i + 2]
        kind = "query" if r < mix[0] else ("upsert" if r < mix[0] + mix[1] else "insert")
        n = int(2.0 ** (log2_min + (log2_max - log2_min) * u[4 * i + 3]))
        ranks = z.ranks(stream_seed(workload_id, 2), zpos, n)
        keys = splitmix64_at(stream_seed(workload_id, 100 + table), ranks)
        if kind == "insert":
            vals = value_of(keys)
        elif kind == "upsert":
            vals = splitmix64(stream_seed(workload_id, 3), zpos, n)
        else:
            vals = None
        zpos += n
        yield dict(t=t, table=table, kind=kind, keys=keys, vals=vals)


def poisson_arrivals(seed: int, rate_per_s: float, seconds: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process at `rate_per_s` over [0, seconds):
    exponential gaps -ln(1 - u) / rate from a splitmix64 stream."""
    n = int(rate_per_s * seconds * 1.2) + 64
    while True:
        t = np.cumsum(-np.log1p(-unit_float(seed, 0, n)) / rate_per_s)
        if t[-1] >= seconds:
            return t[t < seconds]
        n *= 2


def stream_keys(seed: int, start: int, count: int) -> np.ndarray:
    """Elements [start, start+count) of a splitmix64 stream used directly as 64-bit
    keys.  Disjoint position ranges give disjoint keys (the mix is a bijection of the
    counter).  A stream value equal to one of the three reserved key patterns (odds
    about 3 in 2^64 per key) raises instead of being dropped, so positions stay
    exact."""
    k = splitmix64(seed, start, count)
    if count and int(k.max()) > U64_MAX - 3:
        raise ValueError("stream %#x hit a reserved key pattern in [%d, %d)" % (seed, start, start + count))
    return k


def aging_plan(capacity: int, load: float = 0.85, frac: float = 0.01, iters: int = 1000,
               workload_id: int = 6):
    """The aging (churn) benchmark of Section 6.5.  The table is filled to `load`
    (n0 = floor(load * capacity) keys, v = 3k+1); then every iteration, in ONE
    mixed launch, inserts the next s = floor(frac * n0) new keys, erases the oldest
    s live keys, queries s live keys and s keys never inserted.

    Key j of one stream is inserted by the preload when j < n0, else by iteration
    (j - n0) // s; iteration i erases keys [i*s, (i+1)*s).  Its positive queries are
    the s keys starting at pos_start[i], a seeded offset inside the keys that stay
    live through iteration i; its negative queries are negs[i*s:(i+1)*s], stream
    positions past every inserted key.  Every output of an iteration is therefore
    the same under any order of its operations: inserts and erases succeed,
    positives return 3k+1, negatives miss.

    Returns dict(n0, s, iters, keys, negs, pos_start)."""
    n0 = int(load * capacity)
    s = max(1, int(frac * n0))
    if n0 < 2 * s:
        raise ValueError("the fill must hold at least two slices")
    total = n0 + iters * s
    seed = stream_seed(workload_id, 1)
    keys = stream_keys(seed, 0, total)
    negs = stream_keys(seed, total, iters * s)
    off = uniform_below(stream_seed(workload_id, 2), 0, iters, n0 - 2 * s + 1)
    pos_start = (np.arange(iters, dtype=np.int64) + 1) * s + off.astype(np.int64)
    return dict(n0=n0, s=s, iters=iters, keys=keys, negs=negs, pos_start=pos_start)

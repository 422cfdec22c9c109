"""GPU parity: every HIP-path result against the CPU oracle, element by element.

Batches are built so that every compared output is the same under any
serialisation of the concurrent batch (distinct keys per insert/erase batch,
equal values for duplicate inserts, commutative sums for duplicate upserts);
where the order decides a status among duplicates, per-key counts are compared.
Sizes span many tiles with a ragged tail.  Every test also runs the oracle's
layout checker on the raw table image (no duplicate key, every key in a
candidate bucket, tags consistent, no reservation marker, all locks released).
"""
import numpy as np
import pytest

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import busy_lock_queues, dev, full_is_genuine, host, image, per_key_counts, u8

pytestmark = pytest.mark.gpu

ODESIGN = {"DOUBLE": oracle.DOUBLE, "DOUBLE_M": oracle.DOUBLE_M, "P2": oracle.P2, "P2_M": oracle.P2_M,
           "ICEBERG": oracle.ICEBERG, "ICEBERG_M": oracle.ICEBERG_M, "CUCKOO": oracle.CUCKOO}
ALL = ["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG", "ICEBERG_M"]


def check_layout(t, neg_keys=None, tile_bytes=None):
    slots, tags, locks = image(t)
    tb = tile_bytes or (t.tile * 16)
    nv, rep = oracle.layout_check(ODESIGN[t.design], t.kv_bits, t.num_buckets, t.bucket_slots,
                                  slots, tags, locks, neg_keys=neg_keys, tile_bytes=tb)
    assert nv == 0, rep
    assert busy_lock_queues(t) == 0  # every ticket taken was served
    return rep


def check_dump(t, om):
    k, v = t.export()
    k, v = host(k, t.kv_bits), host(v, t.kv_bits)
    order = np.argsort(k)
    ok, ov = om.dump()
    assert len(k) == len(ok)
    assert np.array_equal(k[order], ok)
    assert np.array_equal(v[order], ov)
    assert t.size() == len(ok)


# ------------------------------------------------------------------ load benchmark, double hashing at 2^20 slots

def test_load_double_hashing_2p20():
    """2^20-slot double hashing, bucket 8: insert 943,718 keys (v = 3k+1), query them
    and 943,718 absent keys; all outputs, the dump and the layout against the oracle."""
    d = w.load_then_query(1 << 20, 0.9, workload_id=1)
    t = hw.Table(1 << 20, "DOUBLE")
    assert t.capacity == 1 << 20 and t.num_buckets == 1 << 17
    om = oracle.OracleMap()
    st = u8(t.insert(dev(d["keys"]), dev(d["vals"])))
    assert np.array_equal(st, om.insert(d["keys"], d["vals"]))
    found, vals = t.query(dev(d["qkeys"]))
    ost, oval = om.query(d["qkeys"])
    assert np.array_equal(u8(found), ost)
    assert np.array_equal(host(vals), oval)
    check_dump(t, om)
    neg = d["qkeys"][~d["expect_found"]][:100000]
    rep = check_layout(t, neg_keys=neg)
    # Table 1 (load probes, query): 1.22 unique lines per positive query
    assert abs(rep["pos_probe_sum"] / rep["live"] - 1.22) < 0.02


# ------------------------------------------------------------------ every design, all ops

CASES = [
    ("DOUBLE", 64, 8, 8), ("DOUBLE", 64, 8, 4), ("DOUBLE", 64, 16, 8), ("DOUBLE", 64, 32, 16),
    ("DOUBLE_M", 64, 32, 4), ("DOUBLE_M", 64, 32, 8), ("DOUBLE_M", 64, 16, 4), ("DOUBLE_M", 64, 64, 8),
    ("P2", 64, 32, 8), ("P2", 64, 32, 4), ("P2", 64, 32, 32), ("P2", 64, 16, 8),
    ("P2_M", 64, 32, 4), ("P2_M", 64, 32, 8), ("P2_M", 64, 32, 16), ("P2_M", 64, 64, 8),
    ("ICEBERG", 64, 32, 8), ("ICEBERG", 64, 32, 4), ("ICEBERG", 64, 32, 16),
    ("ICEBERG_M", 64, 32, 4), ("ICEBERG_M", 64, 32, 8), ("ICEBERG_M", 64, 64, 8),
    ("DOUBLE", 32, 16, 8), ("DOUBLE_M", 32, 32, 4), ("P2", 32, 32, 8), ("P2_M", 32, 32, 4),
    ("P2_M", 32, 32, 32), ("DOUBLE", 32, 64, 32), ("ICEBERG", 32, 32, 8), ("ICEBERG", 32, 32, 4),
    ("ICEBERG_M", 32, 32, 4), ("ICEBERG_M", 32, 32, 8),
    ("CUCKOO", 64, 8, 4), ("CUCKOO", 64, 8, 8), ("CUCKOO", 64, 16, 8),
    ("DOUBLE_M", 64, 32, 2), ("P2_M", 64, 32, 2), ("ICEBERG_M", 64, 32, 2),
]


@pytest.mark.parametrize("design,bits,bucket,tile", CASES,
                         ids=["%s-u%d-b%d-t%d" % c for c in CASES])
def test_all_ops_against_oracle(design, bits, bucket, tile):
    cap = 1 << 16
    t = hw.Table(cap, design, kv_bits=bits, bucket=bucket, tile=tile)
    assert t.capacity == cap
    om = oracle.OracleMap(key_bits=bits)
    seed = w.stream_seed(100 + ODESIGN[design], bits * 1000 + bucket * 10 + tile)
    pool = w.distinct_keys(seed, int(1.3 * cap), key_bits=bits)
    absent = w.distinct_keys(seed, 20000, key_bits=bits, skip=len(pool))
    vals_of = lambda k: w.value_of(k, bits)
    # (a) first load: 0.55 of capacity, ragged batch size
    n1 = int(0.55 * cap) + 7
    k1 = pool[:n1]
    st = u8(t.insert(dev(k1, bits), dev(vals_of(k1), bits)))
    assert np.array_equal(st, om.insert(k1, vals_of(k1)))
    # (b) insert again: half present (EXISTED, value kept), half new
    k2 = np.concatenate([pool[: n1 // 2], pool[n1: n1 + 9001]])
    v2 = vals_of(k2) ^ np.uint64(1)  # present keys must keep their old value
    perm = w.permutation(seed + 1, len(k2))
    k2, v2 = k2[perm], v2[perm]
    st = u8(t.insert(dev(k2, bits), dev(v2, bits)))
    assert np.array_equal(st, om.insert(k2, v2))
    # (c) queries: present and absent, shuffled
    q = np.concatenate([pool[: n1 + 9001: 3], absent])
    q = q[w.permutation(seed + 2, len(q))]
    f, v = t.query(dev(q, bits))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v, bits), ov)
    # (d) SUM upserts with duplicates: existing keys and new keys, each 1-3 times
    base = np.concatenate([pool[1000:4000], pool[n1 + 9001: n1 + 12001]])
    reps = w.uniform_below(seed + 3, 0, len(base), 3) + 1
    ku = np.repeat(base, reps)
    vu = w.splitmix64(seed + 4, 0, len(ku))
    if bits == 32:
        vu &= np.uint64(0xFFFFFFFF)
    p = w.permutation(seed + 5, len(ku))
    ku, vu = ku[p], vu[p]
    st = u8(t.upsert(dev(ku, bits), dev(vu, bits), combine="sum"))
    ost = om.upsert(ku, vu)
    # who inserts among duplicates of a new key is racy: compare per-key counts
    assert per_key_counts(ku, st, 1) == per_key_counts(ku, ost, 1)
    assert per_key_counts(ku, st, 2) == per_key_counts(ku, ost, 2)
    assert not np.isin(st, [3, 4]).any()
    # (e) erase: distinct keys, some absent
    ke = np.concatenate([pool[2000:2000 + 15000:2], absent[:3000]])
    ke = ke[w.permutation(seed + 6, len(ke))]
    st = u8(t.erase(dev(ke, bits)))
    assert np.array_equal(st, om.erase(ke))
    # (f) refill past the first load (reuses freed slots), then re-query everything
    lim = 0.8 if design.startswith("P2") else 0.9
    n_more = int(lim * cap) - om.size()
    k3 = pool[n1 + 12001: n1 + 12001 + n_more]
    st = u8(t.insert(dev(k3, bits), dev(vals_of(k3), bits)))
    assert np.array_equal(st, om.insert(k3, vals_of(k3)))
    q = np.concatenate([pool, absent])
    f, v = t.query(dev(q, bits))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v, bits), ov)
    # (g) other combines on present keys (distinct keys per batch)
    for comb, code in (("replace", oracle.REPLACE), ("min", oracle.MIN), ("max", oracle.MAX),
                       ("keep", oracle.KEEP)):
        kc = pool[5000:9000]
        vc = w.splitmix64(seed + 10 + code, 0, len(kc))
        if bits == 32:
            vc &= np.uint64(0xFFFFFFFF)
        st = u8(t.upsert(dev(kc, bits), dev(vc, bits), combine=comb))
        assert np.array_equal(st, om.upsert(kc, vc, combine=code))
    check_dump(t, om)
    check_layout(t)


# ------------------------------------------------------------------ mixed batches (Zipf 0.99, disjoint erase / upsert / query keys)

@pytest.mark.parametrize("design", ["DOUBLE_M", "P2_M", "DOUBLE", "P2", "ICEBERG_M", "ICEBERG", "CUCKOO"])
def test_mixed_batches_against_oracle(design):
    """Preload a 2^k-key universe to load 0.5, then mixed batches (50% query, 30% SUM
    upsert, 20% erase, Zipf 0.99 keys; erase and upsert keys disjoint, queries avoid
    both): query outputs, erase flags, per-key upsert statuses and the dump after
    every batch match the oracle."""
    cap = 1 << 18
    universe = cap // 2
    t = hw.Table(cap, design)
    om = oracle.OracleMap()
    uk = w.universe_keys(universe, workload_id=3)
    st = u8(t.insert(dev(uk), dev(w.value_of(uk))))
    assert np.array_equal(st, om.insert(uk, w.value_of(uk)))
    for b in w.mixed_batches(universe, 1 << 15, 4, workload_id=3):
        ops = b["ops"]
        import torch
        s, v = t.mixed(torch.from_numpy(ops).cuda(), dev(b["keys"]), dev(b["vals"]), combine="sum")
        s, v = u8(s), host(v)
        os_, ov = om.apply(b["keys"], b["vals"], ops=ops, combine=oracle.SUM)
        det = ops != 2  # query and erase outputs are serialisation-independent
        assert np.array_equal(s[det], os_[det])
        assert np.array_equal(v[det], ov[det])
        up = ops == 2
        assert per_key_counts(b["keys"][up], s[up], 1) == per_key_counts(b["keys"][up], os_[up], 1)
        assert per_key_counts(b["keys"][up], s[up], 2) == per_key_counts(b["keys"][up], os_[up], 2)
        check_dump(t, om)
    check_layout(t)


# ------------------------------------------------------------------ 32-bit group-by over many tables

@pytest.mark.parametrize("flags", [0, hw.F_NO_ERASE], ids=["locked", "noerase"])
@pytest.mark.parametrize("design", ALL)
@pytest.mark.parametrize("logcap", [10, 14, 17])
def test_u32_groupby_sum(design, logcap, flags):
    """Group-by hash aggregation: D = 0.85 * capacity distinct uint32 keys, each upserted
    once plus D extra uniform repeats; result = wrapping sums per key.  In tiny
    power-of-two-choice tables a key may find both buckets full: that FULL is
    accepted only when the final image shows both buckets full."""
    cap = 1 << logcap
    t = hw.Table(cap, design, kv_bits=32, flags=flags)
    cap = t.capacity
    D = int(0.85 * cap)
    seed = w.stream_seed(4, logcap * 8 + ODESIGN[design])
    keys = w.distinct_keys(seed, D, key_bits=32)
    extra = keys[w.uniform_below(seed + 1, 0, D, D)]
    ops_k = np.concatenate([keys, extra])
    ops_k = ops_k[w.permutation(seed + 2, len(ops_k))]
    ops_v = w.splitmix64(seed + 3, 0, len(ops_k)) & np.uint64(0xFFFFFFFF)
    st = u8(t.upsert(dev(ops_k, 32), dev(ops_v, 32), combine="sum"))
    full = st == hw.ST_FULL
    if full.any():
        assert not design.startswith("DOUBLE"), "double hashing reported FULL below capacity"
        full_is_genuine(t, ops_k[full])
        # a key that never got in is absent from the table: drop all its ops
        lost = np.setdiff1d(ops_k[full], ops_k[st == hw.ST_DONE])
        keep = ~np.isin(ops_k, lost)
        keep &= ~full
        ops_k, ops_v, st = ops_k[keep], ops_v[keep], st[keep]
    om = oracle.OracleMap(key_bits=32)
    ost = om.upsert(ops_k, ops_v)
    assert per_key_counts(ops_k, st, 1) == per_key_counts(ops_k, ost, 1)
    check_dump(t, om)
    check_layout(t)


# ------------------------------------------------------------------ edge cases

@pytest.mark.parametrize("design", ALL)
def test_sentinels_and_empty_batches(design):
    import torch
    t = hw.Table(1 << 12, design)
    top = (1 << 64) - 1
    bad = np.array([top, top - 1, top - 2], np.uint64)
    st = u8(t.insert(dev(bad), dev(bad)))
    assert (st == hw.ST_INVALID).all()
    f, v = t.query(dev(bad))
    assert (u8(f) == hw.ST_INVALID).all() and (host(v) == 0).all()
    assert (u8(t.erase(dev(bad))) == hw.ST_INVALID).all()
    assert (u8(t.upsert(dev(bad), dev(bad))) == hw.ST_INVALID).all()
    assert t.size() == 0
    ok = np.array([top - 3, 0, 1], np.uint64)
    assert (u8(t.insert(dev(ok), dev(ok))) == hw.ST_DONE).all()
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    t.insert(e, e)
    t.query(e)
    t.erase(e)
    t.upsert(e, e)
    assert t.size() == 3
    check_layout(t)


@pytest.mark.parametrize("design,bucket", [("DOUBLE", 8), ("DOUBLE_M", 32)])
def test_double_hashing_fills_every_slot(design, bucket):
    """Double hashing visits every bucket, so FULL happens exactly when all
    capacity slots hold keys: 1100 distinct inserts into 1024 slots give 1024
    inserted and 76 FULL; after erasing one key, one more insert succeeds."""
    t = hw.Table(1024, design)
    keys = w.distinct_keys(77, 1100)
    st = u8(t.insert(dev(keys), dev(w.value_of(keys))))
    assert (st == hw.ST_DONE).sum() == 1024 and (st == hw.ST_FULL).sum() == 76
    inserted = keys[st == hw.ST_DONE]
    om = oracle.OracleMap(capacity=1024)
    om.insert(inserted, w.value_of(inserted))
    check_dump(t, om)
    rep = check_layout(t)
    assert rep["live"] == 1024 and rep["empties"] == 0
    full = keys[st == hw.ST_FULL]
    assert (u8(t.erase(dev(inserted[:1]))) == hw.ST_DONE).all()
    st2 = u8(t.insert(dev(full[:2]), dev(w.value_of(full[:2]))))
    assert sorted(st2.tolist()) == [hw.ST_DONE, hw.ST_FULL]
    check_layout(t)


def test_primary_bucket_hook_matches_oracle():
    """The adversarial benchmark's device hook (Section 4.1) agrees with the oracle's
    independent restatement of the hash rule."""
    t = hw.Table(1 << 20, "P2_M")
    keys = w.distinct_keys(5, 10000)
    got = t.primary_bucket(dev(keys)).cpu().numpy()
    exp = np.array([oracle.primary_bucket(int(k), t.num_buckets) for k in keys[:2000]])
    assert np.array_equal(got[:2000], exp)
    assert got.max() < t.num_buckets
    # iceberg: the front-yard bucket (its lock guards the key)
    t = hw.Table(1 << 20, "ICEBERG_M")
    got = t.primary_bucket(dev(keys)).cpu().numpy()
    exp = np.array([oracle.iceberg_buckets(int(k), t.num_buckets)[0] for k in keys[:2000]])
    assert np.array_equal(got[:2000], exp)
    assert got.max() < oracle.iceberg_front_buckets(t.num_buckets)


def test_candidate_bucket_hook_matches_oracle():
    """hwave_candidate_buckets (used to check that a FULL status was legal) agrees
    with the oracle's independent restatement of each design's placement rule:
    two-choice primary and alternate, iceberg front and backyard choices, cuckoo's
    three buckets, double hashing's primary bucket and probe step."""
    keys = w.distinct_keys(6, 3000)
    for design in ("P2_M", "P2", "ICEBERG_M", "CUCKOO", "DOUBLE_M", "DOUBLE"):
        t = hw.Table(1 << 20, design)
        nb = t.num_buckets
        got = t.candidate_buckets(dev(keys)).cpu().numpy().view(np.uint64)
        for i, k in enumerate(keys.tolist()):
            if design.startswith("P2"):
                exp = (oracle.primary_bucket(k, nb), oracle.p2_alternate(k, nb), (1 << 64) - 1)
            elif design.startswith("ICEBERG"):
                exp = oracle.iceberg_buckets(k, nb)
            elif design == "CUCKOO":
                exp = oracle.cuckoo_buckets(k, nb)
            else:
                b0 = oracle.double_probe(k, nb, 0)
                exp = (b0, (oracle.double_probe(k, nb, 1) - b0) % nb, (1 << 64) - 1)
            assert tuple(int(x) for x in got[i]) == tuple(exp), (design, k)


# ------------------------------------------------------------------ iceberg load

@pytest.mark.parametrize("design,paper", [("ICEBERG", 2.97), ("ICEBERG_M", 2.16)])
def test_iceberg_load_2p20(design, paper):
    """2^20-slot iceberg table, one insert batch to 0.9 load and a query batch of
    those keys plus as many absent ones: every output, the dump and the layout
    against the oracle; no backyard key has room in its front bucket (the table
    never erased); positive-query probes near Table 1's load-phase figure."""
    d = w.load_then_query(1 << 20, 0.9, workload_id=1)
    t = hw.Table(1 << 20, design)
    om = oracle.OracleMap()
    st = u8(t.insert(dev(d["keys"]), dev(d["vals"])))
    assert np.array_equal(st, om.insert(d["keys"], d["vals"]))
    found, vals = t.query(dev(d["qkeys"]))
    ost, oval = om.query(d["qkeys"])
    assert np.array_equal(u8(found), ost)
    assert np.array_equal(host(vals), oval)
    check_dump(t, om)
    neg = d["qkeys"][~d["expect_found"]][:100000]
    rep = check_layout(t, neg_keys=neg)
    assert rep["front_room"] == 0
    # concurrent placement differs from the sequential one only in which of
    # several equal choices a key takes
    assert abs(rep["pos_probe_sum"] / rep["live"] - paper) < 0.03


@pytest.mark.parametrize("design", ALL)
def test_no_erase_table_rejects_erase(design):
    import torch
    t = hw.Table(1 << 12, design, flags=hw.F_NO_ERASE)
    k = w.distinct_keys(3, 100)
    assert (u8(t.insert(dev(k), dev(k))) == hw.ST_DONE).all()
    with pytest.raises(hw.HashWaveError):
        t.erase(dev(k))
    ops = torch.full((100,), 3, dtype=torch.uint8, device="cuda")
    st, _ = t.mixed(ops, dev(k), dev(k))
    assert (u8(st) == hw.ST_INVALID).all()
    assert t.size() == 100
    f, v = t.query(dev(k))
    assert (u8(f) == hw.ST_DONE).all() and np.array_equal(host(v), k)


# ------------------------------------------------------------------ phased variant

@pytest.mark.parametrize("design", ALL + ["CHAINING", "CUCKOO"])
def test_phased_variant_against_oracle(design):
    """The phased (bulk-synchronous) variant, used in phased fashion: distinct-key
    insert batches, then queries, then an erase batch and a refill, then queries --
    every output, the dump and the layout against the oracle."""
    cap = 1 << 16
    t = hw.Table(cap, design, flags=hw.F_BSP)
    om = oracle.OracleMap()
    seed = w.stream_seed(110, hw.DESIGNS[design])
    pool = w.distinct_keys(seed, int(0.95 * cap))
    absent = w.distinct_keys(seed, 20000, skip=len(pool))
    n1 = int(0.8 * cap) + 5
    for a, b in ((0, n1 // 2), (n1 // 2, n1)):
        k = pool[a:b]
        st = u8(t.insert(dev(k), dev(w.value_of(k))))
        assert np.array_equal(st, om.insert(k, w.value_of(k)))
    q = np.concatenate([pool, absent])
    q = q[w.permutation(seed + 1, len(q))]
    f, v = t.query(dev(q))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov)
    ke = pool[: n1: 3]
    assert np.array_equal(u8(t.erase(dev(ke))), om.erase(ke))
    k = pool[n1: int(0.9 * cap)]
    assert np.array_equal(u8(t.insert(dev(k), dev(w.value_of(k)))), om.insert(k, w.value_of(k)))
    f, v = t.query(dev(q))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov)
    check_dump(t, om)
    if design == "CHAINING":
        slots, _, locks = image(t)
        nv, rep = oracle.chain_check(t.num_buckets, slots, locks)
        assert nv == 0, rep
    else:
        check_layout(t)


def test_phased_variant_not_accepted_by_multi():
    t = hw.Table(1 << 12, "P2_M", flags=hw.F_BSP)
    with pytest.raises(hw.HashWaveError):
        hw.Multi([t])


# ------------------------------------------------------------------ cuckoo at high load

@pytest.mark.parametrize("tile", [4, 8])
def test_cuckoo_high_load_moves_keys(tile):
    """Three-way cuckoo filled to 0.93 in two batches: the second batch finds most
    candidate buckets full and has to move keys along displacement paths; every
    insert still succeeds, every key is found with its value, the layout holds
    (each key in one of its three buckets), and erase then re-query agree with
    the oracle."""
    cap = 1 << 16
    t = hw.Table(cap, "CUCKOO", tile=tile)
    om = oracle.OracleMap()
    keys = w.distinct_keys(w.stream_seed(140, tile), int(0.93 * cap))
    for part in (keys[: int(0.8 * cap)], keys[int(0.8 * cap):]):
        st = u8(t.insert(dev(part), dev(w.value_of(part))))
        assert np.array_equal(st, om.insert(part, w.value_of(part)))
    rep = check_layout(t)
    assert rep["in_alternate"] > 0
    f, v = t.query(dev(keys))
    assert (u8(f) == hw.ST_DONE).all() and np.array_equal(host(v), w.value_of(keys))
    ke = keys[::3]
    assert np.array_equal(u8(t.erase(dev(ke))), om.erase(ke))
    f, v = t.query(dev(keys))
    of, ov = om.query(keys)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov)
    check_dump(t, om)
    check_layout(t)

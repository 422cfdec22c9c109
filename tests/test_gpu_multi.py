"""The batched form: one persistent launch over many tables of uneven
capacities and configurations, compared bit-exactly with one plain launch per
table and with the oracle; plus the autotuner."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, u8

pytestmark = pytest.mark.gpu

MENU32 = [("DOUBLE", 16, 4), ("DOUBLE", 16, 8), ("DOUBLE", 32, 16), ("DOUBLE", 64, 32),
          ("DOUBLE", 128, 64), ("DOUBLE_M", 32, 4), ("P2", 32, 8), ("P2_M", 16, 4), ("P2_M", 32, 4),
          ("P2_M", 32, 8)]
MENU64 = [("DOUBLE", 8, 8), ("DOUBLE", 16, 8), ("DOUBLE_M", 32, 4), ("DOUBLE_M", 32, 8), ("P2", 32, 8),
          ("P2_M", 32, 4), ("P2_M", 32, 8), ("P2_M", 64, 8)]
# the extended 64-bit menu adds these (a group holding one runs on it)
MENU64X = MENU64 + [("ICEBERG", 32, 8), ("ICEBERG_M", 32, 4), ("CHAINING", 7, 8), ("CUCKOO", 8, 4)]


def _dump(t):
    k, v = t.export()
    k, v = host(k, t.kv_bits), host(v, t.kv_bits)
    o = np.argsort(k)
    return k[o], v[o]


def test_menus_match_library():
    for d, b, t in MENU32:
        assert hw.multi_supported(32, d, b, t)
    for d, b, t in MENU64X:
        assert hw.multi_supported(64, d, b, t)
    assert not hw.multi_supported(32, "P2", 64, 32)
    assert not hw.multi_supported(32, "CUCKOO", 8, 4)


def test_multi_upsert_tables_with_device_offsets():
    """The table-array form with device offsets (hwave_multi_upsert_tables): the
    same group-by as a group's call, twice in a row on the same tables (the
    library reuses its group), equal to the oracle's sums table by table."""
    n = 12
    exps = w.table_exponents(n, 9, 13, workload_id=43)
    cfgs = [MENU32[i % len(MENU32)] for i in range(n)]
    offsets, keys, vals = w.groupby_tables(exps, 0.6, workload_id=43)
    A = [hw.Table(1 << int(e), d, kv_bits=32, bucket=b, tile=t) for e, (d, b, t) in zip(exps, cfgs)]
    kd = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    od = torch.from_numpy(np.asarray(offsets, dtype=np.int64)).cuda()
    for rnd in range(2):
        st = u8(hw.multi_upsert_tables(A, od, kd, vd, combine="sum"))
        assert ((st == hw.ST_DONE) | (st == hw.ST_EXISTED)).all()
    for i in range(n):
        a, b = int(offsets[i]), int(offsets[i + 1])
        om = oracle.OracleMap(key_bits=32)
        kk, vv = keys[a:b].astype(np.uint64), vals[a:b].astype(np.uint64)
        om.upsert(kk, vv)
        om.upsert(kk, vv)
        k, v = _dump(A[i])
        ok, ov = om.dump()
        assert np.array_equal(k, ok) and np.array_equal(v, ov), i


@pytest.mark.parametrize("flags", [0, hw.F_NO_ERASE], ids=["locked", "noerase"])
def test_multi_groupby_equals_plain_and_oracle(flags):
    n = 2 * len(MENU32) * 3
    exps = w.table_exponents(n, 9, 14, workload_id=41)
    cfgs = [MENU32[i % len(MENU32)] for i in range(n)]
    # power-of-two-choice tables get a lower fill so no key finds both buckets full
    offsets, keys, vals = w.groupby_tables(exps, 0.65, workload_id=41)
    A = [hw.Table(1 << int(e), d, kv_bits=32, bucket=b, tile=t, flags=flags) for e, (d, b, t) in zip(exps, cfgs)]
    B = [hw.Table(1 << int(e), d, kv_bits=32, bucket=b, tile=t, flags=flags) for e, (d, b, t) in zip(exps, cfgs)]
    m = hw.Multi(A)
    kd = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    st = u8(m.upsert(offsets, kd, vd, combine="sum"))
    for i, t in enumerate(B):  # plain form: one launch per table
        a, b = int(offsets[i]), int(offsets[i + 1])
        t.upsert(kd[a:b], vd[a:b], combine="sum")
    for i in range(n):
        a, b = int(offsets[i]), int(offsets[i + 1])
        kk = keys[a:b].astype(np.uint64)
        vv = vals[a:b].astype(np.uint64)
        om = oracle.OracleMap(key_bits=32)
        ost = om.upsert(kk, vv)
        assert (st[a:b] == hw.ST_DONE).sum() == (ost == oracle.DONE).sum(), i
        assert not (st[a:b] == hw.ST_FULL).any(), i
        ok, ov = om.dump()
        ka, va = _dump(A[i])
        kb, vb = _dump(B[i])
        assert np.array_equal(ka, ok) and np.array_equal(va, ov), i
        assert np.array_equal(kb, ok) and np.array_equal(vb, ov), i
    m.clear()
    assert all(t.size() == 0 for t in A)


@pytest.mark.parametrize("menu", ["base", "extended"])
def test_multi_mixed_items_u64(menu):
    """Items of every kind across tables of every configuration of the u64 menu
    (base, or extended with iceberg, chaining and cuckoo); at most one writing
    item per table per launch, so every output is deterministic; a third launch
    erases."""
    tabs = [hw.Table(1 << 14, d, bucket=b, tile=t) for d, b, t in (MENU64 if menu == "base" else MENU64X)]
    m = hw.Multi(tabs)
    assert m.kernel() == (("menu", 6) if menu == "base" else ("extended", 4))
    _mixed_items_u64(tabs, m)


@pytest.mark.parametrize("cfg", MENU64X, ids=["%s-b%d-t%d" % c for c in MENU64X])
def test_multi_solo_mixed_items_u64(cfg):
    """A group whose tables share one configuration runs on that configuration's
    own kernel (eight waves per SIMD; iceberg six, cuckoo four): the same three
    launches as above, on four tables of uneven capacities."""
    d, b, t = cfg
    tabs = [hw.Table(1 << e, d, bucket=b, tile=t) for e in (14, 15, 14, 16)]
    m = hw.Multi(tabs)
    assert m.kernel() == ("solo", {"ICEBERG": 6, "ICEBERG_M": 6, "CUCKOO": 4}.get(d, 8))
    _mixed_items_u64(tabs, m)


def _mixed_items_u64(tabs, m):
    oms = [oracle.OracleMap() for _ in tabs]
    pool = [w.distinct_keys(w.stream_seed(42, i), 20000) for i in range(len(tabs))]
    # launch 1: insert 10000 keys per table
    keys = np.concatenate([p[:10000] for p in pool])
    vals = w.value_of(keys)
    items = [(i, hw.OPS["insert"], i * 10000, (i + 1) * 10000) for i in range(len(tabs))]
    st, _ = m.run(items, dev(keys), dev(vals))
    st = u8(st)
    for i, om in enumerate(oms):
        assert np.array_equal(st[i * 10000:(i + 1) * 10000], om.insert(pool[i][:10000], w.value_of(pool[i][:10000])))
    # launch 2: per table either a query item (present + absent keys) or an upsert item
    segs, items, pos = [], [], 0
    for i in range(len(tabs)):
        if i % 2 == 0:
            k = np.concatenate([pool[i][:5000], pool[i][15000:18000]])
            op = hw.OPS["query"]
        else:
            k = np.concatenate([pool[i][2000:6000], pool[i][10000:12000]])
            op = hw.OPS["upsert"] | (hw.COMBINES["sum"] << 8)
        segs.append(k)
        items.append((i, op, pos, pos + len(k)))
        pos += len(k)
    keys = np.concatenate(segs)
    vals = w.splitmix64(43, 0, len(keys))
    st, out = m.run(items, dev(keys), dev(vals))
    st, out = u8(st), host(out)
    for i, (t, op, a, b) in enumerate(items):
        if op == hw.OPS["query"]:
            os_, ov = oms[i].query(keys[a:b])
            assert np.array_equal(st[a:b], os_) and np.array_equal(out[a:b], ov)
        else:
            os_ = oms[i].upsert(keys[a:b], vals[a:b])
            assert np.array_equal(st[a:b], os_)
    # launch 3: erase items (present and absent keys) on every table
    segs, items, pos = [], [], 0
    for i in range(len(tabs)):
        k = np.concatenate([pool[i][:3000:2], pool[i][19000:19500]])
        segs.append(k)
        items.append((i, hw.OPS["erase"], pos, pos + len(k)))
        pos += len(k)
    keys = np.concatenate(segs)
    st, _ = m.run(items, dev(keys), None)
    st = u8(st)
    for i, (t, op, a, b) in enumerate(items):
        assert np.array_equal(st[a:b], oms[i].erase(keys[a:b]))
    for i, t in enumerate(tabs):
        ok, ov = oms[i].dump()
        k, v = _dump(t)
        assert np.array_equal(k, ok) and np.array_equal(v, ov)


@pytest.mark.parametrize("cfg", MENU32, ids=["%s-b%d-t%d" % c for c in MENU32])
def test_multi_solo_groupby_u32(cfg):
    """Group-by SUM upserts on a group of 32-bit tables of one configuration (its
    own kernel, eight waves per SIMD), twice in a row, equal to the oracle table
    by table; the same tables with one of another configuration added run on the
    menu's kernel."""
    d, b, t = cfg
    n = 9
    exps = w.table_exponents(n, 9, 14, workload_id=45)
    offsets, keys, vals = w.groupby_tables(exps, 0.65, workload_id=45)
    A = [hw.Table(1 << int(e), d, kv_bits=32, bucket=b, tile=t) for e in exps]
    m = hw.Multi(A)
    assert m.kernel() == ("solo", 8)
    other = next(c for c in MENU32 if c != cfg)
    assert hw.Multi(A + [hw.Table(1 << 10, other[0], kv_bits=32, bucket=other[1], tile=other[2])]).kernel() == \
        ("menu", 6)
    kd = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    for rnd in range(2):
        st = u8(m.upsert(offsets, kd, vd, combine="sum"))
        assert ((st == hw.ST_DONE) | (st == hw.ST_EXISTED)).all()
    for i in range(n):
        a, b_ = int(offsets[i]), int(offsets[i + 1])
        kk, vv = keys[a:b_].astype(np.uint64), vals[a:b_].astype(np.uint64)
        om = oracle.OracleMap(key_bits=32)
        om.upsert(kk, vv)
        om.upsert(kk, vv)
        k, v = _dump(A[i])
        ok, ov = om.dump()
        assert np.array_equal(k, ok) and np.array_equal(v, ov), i


SOLO_MERGING = [("P2_M", 32, 4), ("DOUBLE_M", 32, 4), ("DOUBLE", 8, 8), ("ICEBERG_M", 32, 4), ("CHAINING", 7, 8),
                ("CUCKOO", 8, 4)]


@pytest.mark.parametrize("cfg", SOLO_MERGING, ids=["%s-b%d-t%d" % c for c in SOLO_MERGING])
def test_multi_solo_merging_u64(cfg):
    """64-bit tables of one configuration that merge duplicate keys
    (HWAVE_F_AGGREGATE, erase-free as in the served form) run on the solo kernel
    with the merging path (six waves per SIMD, cuckoo four); Zipf-skewed SUM
    upserts equal the oracle's sums table by table."""
    d, b, t = cfg
    n = 6
    tabs = [hw.Table(1 << 14, d, bucket=b, tile=t, flags=hw.F_NO_ERASE | hw.F_AGGREGATE) for _ in range(n)]
    m = hw.Multi(tabs)
    assert m.kernel() == ("solo", 4 if d == "CUCKOO" else 6)
    per = 12000
    z = w.Zipf(4000, 0.99)
    keys = np.concatenate([w.distinct_keys(w.stream_seed(46, 100 + i), 4000)[z.ranks(w.stream_seed(46, i), 0, per)]
                           for i in range(n)])
    vals = w.splitmix64(w.stream_seed(46, 99), 0, len(keys))
    offsets = np.arange(n + 1, dtype=np.int64) * per
    st = u8(m.upsert(offsets, dev(keys), dev(vals), combine="sum"))
    assert ((st == hw.ST_DONE) | (st == hw.ST_EXISTED)).all()
    for i in range(n):
        a, b_ = int(offsets[i]), int(offsets[i + 1])
        om = oracle.OracleMap()
        ost = om.upsert(keys[a:b_], vals[a:b_])
        assert (st[a:b_] == hw.ST_DONE).sum() == (ost == oracle.DONE).sum(), i
        k, v = _dump(tabs[i])
        ok, ov = om.dump()
        assert np.array_equal(k, ok) and np.array_equal(v, ov), i


@pytest.mark.parametrize("logcap", [10, 12])
def test_autotune_small_class(logcap):
    """The tuner picks the fastest configuration among those that held the whole
    batch (no FULL status); in 1024-slot tables at 0.85 load some two-choice
    configurations overflow and must not be chosen."""
    best, alls = hw.autotune(32, 1 << logcap, reps=1)
    assert len(alls) == len(MENU32)
    assert (best["design"], best["bucket"], best["tile"]) in MENU32
    ok = [a for a in alls if a["full_ops"] == 0]
    assert best["full_ops"] == 0 and best["gops"] == max(a["gops"] for a in ok) and best["gops"] > 0
    assert all(a["full_ops"] == 0 for a in alls if a["design"].startswith("DOUBLE"))


def test_tune_classes_round_trip_and_extended_menu(tmp_path):
    """tune_classes on two classes, saved and loaded through the C-ABI tuning
    file, equals what it returned; the 64-bit tuner also times the extended
    menu's designs when asked, and every choice can build a table."""
    path = str(tmp_path / "tune.txt")
    table = hw.tune_classes(32, [10, 13], path=path, reps=1, load=0.8, flags=hw.F_NO_ERASE)
    assert hw.load_tuning(path) == table
    assert all(v["load"] == 0.8 and v["flags"] == hw.F_NO_ERASE for v in table.values())
    best, alls = hw.autotune(64, 1 << 12, designs=("P2_M", "ICEBERG_M", "CHAINING", "CUCKOO"), reps=1)
    assert {a["design"] for a in alls} == {"P2_M", "ICEBERG_M", "CHAINING", "CUCKOO"}
    assert best["full_ops"] == 0 and best["gops"] > 0
    hw.Table(1 << 12, best["design"], bucket=best["bucket"], tile=best["tile"])


def test_multi_erase_items_on_erase_free_tables_are_invalid():
    """An erase item on a table built with HWAVE_F_NO_ERASE reports INVALID for
    every key and leaves the table as it was; an erase item on an ordinary table
    of the same launch erases."""
    a = hw.Table(1 << 13, "P2_M", flags=hw.F_NO_ERASE)
    b = hw.Table(1 << 13, "P2_M")
    m = hw.Multi([a, b])
    keys = w.distinct_keys(w.stream_seed(44, 0), 4000)
    vals = w.value_of(keys)
    for t in (a, b):
        assert (u8(t.insert(dev(keys), dev(vals))) == hw.ST_DONE).all()
    items = [(0, hw.OPS["erase"], 0, 2000), (1, hw.OPS["erase"], 2000, 4000)]
    st, _ = m.run(items, dev(keys), None)
    st = u8(st)
    assert (st[:2000] == hw.ST_INVALID).all() and (st[2000:] == hw.ST_DONE).all()
    assert a.size() == 4000 and b.size() == 2000
    found, v = a.query(dev(keys))
    assert (u8(found) == hw.ST_DONE).all() and np.array_equal(host(v), vals)

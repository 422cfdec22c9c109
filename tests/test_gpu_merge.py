"""Mixed calls whose upserts are merged by key (HWAVE_F_MERGE_MIXED) against the oracle.

With merging, each key's upserts run as one table upsert led by the smallest
index among them, and the others follow it (EXISTED).  Applied in input order,
the oracle gives a key's first upsert INSERTED when the key was absent and the
rest EXISTED: on batches whose erase, upsert and query keys are disjoint (the
mixed generator's guarantee), every status and value is then the same element
by element, as are the dumps.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, image, u8

pytestmark = pytest.mark.gpu

ODESIGN = {"DOUBLE": oracle.DOUBLE, "DOUBLE_M": oracle.DOUBLE_M, "P2": oracle.P2, "P2_M": oracle.P2_M,
           "ICEBERG": oracle.ICEBERG, "ICEBERG_M": oracle.ICEBERG_M, "CUCKOO": oracle.CUCKOO}
COMB = {"sum": oracle.SUM, "keep": oracle.KEEP, "min": oracle.MIN, "max": oracle.MAX, "replace": oracle.REPLACE}


def _check_dump(t, om, bits=64):
    k, v = t.export()
    k, v = host(k, bits), host(v, bits)
    o = np.argsort(k)
    ok, ov = om.dump()
    assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)


def _layout(t):
    slots, tags, locks = image(t)
    nv, rep = oracle.layout_check(ODESIGN[t.design], t.kv_bits, t.num_buckets, t.bucket_slots, slots, tags, locks)
    assert nv == 0, rep


def _run(t, om, b, combine, bits=64):
    s, v = t.mixed(torch.from_numpy(b["ops"]).cuda(), dev(b["keys"], bits), dev(b["vals"], bits), combine=combine)
    os_, ov = om.apply(b["keys"], b["vals"], ops=b["ops"], combine=COMB[combine])
    return u8(s), host(v, bits), os_, ov


@pytest.mark.parametrize("design", ["P2_M", "DOUBLE_M", "P2", "DOUBLE", "ICEBERG_M", "CUCKOO"])
def test_merged_zipf_batches_match_the_oracle_exactly(design):
    """Zipf 0.99 mixed batches (hot keys are upserted thousands of times per
    batch): every status and query value, and the dump after each batch."""
    cap = 1 << 18
    universe = cap // 2
    t = hw.Table(cap, design, flags=hw.F_MERGE_MIXED)
    om = oracle.OracleMap()
    uk = w.universe_keys(universe, workload_id=3)
    assert np.array_equal(u8(t.insert(dev(uk), dev(w.value_of(uk)))), om.insert(uk, w.value_of(uk)))
    shares = []
    for b in w.mixed_batches(universe, 1 << 15, 4, workload_id=3):
        shares.append(w.hottest_upsert_share(b))
        s, v, os_, ov = _run(t, om, b, "sum")
        assert np.array_equal(s, os_)
        assert np.array_equal(v, ov)
        _check_dump(t, om)
    assert max(shares) > 0.01  # the batches do put hot keys among the upserts
    _layout(t)


@pytest.mark.parametrize("combine", ["sum", "min", "max", "keep", "replace"])
@pytest.mark.parametrize("bits", [64, 32])
def test_merged_combines(combine, bits):
    """Every combine on dense duplicates (SUM, MIN and MAX merge into one value,
    KEEP keeps the leader's, REPLACE is not merged), absent and present keys."""
    t = hw.Table(1 << 16, "P2_M", kv_bits=bits, flags=hw.F_MERGE_MIXED)
    om = oracle.OracleMap(key_bits=bits)
    keys = w.distinct_keys(w.stream_seed(70, bits), 3000, key_bits=bits)
    pre = keys[:1000]
    pv = w.splitmix64(w.stream_seed(71, bits), 0, len(pre))
    if bits == 32:
        pv &= np.uint64(0xFFFFFFFF)
    t.insert(dev(pre, bits), dev(pv, bits))
    om.insert(pre, pv)
    n = 40000
    ks = keys[w.uniform_below(w.stream_seed(72, bits), 0, n, len(keys))]
    vs = w.splitmix64(w.stream_seed(73, bits), 0, n)
    if bits == 32:
        vs &= np.uint64(0xFFFFFFFF)
    ops = np.full(n, 2, np.uint8)
    s, v, os_, ov = _run(t, om, dict(ops=ops, keys=ks, vals=vs), combine, bits)
    if combine == "replace":
        # unmerged: a serialisation-dependent winner; compare counts per key
        for code in (hw.ST_DONE, hw.ST_EXISTED):
            a = np.unique(ks[s == code], return_counts=True)
            b = np.unique(ks[os_ == code], return_counts=True)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        return
    assert np.array_equal(s, os_)
    _check_dump(t, om, bits)


def test_merged_call_larger_than_one_chunk():
    """2^20 + 4097 operations: two chunks of the workspace, run one after the
    other; statuses and state still equal the in-order oracle."""
    t = hw.Table(1 << 22, "P2_M", flags=hw.F_MERGE_MIXED)
    om = oracle.OracleMap()
    keys = w.distinct_keys(w.stream_seed(74, 1), 200000)
    n = (1 << 20) + 4097
    z = w.Zipf(len(keys), 0.99)
    ks = keys[z.ranks(w.stream_seed(75, 1), 0, n)]
    vs = w.splitmix64(w.stream_seed(76, 1), 0, n)
    ops = np.full(n, 2, np.uint8)
    s, v, os_, ov = _run(t, om, dict(ops=ops, keys=ks, vals=vs), "sum")
    assert np.array_equal(s, os_)
    _check_dump(t, om)


@pytest.mark.parametrize("design", ["DOUBLE", "P2_M"])
def test_merged_storm_on_one_bucket(design):
    """The same-bucket storm (2^16 SUM upserts over 16 keys sharing one primary
    bucket, an erase-capable table) as a merged mixed call: 16 table upserts."""
    t = hw.Table(1 << 14, design, flags=hw.F_MERGE_MIXED)
    cand = w.distinct_keys(w.stream_seed(77, 1), 200000)
    prim = t.primary_bucket(dev(cand)).cpu().numpy()
    keys16 = cand[prim == np.bincount(prim).argmax()][:16]
    n = 1 << 16
    ks = keys16[w.uniform_below(w.stream_seed(78, 1), 0, n, 16)]
    vs = w.splitmix64(w.stream_seed(79, 1), 0, n)
    om = oracle.OracleMap()
    s, v, os_, ov = _run(t, om, dict(ops=np.full(n, 2, np.uint8), keys=ks, vals=vs), "sum")
    assert np.array_equal(s, os_)
    assert (s == hw.ST_DONE).sum() == 16
    _check_dump(t, om)
    _layout(t)


def test_merged_calls_in_a_row():
    """Leaders return their workspace entries to empty, so each call starts
    clean: three different batches on the same few hundred keys (queries only on
    keys no upsert of the batch touches) each match the oracle exactly."""
    t = hw.Table(1 << 16, "DOUBLE_M", flags=hw.F_MERGE_MIXED)
    om = oracle.OracleMap()
    keys = w.distinct_keys(w.stream_seed(80, 1), 500)
    for rnd in range(3):
        n = 20000
        ks = keys[w.uniform_below(w.stream_seed(81, rnd), 0, n, len(keys))]
        vs = w.splitmix64(w.stream_seed(82, rnd), 0, n)
        ops = np.where(w.uniform_below(w.stream_seed(83, rnd), 0, n, 4) == 0, 0, 2).astype(np.uint8)
        # queries only on keys no upsert of this batch touches
        q = ops == 0
        up_keys = np.unique(ks[~q])
        ops[q & np.isin(ks, up_keys)] = 2
        s, v, os_, ov = _run(t, om, dict(ops=ops, keys=ks, vals=vs), "sum")
        assert np.array_equal(s, os_) and np.array_equal(v, ov)
    _check_dump(t, om)

"""Merging duplicate keys before they reach the table (HWAVE_F_AGGREGATE):
every status, the dump and the layout against the oracle, on the single-table
kernel and on the multi-table kernel.

Statuses of merged duplicates follow one serialisation of each 128-operation
window (the key's first operation first), so they are compared as per-key
counts, like every other batch with duplicate keys.  Zipf-hot keys are used
only on tables that never erase; tables with erase see duplicates of at most
three per key."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, image, per_key_counts, u8

pytestmark = pytest.mark.gpu

ODESIGN = {"DOUBLE": oracle.DOUBLE, "DOUBLE_M": oracle.DOUBLE_M, "P2": oracle.P2, "P2_M": oracle.P2_M,
           "ICEBERG": oracle.ICEBERG, "ICEBERG_M": oracle.ICEBERG_M}
COMB = {"sum": oracle.SUM, "keep": oracle.KEEP, "min": oracle.MIN, "max": oracle.MAX, "replace": oracle.REPLACE}


def _check_dump(t, om):
    k, v = t.export()
    k, v = host(k, t.kv_bits), host(v, t.kv_bits)
    o = np.argsort(k)
    ok, ov = om.dump()
    assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)


def _check_layout(t):
    slots, tags, locks = image(t)
    nv, rep = oracle.layout_check(ODESIGN[t.design], t.kv_bits, t.num_buckets, t.bucket_slots, slots, tags, locks)
    assert nv == 0, rep


def _counts_match(keys, st, ost):
    for code in (hw.ST_DONE, hw.ST_EXISTED, hw.ST_FULL, hw.ST_INVALID):
        assert per_key_counts(keys, st, code) == per_key_counts(keys, ost, code), code


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("design", ["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG", "ICEBERG_M"])
def test_merged_upserts_with_few_repeats(design, bits):
    """Each key 1-3 times in a shuffled batch, every combine, a ragged length and
    reserved keys mixed in; then a second batch over present and new keys."""
    cap = 1 << 15
    t = hw.Table(cap, design, kv_bits=bits, flags=hw.F_AGGREGATE)
    om = oracle.OracleMap(key_bits=bits)
    seed = w.stream_seed(120, ODESIGN[design] * 100 + bits)
    pool = w.distinct_keys(seed, int(0.7 * cap), key_bits=bits)
    top = (1 << bits) - 1
    for rnd, comb in enumerate(["sum", "keep", "min", "max", "replace", "sum"]):
        base = pool[rnd * 2000: rnd * 2000 + 6000]
        # REPLACE keeps the last value, which depends on the order: distinct keys
        reps = w.uniform_below(seed + rnd, 0, len(base), 3) + 1 if comb != "replace" else 1
        ks = np.repeat(base, reps)
        ks = np.concatenate([ks, np.array([top, top - 1], np.uint64)])  # reserved patterns
        vs = w.splitmix64(seed + 10 + rnd, 0, len(ks))
        if comb == "keep":  # which duplicate inserts is racy: equal values per key
            vs = w.value_of(ks, bits)
        if bits == 32:
            vs &= np.uint64(0xFFFFFFFF)
        p = w.permutation(seed + 20 + rnd, len(ks))
        ks, vs = ks[p][: len(ks) - 5], vs[p][: len(ks) - 5]  # ragged tail
        st = u8(t.upsert(dev(ks, bits), dev(vs, bits), combine=comb))
        ost = om.upsert(ks, vs, combine=COMB[comb])
        _counts_match(ks, st, ost)
        _check_dump(t, om)
    _check_layout(t)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("design", ["DOUBLE_M", "P2_M", "ICEBERG_M", "P2"])
def test_merged_zipf_hot_keys_no_erase(design, bits):
    """2^18 SUM upserts with Zipf(0.99) keys over 2^14 keys (the hottest takes ~9%
    of the batch) on an erase-free table: the sums and the per-key statuses equal
    the oracle's."""
    t = hw.Table(1 << 16, design, kv_bits=bits, flags=hw.F_AGGREGATE | hw.F_NO_ERASE)
    uni = w.distinct_keys(w.stream_seed(121, bits), 1 << 14, key_bits=bits)
    ranks = w.Zipf(len(uni), 0.99).ranks(w.stream_seed(122, bits), 0, 1 << 18)
    ks = uni[ranks]
    vs = w.splitmix64(w.stream_seed(123, bits), 0, len(ks))
    if bits == 32:
        vs &= np.uint64(0xFFFFFFFF)
    om = oracle.OracleMap(key_bits=bits)
    for half in (slice(0, len(ks) // 2), slice(len(ks) // 2, len(ks))):
        st = u8(t.upsert(dev(ks[half], bits), dev(vs[half], bits), combine="sum"))
        ost = om.upsert(ks[half], vs[half])
        _counts_match(ks[half], st, ost)
    _check_dump(t, om)
    _check_layout(t)


def test_merged_multi_table_equals_oracle():
    """The persistent multi-table kernel with merging tables (64-bit menu): a
    Zipf-skewed SUM batch per table, every table against the oracle."""
    menu = [("DOUBLE", 8, 8), ("DOUBLE_M", 32, 4), ("P2", 32, 8), ("P2_M", 32, 4), ("P2_M", 64, 8)]
    tabs = [hw.Table(1 << 14, d, bucket=b, tile=tt, flags=hw.F_AGGREGATE | hw.F_NO_ERASE)
            for d, b, tt in menu for _ in range(3)]
    m = hw.Multi(tabs)
    z = w.Zipf(4000, 0.99)
    parts, offs = [], [0]
    for i in range(len(tabs)):
        uni = w.distinct_keys(w.stream_seed(124, i), 4000)
        n = 3000 + 997 * i
        parts.append(uni[z.ranks(w.stream_seed(125, i), 0, n)])
        offs.append(offs[-1] + n)
    ks = np.concatenate(parts)
    vs = w.splitmix64(w.stream_seed(126, 0), 0, len(ks))
    st = u8(m.upsert(np.array(offs, np.uint64), dev(ks), dev(vs), combine="sum"))
    for i, t in enumerate(tabs):
        a, b = offs[i], offs[i + 1]
        om = oracle.OracleMap()
        ost = om.upsert(ks[a:b], vs[a:b])
        _counts_match(ks[a:b], st[a:b], ost)
        _check_dump(t, om)

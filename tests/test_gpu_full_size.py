"""Full size: the load benchmark's step at 2^28 slots on the power-of-two-choice
table with tags (bucket 32, tile 4), built and launched exactly as the benchmark
times it.

* Every output of the step (inserts to 0.9 load, 2^27 positive and negative
  queries, 2^27 SUM upserts, the 50% erase and the re-queries) is checked
  against closed forms that hold at any size: values are 3k+1 (3k+2 after the
  upsert), absent and erased keys miss, the size is inserted - erased.
* Then one of the step's mixed 2^20-operation Zipf batches runs on that table,
  and every one of its outputs is compared with the oracle, which is given only
  the keys the batch touches, in the state the closed forms fix for them."""
import numpy as np
import pytest

import bench
import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, per_key_counts, u8

pytestmark = pytest.mark.gpu


def test_full_size_step_and_mixed_batch_against_oracle():
    d = bench.make_inputs(28, 1, 1 << 20)
    step = bench.Step(d, "P2_M", 0, 0)  # the benchmark's defaults: bucket 32, tile 4
    assert (step.t.bucket_slots, step.t.tile, step.t.capacity) == (32, 4, 1 << 28)
    # raises on any output that breaks its closed form, or on a FULL insert with a
    # free slot in one of its key's buckets
    n_full = bench.verify_step(step, d)
    print("full-size step verified; %d insert(s) ended FULL, each with both buckets full" % n_full)

    keys = d["keys"]
    n = len(keys)
    erased = np.zeros(n, dtype=bool)
    erased[d["er_idx"]] = True
    upserted = np.zeros(n, dtype=bool)
    upserted[d["pos_idx"]] = True
    bt = d["mixed"][0]
    ur = np.unique(bt["ranks"])
    live = ur[~erased[ur]]
    om = oracle.OracleMap()
    om.insert(keys[live], w.value_of(keys[live]) + upserted[live].astype(np.uint64))

    ops, kd, vd = step.mixed[0]
    st, out = step.t.mixed(ops, kd, vd, combine="sum")
    st, out = u8(st), host(out)
    ost, oout = om.apply(bt["keys"], bt["vals"], ops=bt["ops"])
    q, u, e = bt["ops"] == 0, bt["ops"] == 2, bt["ops"] == 3
    assert q.sum() + u.sum() + e.sum() == len(ops)
    assert np.array_equal(st[q], ost[q]) and np.array_equal(out[q], oout[q]), "queries"
    assert np.array_equal(st[e], ost[e]), "erases"
    for code in (hw.ST_DONE, hw.ST_EXISTED, hw.ST_FULL, hw.ST_INVALID):
        assert per_key_counts(bt["keys"][u], st[u], code) == per_key_counts(bt["keys"][u], ost[u], code), code
    touched = keys[ur]
    f, v = step.t.query(dev(touched))
    of, ov = om.query(touched)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov), "state after the batch"
    assert step.t.size() == n - len(d["er_idx"]) - int((ost[e] == oracle.DONE).sum()) + int((ost[u] == oracle.DONE).sum())


def test_full_size_mixed_zipf_batches_against_oracle():
    """The mixed Zipf workload at full size: a 2^27-slot DOUBLE_M table holding
    the whole 2^26-key universe (v = 3k+1), then three shuffled 2^20-operation
    batches (50% query, 30% SUM upsert, 20% erase).  Every output of every batch
    equals the oracle's; the oracle holds the keys the batches have touched so
    far, each entering in its preloaded state the first time a batch touches it.
    Afterwards every touched key's state, and the table's size, agree."""
    import torch
    U = 1 << 26
    uk = w.universe_keys(U, workload_id=3)
    t = hw.Table(1 << 27, "DOUBLE_M")
    ukd = dev(uk)
    assert bool((t.insert(ukd, ukd * 3 + 1) == 1).all())
    del ukd
    om = oracle.OracleMap()
    seen = np.zeros(U, dtype=bool)
    erased_total = inserted_total = 0
    for bt in w.mixed_batches(U, 1 << 20, 3, workload_id=3, ukeys=uk):
        ur = np.unique(bt["ranks"])
        new = ur[~seen[ur]]
        seen[new] = True
        om.insert(uk[new], w.value_of(uk[new]))
        st, out = t.mixed(torch.from_numpy(bt["ops"]).cuda(), dev(bt["keys"]), dev(bt["vals"]), combine="sum")
        st, out = u8(st), host(out)
        ost, oout = om.apply(bt["keys"], bt["vals"], ops=bt["ops"])
        q, u, e = bt["ops"] == 0, bt["ops"] == 2, bt["ops"] == 3
        assert np.array_equal(st[q], ost[q]) and np.array_equal(out[q], oout[q]), "queries"
        assert np.array_equal(st[e], ost[e]), "erases"
        for code in (hw.ST_DONE, hw.ST_EXISTED, hw.ST_FULL, hw.ST_INVALID):
            assert per_key_counts(bt["keys"][u], st[u], code) == per_key_counts(bt["keys"][u], ost[u], code), code
        erased_total += int((ost[e] == oracle.DONE).sum())
        inserted_total += int((ost[u] == oracle.DONE).sum())
    touched = uk[seen]
    f, v = t.query(dev(touched))
    of, ov = om.query(touched)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov), "state of the touched keys"
    assert t.size() == U - erased_total + inserted_total


def test_full_size_batched_groupby_against_oracle():
    """The batched form at full size: 4096 uint32 tables with capacities 2^e (e
    uniform in 10..22, ~2.7e9 slots in all), each receiving a group-by SUM-upsert
    batch that fills it to 0.85, in one persistent multi-table launch (double
    hashing, bucket 16, tile 4 for every table: the batched result the benchmark
    reports, on that configuration's own kernel).  Per table,
    exactly its distinct keys insert and its size equals their count; twelve
    sampled tables and the first of the largest class equal the oracle's
    group-by, key by key."""
    import torch
    exps = w.table_exponents(4096, 10, 22, workload_id=4)
    offsets, keys, vals = w.groupby_tables(exps, 0.85, workload_id=4)
    ds = (offsets[1:] - offsets[:-1]) // 2
    tabs = [hw.Table(1 << int(e), "DOUBLE", kv_bits=32, bucket=16, tile=4) for e in exps]
    m = hw.Multi(tabs)
    assert m.kernel() == ("solo", 8)
    kd = torch.from_numpy(keys.view(np.int32)).cuda()
    vd = torch.from_numpy(vals.view(np.int32)).cuda()
    st = m.upsert(offsets, kd, vd, combine="sum")
    del kd, vd
    assert int((st == hw.ST_DONE).sum()) == int(ds.sum())
    assert int((st == hw.ST_EXISTED).sum()) == int(ds.sum())
    del st
    assert [t.size() for t in tabs] == [int(x) for x in ds]
    pick = w.sample_without_replacement(w.stream_seed(4, 10), len(tabs), 12).tolist()
    pick.append(int(np.argmax(exps)))
    for i in pick:
        a, b = int(offsets[i]), int(offsets[i + 1])
        om = oracle.OracleMap(key_bits=32)
        om.upsert(keys[a:b].astype(np.uint64), vals[a:b].astype(np.uint64))
        k, v = tabs[i].export()
        k = k.cpu().numpy().view(np.uint32).astype(np.uint64)
        v = v.cpu().numpy().view(np.uint32).astype(np.uint64)
        o = np.argsort(k)
        ok, ov = om.dump()
        assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov), i

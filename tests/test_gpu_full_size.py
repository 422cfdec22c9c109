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
    bench.verify_step(step, d)  # raises on any output that breaks its closed form

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

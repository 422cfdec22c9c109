"""Chaining on the GPU (Section 5: chains of 128-byte nodes of 7 pairs and a link):
every output, the dump and the chain layout against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, image, per_key_counts, u8

pytestmark = pytest.mark.gpu


def _check(t, om=None, neg=None):
    slots, _, locks = image(t)
    nv, rep = oracle.chain_check(t.num_buckets, slots, locks, neg_keys=neg)
    assert nv == 0, rep
    if om is not None:
        k, v = t.export()
        k, v = host(k), host(v)
        o = np.argsort(k)
        ok, ov = om.dump()
        assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)
        assert t.size() == om.size()
    return rep


def test_chaining_geometry():
    t = hw.Table(1 << 16, "CHAINING")
    nb = (65536 + 6) // 7
    assert t.num_buckets == nb and t.bucket_slots == 7 and t.tile == 8
    assert t.capacity == 3 * nb * 7


def test_chaining_all_ops_against_oracle():
    cap = 1 << 16
    t = hw.Table(cap, "CHAINING")
    om = oracle.OracleMap()
    seed = w.stream_seed(130, 1)
    pool = w.distinct_keys(seed, int(1.3 * cap))
    absent = w.distinct_keys(seed, 20000, skip=len(pool))
    n1 = int(0.55 * cap) + 7
    k1 = pool[:n1]
    assert np.array_equal(u8(t.insert(dev(k1), dev(w.value_of(k1)))), om.insert(k1, w.value_of(k1)))
    k2 = np.concatenate([pool[: n1 // 2], pool[n1: n1 + 9001]])
    v2 = w.value_of(k2) ^ np.uint64(1)
    p = w.permutation(seed + 1, len(k2))
    k2, v2 = k2[p], v2[p]
    assert np.array_equal(u8(t.insert(dev(k2), dev(v2))), om.insert(k2, v2))
    q = np.concatenate([pool[: n1 + 9001: 3], absent])
    q = q[w.permutation(seed + 2, len(q))]
    f, v = t.query(dev(q))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov)
    base = np.concatenate([pool[1000:4000], pool[n1 + 9001: n1 + 12001]])
    reps = w.uniform_below(seed + 3, 0, len(base), 3) + 1
    ku = np.repeat(base, reps)
    vu = w.splitmix64(seed + 4, 0, len(ku))
    p = w.permutation(seed + 5, len(ku))
    ku, vu = ku[p], vu[p]
    st = u8(t.upsert(dev(ku), dev(vu), combine="sum"))
    ost = om.upsert(ku, vu)
    assert per_key_counts(ku, st, 1) == per_key_counts(ku, ost, 1)
    assert per_key_counts(ku, st, 2) == per_key_counts(ku, ost, 2)
    ke = np.concatenate([pool[2000:2000 + 15000:2], absent[:3000]])
    ke = ke[w.permutation(seed + 6, len(ke))]
    assert np.array_equal(u8(t.erase(dev(ke))), om.erase(ke))
    k3 = pool[n1 + 12001: n1 + 12001 + int(0.9 * cap) - om.size()]
    assert np.array_equal(u8(t.insert(dev(k3), dev(w.value_of(k3)))), om.insert(k3, w.value_of(k3)))
    q = np.concatenate([pool, absent])
    f, v = t.query(dev(q))
    of, ov = om.query(q)
    assert np.array_equal(u8(f), of) and np.array_equal(host(v), ov)
    for comb, code in (("replace", oracle.REPLACE), ("min", oracle.MIN), ("max", oracle.MAX)):
        kc = pool[5000:9000]
        vc = w.splitmix64(seed + 10 + code, 0, len(kc))
        assert np.array_equal(u8(t.upsert(dev(kc), dev(vc), combine=comb)), om.upsert(kc, vc, combine=code))
    _check(t, om)


def test_chaining_layout_equals_sequential_placement():
    """Seven keys per bucket (chains of length 1 in expectation): under the bucket
    lock the k-th key of a bucket lands in node k // 7 + 1 whatever the order, so
    the positive-probe total equals the sequential simulator's exactly, and the
    negative probes (chain lengths) too."""
    t = hw.Table(7 * 8192, "CHAINING")
    nb = t.num_buckets
    keys = w.distinct_keys(w.stream_seed(131, 1), 7 * nb)
    neg = w.distinct_keys(w.stream_seed(131, 1), 50000, skip=len(keys))
    st = u8(t.insert(dev(keys), dev(w.value_of(keys))))
    assert (st == hw.ST_DONE).all()
    rep = _check(t, neg=neg)
    nodes, failed = oracle.sim_chain_insert(nb, nb + nb // 2 + 1, keys)
    assert failed == 0
    _, srep = oracle.chain_check(nb, nodes, neg_keys=neg)
    assert rep["live"] == srep["live"] == len(keys)
    assert rep["pos_probe_sum"] == srep["pos_probe_sum"]
    assert rep["neg_probe_sum"] == srep["neg_probe_sum"]


def test_chaining_pool_exhaustion_reports_full():
    """One bucket and a two-node pool hold 21 keys; the rest report FULL; an erase
    makes room for exactly one more."""
    t = hw.Table(7, "CHAINING")
    assert t.num_buckets == 1
    keys = w.distinct_keys(132, 30)
    st = u8(t.insert(dev(keys), dev(w.value_of(keys))))
    assert (st == hw.ST_DONE).sum() == 21 and (st == hw.ST_FULL).sum() == 9
    done = keys[st == hw.ST_DONE]
    om = oracle.OracleMap()
    om.insert(done, w.value_of(done))
    _check(t, om)
    assert (u8(t.erase(dev(done[:1]))) == hw.ST_DONE).all()
    full = keys[st == hw.ST_FULL]
    st2 = u8(t.insert(dev(full[:2]), dev(w.value_of(full[:2]))))
    assert sorted(st2.tolist()) == [hw.ST_DONE, hw.ST_FULL]


def test_chaining_mixed_and_litmus():
    """Mixed Zipf batches with disjoint erase, upsert and query keys and concurrent inserts with queries of the
    same fresh keys: a reported key always carries its own value."""
    cap = 1 << 18
    t = hw.Table(cap, "CHAINING")
    om = oracle.OracleMap()
    uk = w.universe_keys(cap // 2, workload_id=3)
    assert np.array_equal(u8(t.insert(dev(uk), dev(w.value_of(uk)))), om.insert(uk, w.value_of(uk)))
    for b in w.mixed_batches(cap // 2, 1 << 15, 3, workload_id=3):
        ops = b["ops"]
        s, v = t.mixed(torch.from_numpy(ops).cuda(), dev(b["keys"]), dev(b["vals"]), combine="sum")
        s, v = u8(s), host(v)
        os_, ov = om.apply(b["keys"], b["vals"], ops=ops, combine=oracle.SUM)
        det = ops != 2
        assert np.array_equal(s[det], os_[det]) and np.array_equal(v[det], ov[det])
    _check(t, om)
    t2 = hw.Table(1 << 18, "CHAINING")
    fresh = w.distinct_keys(w.stream_seed(133, 1), 1 << 16)
    ops = np.concatenate([np.full(len(fresh), 1), np.full(3 * len(fresh), 0)]).astype(np.uint8)
    keys = np.concatenate([fresh] * 4)
    vals = np.concatenate([w.value_of(fresh), np.zeros(3 * len(fresh), np.uint64)])
    p = w.permutation(w.stream_seed(133, 2), len(ops))
    ops, keys, vals = ops[p], keys[p], vals[p]
    st, out = t2.mixed(torch.from_numpy(ops).cuda(), dev(keys), dev(vals))
    st, out = u8(st), host(out)
    q = ops == 0
    found = st[q] == hw.ST_DONE
    assert (out[q][found] == w.value_of(keys[q][found])).all()
    assert (st[ops == 1] == hw.ST_DONE).all()
    _check(t2)

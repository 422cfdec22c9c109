"""Concurrency tests on the GPU: operations on the same keys and buckets inside
one launch.

* Adversarial benchmark (Section 4.1, Fig. 2) adapted to buckets: every target
  bucket is full and holds X; in one launch X is erased while two operations
  insert Y, whose primary (iceberg: front-yard) bucket is the same bucket and
  whose other candidate bucket has room.  Exactly one copy of Y may result.
* Same-key storm: 2^16 SUM upserts over 16 keys that all share one primary
  bucket (every tile of every wave finds the lock byte held and queues in the
  bucket's ticket queue): the launch ends and every sum is exact.  With
  test-and-set locks alone this case never finished: the waiters' requests
  queued at the lock word delayed every release (the CPU model in
  lock_model.py reproduces it); queued waiters issue no read-modify-write and
  poll rarely, and one tile per queue polls the byte.
* Lock time limit forced from the host: with a 1 us limit, waiters of a storm
  give up with TIMEOUT, the launch ends, and exactly the operations that did
  not time out took effect.
* Publish litmus: in one launch fresh keys are inserted while other tiles query
  them, and present keys are overwritten (REPLACE) while others read them.  A
  reader may miss a key that is being inserted, but whenever it reports a key
  the value must be one that was written with it -- never a half-published slot.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import busy_lock_queues, dev, host, image, u8

pytestmark = pytest.mark.gpu

ODESIGN = {"DOUBLE": oracle.DOUBLE, "DOUBLE_M": oracle.DOUBLE_M, "P2": oracle.P2, "P2_M": oracle.P2_M,
           "ICEBERG": oracle.ICEBERG, "ICEBERG_M": oracle.ICEBERG_M, "CUCKOO": oracle.CUCKOO}
ALL = ["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG", "ICEBERG_M"]
OPQ, OPI, OPU, OPE = 0, 1, 2, 3


def _tags_of(keys):
    t = (keys & np.uint64(0xFFFF)).astype(np.uint32)
    t[t >= 0xFFFE] -= 2
    return t.astype(np.uint16)


def _layout_ok(t):
    slots, tags, locks = image(t)
    nv, rep = oracle.layout_check(ODESIGN[t.design], t.kv_bits, t.num_buckets, t.bucket_slots,
                                  slots, tags, locks)
    assert nv == 0, rep
    assert busy_lock_queues(t) == 0  # every ticket taken was served
    return rep


@pytest.mark.parametrize("design", ALL)
def test_adversarial_erase_vs_duplicate_insert(design):
    t = hw.Table(1 << 16, design)
    nb, B = t.num_buckets, t.bucket_slots
    cand = w.distinct_keys(w.stream_seed(50, ODESIGN[design]), nb * B * 6)
    prim = t.primary_bucket(dev(cand)).cpu().numpy()
    # even buckets are filled; odd ones stay empty (iceberg: even front-yard
    # buckets; the backyard stays empty)
    top = oracle.iceberg_front_buckets(nb) if design.startswith("ICEBERG") else nb
    targets = np.arange(0, top, 2)
    order = np.argsort(prim, kind="stable")
    ps = prim[order]
    slots_img = np.full((nb * B, 2), np.uint64((1 << 64) - 1), dtype=np.uint64)
    X, Y = [], []
    for b in targets:
        lo, hi = np.searchsorted(ps, [b, b + 1])
        ks = cand[order[lo:hi]]
        assert len(ks) >= B + 8, "not enough keys for bucket %d" % b
        resident = ks[:B]
        y = None
        for k in ks[B:]:
            if design.startswith("P2"):
                if oracle.p2_alternate(int(k), nb) % 2 == 1:  # alternate has room
                    y = k
                    break
            else:
                # double hashing: the second bucket on the sequence is b + odd step,
                # an odd, empty bucket; iceberg: the backyard is empty
                y = k
                break
        assert y is not None
        slots_img[b * B: (b + 1) * B, 0] = resident
        slots_img[b * B: (b + 1) * B, 1] = w.value_of(resident)
        X.append(resident[int(b) % B])
        Y.append(y)
    X, Y = np.array(X, np.uint64), np.array(Y, np.uint64)
    live = slots_img[:, 0] != np.uint64((1 << 64) - 1)
    tags_img = None
    if design.endswith("_M"):
        tags_img = np.full(nb * B, 0xFFFF, np.uint16)
        tags_img[live] = _tags_of(slots_img[live, 0])
    raw = t.raw()
    for rnd in range(6):
        raw["slots"].copy_(torch.from_numpy(slots_img.view(np.uint8).reshape(-1)))
        if tags_img is not None:
            raw["tags"].copy_(torch.from_numpy(tags_img.view(np.int16)))
        torch.cuda.synchronize()
        _layout_ok(t)
        ops = np.concatenate([np.full(len(X), OPE), np.full(2 * len(Y), OPI)]).astype(np.uint8)
        keys = np.concatenate([X, Y, Y])
        vals = np.concatenate([np.zeros(len(X), np.uint64), w.value_of(Y), w.value_of(Y)])
        p = w.permutation(w.stream_seed(51, rnd), len(ops))
        ops, keys, vals = ops[p], keys[p], vals[p]
        st, _ = t.mixed(torch.from_numpy(ops).cuda(), dev(keys), dev(vals))
        st = u8(st)
        assert (st[ops == OPE] == hw.ST_DONE).all()
        ins = ops == OPI
        # per Y: one DONE and one EXISTED
        yk = keys[ins]
        ys = st[ins]
        done = np.unique(yk[ys == hw.ST_DONE], return_counts=True)
        assert len(done[0]) == len(Y) and (done[1] == 1).all()
        assert ((ys == hw.ST_DONE) | (ys == hw.ST_EXISTED)).all()
        rep = _layout_ok(t)  # no duplicate key anywhere
        assert rep["live"] == int(live.sum())
        f, v = t.query(dev(np.concatenate([X, Y])))
        f = u8(f)
        assert (f[: len(X)] == hw.ST_MISS).all() and (f[len(X):] == hw.ST_DONE).all()
        assert np.array_equal(host(v)[len(X):], w.value_of(Y))


def _storm(design, bits, n, seed, **kw):
    """A table of 2^14 slots and n SUM upserts over 16 keys sharing one primary
    bucket: (table, keys, values)."""
    t = hw.Table(1 << 14, design, kv_bits=bits, **kw)
    cand = w.distinct_keys(w.stream_seed(seed, ODESIGN[design] + bits), 200000, key_bits=bits)
    prim = t.primary_bucket(dev(cand, bits)).cpu().numpy()
    b0 = np.bincount(prim).argmax()
    keys16 = cand[prim == b0][:16]
    assert len(keys16) == 16
    idx = w.uniform_below(w.stream_seed(seed + 1, bits), 0, n, 16)
    ks = keys16[idx]
    vs = w.splitmix64(w.stream_seed(seed + 2, bits), 0, n)
    if bits == 32:
        vs &= np.uint64(0xFFFFFFFF)
    return t, ks, vs


@pytest.mark.parametrize("design", ["DOUBLE", "DOUBLE_M", "P2", "P2_M"])
@pytest.mark.parametrize("bits", [64, 32])
def test_same_key_storm_one_lock(design, bits):
    # a 2 s lock limit: the FIFO lock needs ~0.3 s for the whole storm
    t, ks, vs = _storm(design, bits, 1 << 16, 52, lock_timeout_us=2000000)
    n = len(ks)
    print("storm %s/%d: %d upserts on one bucket" % (design, bits, n), flush=True)
    st = u8(t.upsert(dev(ks, bits), dev(vs, bits), combine="sum"))
    om = oracle.OracleMap(key_bits=bits)
    ost = om.upsert(ks, vs)
    assert (st == hw.ST_DONE).sum() == 16 and (st == hw.ST_EXISTED).sum() == n - 16
    assert (ost == oracle.DONE).sum() == 16
    k, v = t.export()
    k, v = host(k, bits), host(v, bits)
    o = np.argsort(k)
    ok, ov = om.dump()
    assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)
    _layout_ok(t)


@pytest.mark.parametrize("design", ["DOUBLE_M", "P2_M"])
def test_lock_time_limit_forced_from_the_host(design):
    """A 1 us lock limit set from the host: in a same-bucket storm the waiters
    give up with TIMEOUT instead of waiting their turn, the launch ends, every
    status is DONE, EXISTED or TIMEOUT, and the table holds exactly the sums of
    the operations that did not time out (a timed-out operation has no effect).
    Clearing the table makes it usable again."""
    t, ks, vs = _storm(design, 64, 1 << 14, 61, lock_timeout_us=1)
    st = u8(t.upsert(dev(ks), dev(vs), combine="sum"))
    assert set(np.unique(st).tolist()) <= {hw.ST_DONE, hw.ST_EXISTED, hw.ST_TIMEOUT}
    assert (st == hw.ST_TIMEOUT).sum() > 0
    ok = st != hw.ST_TIMEOUT
    om = oracle.OracleMap()
    ost = om.upsert(ks[ok], vs[ok])
    # one DONE per key that had an applied operation
    assert (st == hw.ST_DONE).sum() == (ost == oracle.DONE).sum()
    k, v = t.export()
    k, v = host(k), host(v)
    o = np.argsort(k)
    okeys, ovals = om.dump()
    assert np.array_equal(k[o], okeys) and np.array_equal(v[o], ovals)
    # the storm's queue now holds abandoned tickets, but no lock byte is left
    # held (a tile holds one only inside its critical section): a lone upsert
    # takes the byte at once.  hwave_clear resets the queues and the flag.
    slots, tags, locks = image(t)
    assert not locks.any()
    assert busy_lock_queues(t) > 0
    one, v1 = dev(ks[:1]), dev(vs[:1])
    present = bool(np.isin(ks[:1], okeys)[0])
    assert u8(t.upsert(one, v1, combine="sum"))[0] == (hw.ST_EXISTED if present else hw.ST_DONE)
    t.clear()
    assert busy_lock_queues(t) == 0
    assert u8(t.upsert(one, v1, combine="sum"))[0] == hw.ST_DONE


@pytest.mark.parametrize("design", ALL)
@pytest.mark.parametrize("bits", [64, 32])
def test_hot_keys_no_erase_table(design, bits):
    """Hot keys on a table that never erases: 2^14 SUM upserts over 16 keys sharing
    one primary bucket.  Present keys are combined without the lock, so only the 16
    first inserts serialise on it; sums and statuses are exact."""
    t = hw.Table(1 << 14, design, kv_bits=bits, flags=hw.F_NO_ERASE)
    cand = w.distinct_keys(w.stream_seed(58, ODESIGN[design] + bits), 200000, key_bits=bits)
    prim = t.primary_bucket(dev(cand, bits)).cpu().numpy()
    b0 = np.bincount(prim).argmax()
    keys16 = cand[prim == b0][:16]
    assert len(keys16) == 16
    n = 1 << 14
    ks = keys16[w.uniform_below(w.stream_seed(59, bits), 0, n, 16)]
    vs = w.splitmix64(w.stream_seed(60, bits), 0, n)
    if bits == 32:
        vs &= np.uint64(0xFFFFFFFF)
    st = u8(t.upsert(dev(ks, bits), dev(vs, bits), combine="sum"))
    om = oracle.OracleMap(key_bits=bits)
    om.upsert(ks, vs)
    assert (st == hw.ST_DONE).sum() == 16 and (st == hw.ST_EXISTED).sum() == n - 16
    k, v = t.export()
    k, v = host(k, bits), host(v, bits)
    o = np.argsort(k)
    ok, ov = om.dump()
    assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)
    _layout_ok(t)


@pytest.mark.parametrize("design", ALL + ["CUCKOO"])
@pytest.mark.parametrize("bits", [64, 32])
def test_publish_litmus_insert_vs_query(design, bits):
    if design == "CUCKOO" and bits == 32:
        pytest.skip("cuckoo tables hold 64-bit keys")
    t = hw.Table(1 << 20, design, kv_bits=bits)
    seed = w.stream_seed(55, ODESIGN[design] * 100 + bits)
    torn = 0
    seen = 0
    for rnd in range(8):
        t.clear()
        fresh = w.distinct_keys(seed, 1 << 18, key_bits=bits, skip=rnd << 18)
        ops = np.concatenate([np.full(len(fresh), OPI), np.full(3 * len(fresh), OPQ)]).astype(np.uint8)
        keys = np.concatenate([fresh, fresh, fresh, fresh])
        vals = np.concatenate([w.value_of(fresh, bits), np.zeros(3 * len(fresh), np.uint64)])
        p = w.permutation(seed + rnd, len(ops))
        ops, keys, vals = ops[p], keys[p], vals[p]
        st, out = t.mixed(torch.from_numpy(ops).cuda(), dev(keys, bits), dev(vals, bits))
        st, out = u8(st), host(out, bits)
        q = ops == OPQ
        found = st[q] == hw.ST_DONE
        seen += int(found.sum())
        torn += int((out[q][found] != w.value_of(keys[q][found], bits)).sum())
        assert (out[q][~found] == 0).all() and (st[q][~found] == hw.ST_MISS).all()
        assert (st[ops == OPI] == hw.ST_DONE).all()
    assert torn == 0, "%d of %d reads saw a key with a value it was never written with" % (torn, seen)
    _layout_ok(t)


@pytest.mark.parametrize("design", ["DOUBLE_M", "P2_M", "DOUBLE", "P2", "ICEBERG_M", "ICEBERG", "CUCKOO"])
def test_publish_litmus_replace_vs_query(design):
    """Present keys overwritten with REPLACE while other tiles read them: every read
    returns the old value or one of the values written in this launch."""
    t = hw.Table(1 << 18, design)
    base = w.distinct_keys(w.stream_seed(56, ODESIGN[design]), 1 << 16)
    t.insert(dev(base), dev(w.value_of(base)))
    bad = 0
    for rnd in range(6):
        cur = w.value_of(base) + np.uint64(10 * rnd)
        a = cur + np.uint64(1)
        b = cur + np.uint64(2)
        ops = np.concatenate([np.full(2 * len(base), OPU), np.full(4 * len(base), OPQ)]).astype(np.uint8)
        keys = np.concatenate([base] * 6)
        vals = np.concatenate([a, b, np.zeros(4 * len(base), np.uint64)])
        p = w.permutation(w.stream_seed(57, rnd), len(ops))
        ops, keys, vals = ops[p], keys[p], vals[p]
        st, out = t.mixed(torch.from_numpy(ops).cuda(), dev(keys), dev(vals), combine="replace")
        st, out = u8(st), host(out)
        q = ops == OPQ
        assert (st[q] == hw.ST_DONE).all()
        c = w.value_of(keys[q]) + np.uint64(10 * rnd)
        ok = (out[q] == c) | (out[q] == c + np.uint64(1)) | (out[q] == c + np.uint64(2))
        bad += int((~ok).sum())
        # settle to a known value for the next round
        t.upsert(dev(base), dev(w.value_of(base) + np.uint64(10 * (rnd + 1))), combine="replace")
    assert bad == 0
    _layout_ok(t)


@pytest.mark.parametrize("design,cap", [("P2_M", 1 << 16), ("DOUBLE", 1 << 26)])
def test_lock_byte_at_its_stride_holds_off_writers(design, cap):
    """The lock array's layout, pinned from the host: bucket b's lock is byte
    b * lock_stride, stride = clamp(2^23 / buckets, 1, 8) (8 for the small table,
    1 for 2^23 buckets).  With that byte set from the host, the writers of bucket
    b wait, reach the table's 1 ms limit and report TIMEOUT without effect, while
    keys of other buckets (one per bucket, so none waits) insert.  Clearing the
    table frees the lock again."""
    t = hw.Table(cap, design, lock_timeout_us=1000)
    r = t.raw()
    stride = r["lock_stride"]
    assert stride == max(1, min(8, (1 << 23) // t.num_buckets))
    cand = w.distinct_keys(w.stream_seed(90, ODESIGN[design]), 4096)
    prim = t.primary_bucket(dev(cand)).cpu().numpy()
    b = int(np.bincount(prim).argmax())
    on_b = cand[prim == b][:8]
    _, first = np.unique(prim, return_index=True)
    others = np.array([cand[i] for i in first if prim[i] != b][:56], dtype=np.uint64)
    keys = np.concatenate([on_b, others])
    vals = w.value_of(keys)
    r["locks"].view(torch.uint8)[b * stride] = 1  # bucket b's lock, held by nobody
    st = u8(t.upsert(dev(keys), dev(vals), combine="sum"))
    assert (st[: len(on_b)] == hw.ST_TIMEOUT).all()
    assert (st[len(on_b):] == hw.ST_DONE).all()
    f, _ = t.query(dev(on_b))
    assert (u8(f) == hw.ST_MISS).all()  # timed-out writes had no effect
    t.clear()
    assert (u8(t.upsert(dev(keys), dev(vals), combine="sum")) == hw.ST_DONE).all()

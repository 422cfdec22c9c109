"""The served form: requests of uneven sizes arriving over time are batched
continuously into multi-table launches; every request's outputs must equal a
one-at-a-time replay in submission order (plain mode) and the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w

pytestmark = pytest.mark.gpu

OPQ = hw.OPS["query"]
OPI = hw.OPS["insert"]
OPU = hw.OPS["upsert"] | (hw.COMBINES["sum"] << 8)


def _host(a, bits=64, pinned=True):
    a = np.ascontiguousarray(a, np.uint64)
    t = torch.from_numpy(a.view(np.int64).copy() if bits == 64 else a.astype(np.uint32).view(np.int32).copy())
    return t.pin_memory() if pinned else t


def _pinned(a):
    return _host(a)


def _make_requests(n_tables, universe, n_req, seed, bits=64):
    """Zipf keys per table; op kinds query/upsert/insert 50/30/20; sizes 2^U, U ~ U[3, 11];
    insert values 3k+1 so duplicate inserts are deterministic."""
    uk = [w.distinct_keys(w.stream_seed(seed, 100 + t), universe, key_bits=bits) for t in range(n_tables)]
    z = w.Zipf(universe, 0.99)
    u = w.unit_float(w.stream_seed(seed, 1), 0, 3 * n_req)
    reqs = []
    zpos = 0
    for i in range(n_req):
        t = int(u[3 * i] * n_tables)
        r = u[3 * i + 1]
        op = OPQ if r < 0.5 else (OPU if r < 0.8 else OPI)
        n = int(2 ** (3 + 8 * u[3 * i + 2]))
        ranks = z.ranks(w.stream_seed(seed, 2), zpos, n)
        zpos += n
        keys = uk[t][ranks]
        if op == OPI:
            vals = w.value_of(keys, bits)
        elif op == OPU:
            vals = w.splitmix64(w.stream_seed(seed, 3), zpos, n)
            if bits == 32:
                vals &= np.uint64(0xFFFFFFFF)
        else:
            vals = None
        reqs.append((t, op, keys, vals))
    return uk, reqs


def _serve(tables, reqs, mode, gap_s, bits=64, pageable_every=0):
    """Serves reqs; with pageable_every = k, every k-th request's arrays are
    ordinary (pageable) host memory, which the server copies with runtime copies."""
    srv = hw.Server(tables, mode=mode, slots=3, slot_ops=1 << 16)
    bufs, rs = [], []
    dt = torch.int64 if bits == 64 else torch.int32
    for i, (t, op, keys, vals) in enumerate(reqs):
        pin = not (pageable_every and i % pageable_every == 0)
        kt = _host(keys, bits, pin)
        vt = None if vals is None else _host(vals, bits, pin)
        out = torch.zeros(len(keys), dtype=dt)
        st = torch.zeros(len(keys), dtype=torch.uint8)
        if pin:
            out, st = out.pin_memory(), st.pin_memory()
        bufs.append((kt, vt, out, st))
        rs.append(hw.Server.request(t, op, kt, vt, out, st))
    offs = np.arange(len(reqs)) * gap_s
    srv.replay(rs, offs)
    srv.drain()
    stats = srv.stats()
    srv.close()
    res = []
    for b in bufs:
        o = b[2].numpy()
        res.append((o.view(np.uint64).copy() if bits == 64 else o.view(np.uint32).astype(np.uint64), b[3].numpy().copy()))
    return res, stats


def _counts(keys, st, code):
    u, c = np.unique(keys[st == code], return_counts=True)
    return dict(zip(u.tolist(), c.tolist()))


@pytest.mark.parametrize("design", ["P2_M", "DOUBLE_M"])
def test_served_results_equal_serial_replay_and_oracle(design):
    n_tables, universe = 8, 1 << 14
    uk, reqs = _make_requests(n_tables, universe, 600, seed=61)
    A = [hw.Table(1 << 16, design) for _ in range(n_tables)]
    B = [hw.Table(1 << 16, design) for _ in range(n_tables)]
    oms = [oracle.OracleMap() for _ in range(n_tables)]
    for t in range(n_tables):  # preload half of each universe
        pre = uk[t][: universe // 2]
        kk = torch.from_numpy(pre.view(np.int64).copy()).cuda()
        vv = torch.from_numpy(w.value_of(pre).view(np.int64).copy()).cuda()
        A[t].insert(kk, vv)
        B[t].insert(kk, vv)
        oms[t].insert(pre, w.value_of(pre))
    torch.cuda.synchronize()
    served, st_a = _serve(A, reqs, "batched", 20e-6)
    plain, st_b = _serve(B, reqs, "plain", 20e-6)
    assert st_a["requests"] == st_b["requests"] == len(reqs)
    assert st_a["mean_requests_per_batch"] > 1.0  # batching really happened
    for i, (t, op, keys, vals) in enumerate(reqs):
        out_a, s_a = served[i]
        out_b, s_b = plain[i]
        if op == OPQ:
            os_, ov = oms[t].query(keys)
            assert np.array_equal(s_a, os_) and np.array_equal(out_a, ov), i
            assert np.array_equal(s_b, os_) and np.array_equal(out_b, ov), i
        else:
            os_ = oms[t].apply(keys, vals, default_op=hw.OPS["insert"] if op == OPI else hw.OPS["upsert"],
                               combine=oracle.SUM)[0]
            for code in (1, 2):
                assert _counts(keys, s_a, code) == _counts(keys, os_, code), i
                assert _counts(keys, s_b, code) == _counts(keys, os_, code), i
    for t in range(n_tables):
        ok, ov = oms[t].dump()
        for tab in (A[t], B[t]):
            k, v = tab.export()
            k = k.cpu().numpy().view(np.uint64)
            v = v.cpu().numpy().view(np.uint64)
            o = np.argsort(k)
            assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)


@pytest.mark.parametrize("bits,design,flags,pageable_every", [
    (64, "P2_M", hw.F_NO_ERASE | hw.F_AGGREGATE, 0),   # the served benchmark's tables
    (64, "DOUBLE_M", hw.F_NO_ERASE | hw.F_AGGREGATE, 5),
    (64, "P2_M", 0, 3),
    (32, "P2_M", 0, 4),
])
def test_served_copy_paths_and_table_kinds(bits, design, flags, pageable_every):
    """Batched serving with pinned requests (gathered and scattered by the copy
    kernels) mixed with pageable ones (runtime copies), on merging erase-free
    tables (hot-key accumulators) and on 32-bit tables: every output and every
    table equal the oracle's."""
    n_tables, universe = 6, 1 << 13
    uk, reqs = _make_requests(n_tables, universe, 300, seed=62 + bits, bits=bits)
    A = [hw.Table(1 << 15, design, kv_bits=bits, flags=flags) for _ in range(n_tables)]
    oms = [oracle.OracleMap(key_bits=bits) for _ in range(n_tables)]
    for t in range(n_tables):
        pre = uk[t][: universe // 2]
        pv = w.value_of(pre, bits)
        A[t].insert(_host(pre, bits, False).cuda(), _host(pv, bits, False).cuda())
        oms[t].insert(pre, pv)
    torch.cuda.synchronize()
    served, st_a = _serve(A, reqs, "batched", 20e-6, bits=bits, pageable_every=pageable_every)
    assert st_a["requests"] == len(reqs)
    n_pageable = len(range(0, len(reqs), pageable_every)) if pageable_every else 0
    assert st_a["runtime_copied"] == n_pageable
    for i, (t, op, keys, vals) in enumerate(reqs):
        out_a, s_a = served[i]
        if op == OPQ:
            os_, ov = oms[t].query(keys)
            assert np.array_equal(s_a, os_) and np.array_equal(out_a, ov), i
        else:
            os_ = oms[t].apply(keys, vals, default_op=hw.OPS["insert"] if op == OPI else hw.OPS["upsert"],
                               combine=oracle.SUM)[0]
            for code in (1, 2):
                assert _counts(keys, s_a, code) == _counts(keys, os_, code), i
    for t in range(n_tables):
        ok, ov = oms[t].dump()
        k, v = A[t].export()
        k = k.cpu().numpy().view(np.uint64) if bits == 64 else k.cpu().numpy().view(np.uint32).astype(np.uint64)
        v = v.cpu().numpy().view(np.uint64) if bits == 64 else v.cpu().numpy().view(np.uint32).astype(np.uint64)
        o = np.argsort(k)
        assert np.array_equal(k[o], ok) and np.array_equal(v[o], ov)


def test_served_unaligned_pinned_arrays():
    """Request arrays that are views at odd offsets into pinned buffers (keys 8
    bytes past a 16-byte boundary, statuses at byte offsets 1..7): the batch copy
    kernels fall back to word and byte copies, and every output equals the
    oracle's."""
    n_tables, universe = 4, 1 << 12
    uk, reqs = _make_requests(n_tables, universe, 120, seed=71)
    A = [hw.Table(1 << 14, "P2_M") for _ in range(n_tables)]
    oms = [oracle.OracleMap() for _ in range(n_tables)]
    for t in range(n_tables):
        pre = uk[t][: universe // 2]
        A[t].insert(_host(pre, 64, False).cuda(), _host(w.value_of(pre), 64, False).cuda())
        oms[t].insert(pre, w.value_of(pre))
    torch.cuda.synchronize()
    total = sum(len(r[2]) for r in reqs)
    kbuf = torch.zeros(total + 2 * len(reqs), dtype=torch.int64).pin_memory()
    vbuf = torch.zeros(total + 2 * len(reqs), dtype=torch.int64).pin_memory()
    obuf = torch.zeros(total + 2 * len(reqs), dtype=torch.int64).pin_memory()
    sbuf = torch.zeros(total + 8 * len(reqs), dtype=torch.uint8).pin_memory()
    srv = hw.Server(A, mode="batched", slots=3, slot_ops=1 << 16)
    rs, views = [], []
    ka = sa = 0
    for i, (t, op, keys, vals) in enumerate(reqs):
        n = len(keys)
        ka += 1  # 8 bytes past the previous array's end
        sa += 1 + i % 7
        k = kbuf[ka: ka + n]
        k.copy_(torch.from_numpy(keys.view(np.int64)))
        v = None
        if vals is not None:
            v = vbuf[ka: ka + n]
            v.copy_(torch.from_numpy(vals.view(np.int64)))
        o = obuf[ka: ka + n]
        s = sbuf[sa: sa + n]
        views.append((o, s))
        rs.append(hw.Server.request(t, op, k, v, o, s))
        ka += n
        sa += n
    srv.replay(rs, np.arange(len(reqs)) * 20e-6)
    srv.drain()
    assert srv.stats()["runtime_copied"] == 0  # every request went through the copy kernels
    srv.close()
    for i, (t, op, keys, vals) in enumerate(reqs):
        o, s = views[i][0].numpy().view(np.uint64), views[i][1].numpy()
        if op == OPQ:
            os_, ov = oms[t].query(keys)
            assert np.array_equal(s, os_) and np.array_equal(o, ov), i
        else:
            os_ = oms[t].apply(keys, vals, default_op=hw.OPS["insert"] if op == OPI else hw.OPS["upsert"],
                               combine=oracle.SUM)[0]
            for code in (1, 2):
                assert _counts(keys, s, code) == _counts(keys, os_, code), i

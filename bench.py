#!/usr/bin/env python3
"""HashWave benchmark: the load benchmark of the paper (Section 6.3) at 2^28 slots on
one MI355X, on the power-of-two-choice table with 16-bit tags.

One step = one pass of the whole hot path over one synthetic batch set:
  clear; insert distinct uniform keys to load 0.5, 0.75, 0.9 (v = 3k+1);
  2^27 positive and 2^27 negative queries; 2^27 SUM upserts on present keys;
  erase a seeded 50% of the keys; re-query the positive and negative sets;
  16 mixed batches of 2^20 ops (50% query / 30% SUM upsert / 20% erase, Zipf 0.99
  over the inserted keys).
The same step is then run, verified and timed on the other designs (double
hashing, power-of-two-choice and iceberg, with and without tags, chaining and
cuckoo hashing) for comparison,
followed by the aging (churn) benchmark of Section 6.5 on every design.
Inputs are resident in HBM before timing.  `value` = all operations of K steps /
wall time of K steps.  Per-kernel durations come from HIP events on the stream
the kernels run on; p50/p99 batch latency is over the mixed 2^20-op batches.

Prints ONE JSON line (see the `result` dict at the end).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gops/s insert/query/upsert at 0.9 load (2^28 slots); p50/p99 batch latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per operation (64-byte sectors of tag and slot data, plus the
# op's own input/output bytes) for the tagged power-of-two-choice table at 0.9
# load: probed lines from Table 1's probe counts, in 64-byte sectors, plus key,
# value and status bytes of the op batch.
ALGO_BYTES = {
    "insert": 273.0, "query_pos": 153.0, "query_neg": 137.0, "upsert": 222.0,
    "erase": 278.0, "requery_pos": 145.0, "requery_neg": 137.0, "mixed": 180.0,
}

SOURCES_FOR_TRAFFIC = ["paper_2509_16407_amd/csrc/hw_device.hpp", "paper_2509_16407_amd/csrc/hw_ops.hpp",
                       "paper_2509_16407_amd/csrc/hw_launch.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in SOURCES_FOR_TRAFFIC:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(cap_log2: int, n_mixed: int, mixed_batch: int):
    from paper_2509_16407_amd import workloads as w
    cap = 1 << cap_log2
    keys, bounds = w.load_phases(cap, (0.5, 0.75, 0.9), workload_id=2)
    n = bounds[-1]
    nq = min(1 << (cap_log2 - 1), n)  # 2^27 positive and 2^27 negative queries at 2^28
    pos_idx = w.sample_without_replacement(w.stream_seed(2, 3), n, nq)
    qpos = keys[pos_idx]
    qneg = w.distinct_keys(w.stream_seed(2, 1), nq, skip=n)
    er_idx = w.sample_without_replacement(w.stream_seed(2, 4), n, n // 2)
    ekeys = keys[er_idx]
    mixed = []
    if n_mixed:
        for b in w.mixed_batches(n, mixed_batch, n_mixed, workload_id=2, ukeys=keys):
            mixed.append(b)
    return dict(cap=cap, keys=keys, bounds=bounds, qpos=qpos, qneg=qneg, ekeys=ekeys,
                pos_idx=pos_idx, er_idx=er_idx, mixed=mixed)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64)).cuda()


class Step:
    """Device-resident inputs and the kernel sequence of one step."""

    def __init__(self, d, design: str, tile: int, bucket: int):
        import torch
        import paper_2509_16407_amd as hw
        from paper_2509_16407_amd import workloads as w
        # the step's mixed batches put Zipf-hot keys among their upserts: merged by key
        # (HWAVE_F_MERGE_MIXED; bulk calls are unaffected by the flag)
        self.t = hw.Table(d["cap"], design, bucket=bucket, tile=tile, flags=hw.F_MERGE_MIXED)
        self.keys = to_dev(d["keys"])
        self.vals = to_dev(w.value_of(d["keys"]))
        self.bounds = d["bounds"]
        self.qpos = to_dev(d["qpos"])
        self.qneg = to_dev(d["qneg"])
        self.ones = torch.ones(len(d["qpos"]), dtype=torch.int64, device="cuda")
        self.ekeys = to_dev(d["ekeys"])
        nmax = max(len(d["qpos"]), len(d["ekeys"]), len(d["keys"]))
        self.st = torch.empty(nmax, dtype=torch.uint8, device="cuda")
        self.out = torch.empty(len(d["qpos"]), dtype=torch.int64, device="cuda")
        self.mixed = [(torch.from_numpy(b["ops"]).cuda(), to_dev(b["keys"]), to_dev(b["vals"]))
                      for b in d["mixed"]]
        if self.mixed:
            mb = len(d["mixed"][0]["keys"])
            self.mst = torch.empty(mb, dtype=torch.uint8, device="cuda")
            self.mout = torch.empty(mb, dtype=torch.int64, device="cuda")
        self.phase_names = ["insert_0.5", "insert_0.75", "insert_0.9", "query_pos", "query_neg",
                            "upsert", "erase", "requery_pos", "requery_neg"]
        self.ops = {
            "insert_0.5": self.bounds[0], "insert_0.75": self.bounds[1] - self.bounds[0],
            "insert_0.9": self.bounds[2] - self.bounds[1], "query_pos": len(d["qpos"]),
            "query_neg": len(d["qneg"]), "upsert": len(d["qpos"]), "erase": len(d["ekeys"]),
            "requery_pos": len(d["qpos"]), "requery_neg": len(d["qneg"]),
        }
        self.mixed_ops = sum(len(b["keys"]) for b in d["mixed"])

    def ops_per_step(self):
        return sum(self.ops.values()) + self.mixed_ops

    def run(self, events=None):
        """Enqueue one step; if `events` is a dict, record (start, end) per phase."""
        import torch
        t = self.t
        rec = events is not None

        def phase(name, fn):
            if rec:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                events.setdefault(name, []).append((a, b))
            else:
                fn()

        t.clear()
        b0, b1, b2 = self.bounds
        phase("insert_0.5", lambda: t.insert(self.keys[:b0], self.vals[:b0], status=self.st[:b0]))
        phase("insert_0.75", lambda: t.insert(self.keys[b0:b1], self.vals[b0:b1], status=self.st[:b1 - b0]))
        phase("insert_0.9", lambda: t.insert(self.keys[b1:b2], self.vals[b1:b2], status=self.st[:b2 - b1]))
        nq = self.qpos.numel()
        phase("query_pos", lambda: t.query(self.qpos, out=self.out, found=self.st[:nq]))
        phase("query_neg", lambda: t.query(self.qneg, out=self.out, found=self.st[:nq]))
        phase("upsert", lambda: t.upsert(self.qpos, self.ones, combine="sum", status=self.st[:nq]))
        ne = self.ekeys.numel()
        phase("erase", lambda: t.erase(self.ekeys, found=self.st[:ne]))
        phase("requery_pos", lambda: t.query(self.qpos, out=self.out, found=self.st[:nq]))
        phase("requery_neg", lambda: t.query(self.qneg, out=self.out, found=self.st[:nq]))
        for i, (o, k, v) in enumerate(self.mixed):
            phase("mixed", lambda o=o, k=k, v=v: t.mixed(o, k, v, combine="sum", out=self.mout,
                                                         status=self.mst))


def probe_counts(step: Step, design: str) -> dict:
    """Lines per query measured by the GPU (Table 1's probe unit, Section 5.1): an
    instrumented table of the step's size filled to 0.9, then the step's positive
    and negative query sets, counted by the kernels themselves
    (hwave_probe_counters).  Not part of the timed step."""
    import torch
    import paper_2509_16407_amd as hw
    t = hw.Table(step.t.capacity, design, bucket=step.t.bucket_slots, tile=step.t.tile, instrumented=True)
    b2 = step.bounds[-1]
    st = t.insert(step.keys[:b2], step.vals[:b2])
    n_full = int((st == 3).sum().item())
    t.probe_counters(reset=True)
    f, _ = t.query(step.qpos, out=step.out, found=step.st[: len(step.qpos)])
    found = int((f == 1).sum().item())
    pos = t.probe_counters(reset=True)
    t.query(step.qneg, out=step.out, found=step.st[: len(step.qneg)])
    neg = t.probe_counters(reset=True)
    del t
    torch.cuda.empty_cache()
    per = lambda c: round((c["bucket_lines"] + c["slot_lines"]) / max(1, c["queries"]), 4)
    return {"design": design, "load": 0.9, "positive_lines_per_query": per(pos),
            "negative_lines_per_query": per(neg), "positive_found": found, "full_inserts": n_full,
            "counters": {"positive": pos, "negative": neg}}


def upsert_miss(step: Step, reps: int = 3) -> dict:
    """The upsert-miss path (not part of the step): fill a cleared table to 0.75,
    then time the 0.75 -> 0.9 keys as SUM upserts, which all insert.  Median of
    `reps` runs after one untimed run."""
    import torch
    t = step.t
    _, b1, b2 = step.bounds
    ms = []
    for r in range(reps + 1):
        t.clear()
        t.insert(step.keys[:b1], step.vals[:b1])
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        st = t.upsert(step.keys[b1:b2], step.vals[b1:b2], combine="sum", status=step.st[: b2 - b1])
        b.record()
        b.synchronize()
        full = full_inserts_legal(t, step.keys[b1:b2], st)
        assert int((st == 1).sum().item()) + full == b2 - b1, "upsert-miss statuses"
        if r:
            ms.append(a.elapsed_time(b))
    m = float(np.median(ms))
    return {"ms": round(m, 4), "gops": round((b2 - b1) / m / 1e6, 3)}


def full_inserts_legal(t, keys, st) -> int:
    """Checks every FULL status of an insert-only batch against the table image:
    a key may end FULL only when every bucket it may occupy is full (Section
    2.2: a two-choice insert fails only when both of its buckets are full; for
    iceberg, its front bucket and both backyard choices; for double hashing and
    chaining, when no slot is left).  Inserts only add keys, so a bucket full
    when the key was refused is still full in the final image.  The buckets come
    from the library's hwave_candidate_buckets hook, the image from hwave_raw.
    Returns the number of FULL keys; raises AssertionError on an illegal one."""
    import torch
    full = (st == 3).nonzero().flatten()
    nf = int(full.numel())
    if nf == 0:
        return 0
    if t.design in ("DOUBLE", "DOUBLE_M", "CHAINING"):
        assert t.size() == t.capacity, "FULL while the table has free slots"
        return nf
    cand = t.candidate_buckets(keys[full])
    ncand = 3 if t.design.startswith("ICEBERG") or t.design == "CUCKOO" else 2
    b = cand[:, :ncand].reshape(-1)
    B = t.bucket_slots
    raw = t.raw()["slots"]
    kw = raw.view(torch.int64 if t.kv_bits == 64 else torch.int32).view(-1, 2)[:, 0]
    idx = (b[:, None] * B + torch.arange(B, device=b.device)[None, :]).reshape(-1)
    k = kw[idx]
    # the empty, tombstone and reservation patterns are -1, -2, -3 as signed words
    live = (k < -3) | (k >= 0)
    ok = live.view(-1, B).all(dim=1)
    assert bool(ok.all()), "a FULL key has a candidate bucket with a free slot"
    return nf


def verify_step(step: Step, d) -> int:
    """Closed-form checks of one full step at full size (no oracle needed):
    every insert DONE, or FULL when full_inserts_legal() confirms that all of the
    key's buckets are full (concurrent two-choice placement decides on bucket
    fills that other inserts are changing, so at 0.9 load a key can, rarely,
    find both of its 32-slot buckets full); positives return 3k+1 (3k+2 after
    the +1 upsert), negatives miss, erased keys miss, kept keys found, table size
    equals inserted - erased.  A FULL key counts as never inserted throughout:
    its queries miss, its upsert is FULL again (no erase has freed a slot), its
    erase misses.  Returns the number of FULL keys."""
    import torch
    from paper_2509_16407_amd import workloads as w
    t = step.t
    t.clear()
    b2 = step.bounds[-1]
    st = t.insert(step.keys, step.vals, status=step.st[:b2])
    if not bool(((st == 1) | (st == 3)).all()):
        hist = {int(c): int(n) for c, n in zip(*np.unique(st.cpu().numpy(), return_counts=True))}
        raise AssertionError("insert statuses %s (1 done, 2 existed, 3 full, 5 timeout)" % hist)
    n_full = full_inserts_legal(t, step.keys, st)
    isfull = st == 3
    pos_full = isfull[torch.from_numpy(d["pos_idx"]).cuda()]
    er_full = isfull[torch.from_numpy(d["er_idx"]).cuda()]
    n_er_full = int(er_full.sum().item())
    exp = to_dev(w.value_of(d["qpos"]))
    zero = torch.zeros_like(exp)
    f, v = t.query(step.qpos, out=step.out)
    assert bool((f == torch.where(pos_full, 0, 1).to(f.dtype)).all()), "positive queries"
    assert bool((v == torch.where(pos_full, zero, exp)).all()), "positive values"
    f, v = t.query(step.qneg, out=step.out)
    assert bool((f == 0).all()) and bool((v == 0).all()), "negative queries"
    st = t.upsert(step.qpos, step.ones, combine="sum")
    assert bool((st == torch.where(pos_full, 3, 2).to(st.dtype)).all()), "upsert statuses"
    f, v = t.query(step.qpos, out=step.out)
    assert bool((v == torch.where(pos_full, zero, exp + 1)).all()), "upserted values"
    st = t.erase(step.ekeys)
    assert bool((st == torch.where(er_full, 0, 1).to(st.dtype)).all()), "erase statuses"
    assert t.size() == b2 - n_full - (len(d["ekeys"]) - n_er_full), "size after erase"
    erased = np.zeros(b2, dtype=bool)
    erased[d["er_idx"]] = True
    kept_mask = torch.from_numpy(~erased[d["pos_idx"]]).cuda() & ~pos_full
    f, v = t.query(step.qpos, out=step.out)
    assert bool(((f == 1) == kept_mask).all()), "re-query membership"
    assert bool(torch.where(kept_mask, v == exp + 1, v == 0).all()), "re-query values"
    torch.cuda.synchronize()
    del exp, zero
    return n_full


def bench_phased(step: Step, d, design: str, conc_rates: dict, reps=3):
    """Cost of concurrency (Section 6.4): the load phases and the query sets on the
    phased variant of `design` (no locks, plain cacheable loads in queries; chaining
    and cuckoo keep their write locks, so only their queries differ), against
    the same phases of the concurrent table.  Outputs of the first repetition are
    checked by closed form.  Without locks, inserts deciding at once on the same
    bucket pair can crowd it, so a two-choice key may end FULL; such keys are
    counted and excluded from the positive-query check."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    # chaining sized as in the concurrent comparison (7 pairs per chain at the end)
    t = hw.Table(step.bounds[-1] if design == "CHAINING" else d["cap"], design, flags=hw.F_BSP)
    b0, b1, b2 = step.bounds
    nq = step.qpos.numel()
    st_all = torch.empty(b2, dtype=torch.uint8, device="cuda")
    ms = {}

    def timed(name, fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        ms.setdefault(name, []).append((a, b))

    n_full = 0
    for r in range(reps + 1):
        t.clear()
        timed("insert_0.5", lambda: t.insert(step.keys[:b0], step.vals[:b0], status=st_all[:b0]))
        timed("insert_0.75", lambda: t.insert(step.keys[b0:b1], step.vals[b0:b1], status=st_all[b0:b1]))
        timed("insert_0.9", lambda: t.insert(step.keys[b1:b2], step.vals[b1:b2], status=st_all[b1:b2]))
        if r == 0:
            full = st_all == 3
            n_full = full_inserts_legal(t, step.keys, st_all)
            assert bool(((st_all == 1) | full).all()), "phased %s: insert statuses" % design
            assert t.size() == b2 - n_full, "phased %s: size after the load phases" % design
            kept = ~full[torch.from_numpy(d["pos_idx"]).cuda()]
        timed("query_pos", lambda: t.query(step.qpos, out=step.out, found=step.st[:nq]))
        if r == 0:
            exp = to_dev(w.value_of(d["qpos"]))
            assert bool(((step.st[:nq] == 1) == kept).all()), "phased %s: positive flags" % design
            assert bool(torch.where(kept, step.out == exp, step.out == 0).all()), "phased %s: values" % design
            del exp, kept
        timed("query_neg", lambda: t.query(step.qneg, out=step.out, found=step.st[:nq]))
        if r == 0:
            assert bool((step.st[:nq] == 0).all()), "phased %s: negatives" % design
    torch.cuda.synchronize()
    res = {"full_inserts": n_full}
    for name, ev in ms.items():
        m = float(np.mean([a.elapsed_time(b) for a, b in ev[1:]]))
        g = step.ops[name] / m / 1e6
        res[name] = {"gops": round(g, 3), "concurrent_gops": conc_rates[name],
                     "overhead_pct": round(100.0 * (g - conc_rates[name]) / g, 2)}
    del t, st_all
    torch.cuda.empty_cache()
    return res


def bench_designs(step: Step, d, designs, steps=2, warmup=1, verify=True):
    """The same step on other table designs at the same size and inputs (the paper's
    load benchmark compares designs, Section 6.3): per design, closed-form
    verification at full size, then per-phase rates over `steps` timed steps."""
    import torch
    import paper_2509_16407_amd as hw
    main_t = step.t
    out = {}
    for des in designs:
        # chaining is sized, as in the paper's evaluation (Section 5), so that its
        # chains hold 7 pairs (length 1) in expectation once the step has loaded
        # all its keys
        step.t = hw.Table(step.bounds[-1] if des == "CHAINING" else d["cap"], des, flags=hw.F_MERGE_MIXED)
        if verify:
            res_full = verify_step(step, d)
            if res_full:
                log("design %s: %d insert(s) ended FULL, each with all of its buckets full" % (des, res_full))
        for _ in range(warmup):
            step.run()
        events = {}
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(steps):
            step.run(events)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ph = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in events.items()}
        rates = {n: round(step.ops[n] / ph[n] / 1e6, 3) for n in step.phase_names}
        if "mixed" in ph:
            rates["mixed"] = round(step.mixed_ops / len(step.mixed) / ph["mixed"] / 1e6, 3)
        out[des] = {"bucket": step.t.bucket_slots, "tile": step.t.tile, "verified": bool(verify),
                    "step_gops": round(step.ops_per_step() * steps / wall / 1e9, 4), "phase_gops": rates}
        step.t = None
        torch.cuda.empty_cache()
        out[des]["phased"] = bench_phased(step, d, des, rates)
        log("design %s: %.2f Gops/s per step (insert_0.9 %.2f, query+ %.2f, query- %.2f)"
            % (des, out[des]["step_gops"], rates["insert_0.9"], rates["query_pos"], rates["query_neg"]))
    step.t = main_t
    return out


# Table 1's aged positive / negative query probes (A40), for context beside the
# GPU-counted ones
PAPER_AGED_PROBES = {"DOUBLE": (1.61, 80.00), "DOUBLE_M": (2.10, 19.39), "P2": (3.96, 8.01),
                     "P2_M": (2.42, 2.01), "ICEBERG": (3.12, 12.02), "ICEBERG_M": (2.2, 3.02),
                     "CHAINING": (1.2, 2.06)}


# Table 1's load query probes at 0.9 (A40)
# Table 1, "Average load probes", columns Insert and Delete (paper, A40).
PAPER_WRITE_PROBES = {"DOUBLE": (5.44, 4.22), "DOUBLE_M": (5.12, 6.07), "P2": (6.34, 5.83), "P2_M": (5.25, 6.15),
                      "ICEBERG": (6.53, 5.97), "ICEBERG_M": (5.24, 6.19)}
PAPER_LOAD_PROBES = {"DOUBLE": 1.22, "DOUBLE_M": 2.05, "P2": 2.83, "P2_M": 2.13, "ICEBERG": 2.97,
                     "ICEBERG_M": 2.16, "CHAINING": 1.16}


def load_probes(designs, log2cap=22):
    """Positive-query probes at 0.9 load counted by the GPU (instrumented build):
    2^log2cap slots (chaining: sized for its keys, 7 pairs per chain), filled with
    floor(0.9 * 2^log2cap) distinct keys, every key queried once."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    n = int(0.9 * (1 << log2cap))
    keys = to_dev(w.distinct_keys(w.stream_seed(2, 40), n))
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    res = {}
    for des in designs:
        t = hw.Table(n if des == "CHAINING" else 1 << log2cap, des, instrumented=True)
        t.probe_counters(reset=True)
        # nine insert batches (0.1 load each), the same fill as one
        ins = torch.cat([t.insert(part, part * 3 + 1) for part in torch.tensor_split(keys, 9)])
        wc = t.probe_counters(reset=True)
        ok = ins == 1
        f, _ = t.query(keys, out=out, found=st)
        assert bool((f == ok.to(torch.uint8)).all()), "load probes %s: queries" % des
        c = t.probe_counters(reset=True)
        pos = (c["bucket_lines"] + c["slot_lines"]) / max(1, c["queries"])
        r = {"positive": round(pos, 3), "full_inserts": int((~ok).sum().item()),
             "paper_a40": PAPER_LOAD_PROBES.get(des)}
        if des in PAPER_WRITE_PROBES:
            # Table 1's delete column as accesses: the search (a positive query),
            # the lock's acquire and release, and the removal's writes (the key;
            # with tags the tag too)
            r["delete_model"] = round(pos + 2 + (2 if des.endswith("_M") else 1), 3)
            r["paper_a40_delete"] = PAPER_WRITE_PROBES[des][1]
        if des.endswith("_M") and wc["writes"]:
            # and its insert column: one tag line per bucket visited, the lock's
            # two accesses, the claim and the publish
            visits = wc["write_visits"] / wc["writes"]
            r["insert_visits"] = round(visits, 4)
            r["insert_model"] = round(visits + 4, 3)
            r["paper_a40_insert"] = PAPER_WRITE_PROBES[des][0]
        res[des] = r
        del t
        torch.cuda.empty_cache()
    log("load probes at 0.9 (GPU-counted, 2^%d slots): %s" % (log2cap, ", ".join(
        "%s %.2f (Table 1: %s)" % (d, r["positive"], r["paper_a40"]) for d, r in res.items())))
    log("insert/delete probes as accesses (GPU-counted search + lock + writes): %s" % ", ".join(
        "%s %s/%s (Table 1: %s/%s)" % (d, r.get("insert_model", "-"), r.get("delete_model", "-"),
                                       r.get("paper_a40_insert", "-"), r.get("paper_a40_delete", "-"))
        for d, r in res.items() if "delete_model" in r))
    return res


def aging_probes(designs, log2cap=22, iters=1000, probe_cap_lines=80):
    """Query probes of aged tables counted by the GPU (instrumented build): the
    aging recipe of bench_aging at 2^log2cap slots, then one more iteration's
    live and absent query sets, counted separately.  Cuckoo queries are not
    counted by the instrumented build."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    plan = w.aging_plan(1 << log2cap, iters=iters + 1, workload_id=6)
    n0, s = plan["n0"], plan["s"]
    kd = to_dev(plan["keys"])
    nd = to_dev(plan["negs"])
    ops = torch.cat([torch.full((s,), 1, dtype=torch.uint8), torch.full((s,), 3, dtype=torch.uint8),
                     torch.zeros(2 * s, dtype=torch.uint8)]).cuda()
    kb = torch.empty(4 * s, dtype=torch.int64, device="cuda")
    out = torch.empty(4 * s, dtype=torch.int64, device="cuda")
    st = torch.empty(4 * s, dtype=torch.uint8, device="cuda")
    res = {}
    for des in designs:
        cap = 0
        if des.startswith("DOUBLE"):
            cap = probe_cap_lines * 8 // (8 if des == "DOUBLE" else 32)
        t = hw.Table(1 << log2cap, des, probe_cap=cap, instrumented=True)
        t.insert(kd[:n0], kd[:n0] * 3 + 1)
        for i in range(iters):
            ps = int(plan["pos_start"][i])
            torch.cat([kd[n0 + i * s: n0 + (i + 1) * s], kd[i * s: (i + 1) * s], kd[ps: ps + s],
                       nd[i * s: (i + 1) * s]], out=kb)
            t.mixed(ops, kb, kb * 3 + 1, combine="sum", out=out, status=st)
        ps = int(plan["pos_start"][iters])
        t.probe_counters(reset=True)
        f, _ = t.query(kd[ps: ps + s], out=out[:s], found=st[:s])
        assert bool((f == 1).all()), "aged %s: live keys" % des
        pos = t.probe_counters(reset=True)
        f, _ = t.query(nd[iters * s: (iters + 1) * s], out=out[:s], found=st[:s])
        assert bool((f == 0).all()), "aged %s: absent keys" % des
        neg = t.probe_counters(reset=True)
        per = lambda c: round((c["bucket_lines"] + c["slot_lines"]) / max(1, c["queries"]), 3)
        res[des] = {"positive": per(pos), "negative": per(neg), "paper_a40": PAPER_AGED_PROBES.get(des)}
        log("aged probes %s (GPU-counted, 2^%d slots, %d iterations): positive %.2f, negative %.2f (Table 1: %s)"
            % (des, log2cap, iters, res[des]["positive"], res[des]["negative"], PAPER_AGED_PROBES.get(des)))
        del t
        torch.cuda.empty_cache()
    return res


def bench_aging(designs, log2cap=26, iters=1000, probe_cap_lines=80):
    """The aging (churn) benchmark (Section 6.5) on each design: fill 2^log2cap slots
    to 0.85, then `iters` iterations, each ONE mixed launch inserting a new 1% slice,
    erasing the oldest 1% and querying 1% live and 1% never-inserted keys.  Every
    output of every iteration is checked on the device against its closed form
    (inserts and erases succeed, positives return 3k+1, negatives miss).  Double
    hashing stops its probe sequences after 80 cache lines of bucket data (80
    buckets of 8 slots, 20 of 32): the cap Table 1's aged probe counts imply."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    t0 = time.time()
    plan = w.aging_plan(1 << log2cap, iters=iters, workload_id=6)
    n0, s = plan["n0"], plan["s"]
    kd = to_dev(plan["keys"])
    nd = to_dev(plan["negs"])
    log("aging: plan of %d + %d x %d keys ready in %.1f s" % (n0, iters, s, time.time() - t0))
    ops = torch.cat([torch.full((s,), 1, dtype=torch.uint8), torch.full((s,), 3, dtype=torch.uint8),
                     torch.zeros(2 * s, dtype=torch.uint8)]).cuda()
    kb = torch.empty(4 * s, dtype=torch.int64, device="cuda")
    st = torch.empty(4 * s, dtype=torch.uint8, device="cuda")
    out = torch.empty(4 * s, dtype=torch.int64, device="cuda")
    res = {}
    for des in designs:
        cap = 0
        if des.startswith("DOUBLE"):
            bucket = 8 if des == "DOUBLE" else 32
            cap = probe_cap_lines * 8 // bucket  # 128-byte lines of 16-byte slots
        t = hw.Table(1 << log2cap, des, probe_cap=cap)
        pre = t.insert(kd[:n0], kd[:n0] * 3 + 1)
        # full[j]: plan key j ended FULL (both of its buckets full when it was
        # placed; legal, rare); it is then absent: its erase misses and a
        # positive query of it misses
        full = torch.zeros(n0 + iters * s, dtype=torch.bool, device="cuda")
        full[:n0] = pre == 3
        bad = ((pre != 1) & (pre != 3)).sum()
        ev = []
        for i in range(iters):
            ps = int(plan["pos_start"][i])
            torch.cat([kd[n0 + i * s: n0 + (i + 1) * s], kd[i * s: (i + 1) * s], kd[ps: ps + s],
                       nd[i * s: (i + 1) * s]], out=kb)
            vb = kb * 3 + 1
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            t.mixed(ops, kb, vb, combine="sum", out=out, status=st)
            b.record()
            ev.append((a, b))
            ins = st[:s]
            full[n0 + i * s: n0 + (i + 1) * s] = ins == 3
            bad += ((ins != 1) & (ins != 3)).sum()
            bad += (st[s: 2 * s] != (~full[i * s: (i + 1) * s]).to(torch.uint8)).sum()
            live = ~full[ps: ps + s]
            bad += (st[2 * s: 3 * s] != live.to(torch.uint8)).sum()
            bad += (out[2 * s: 3 * s] != torch.where(live, vb[2 * s: 3 * s], 0)).sum()
            bad += (st[3 * s:] != 0).sum() + (out[3 * s:] != 0).sum()
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        g = 4 * s / ms / 1e6
        nbad = int(bad.item())
        n_full = int(full.sum().item())
        assert nbad == 0, "aging %s: %d outputs differ from their closed form" % (des, nbad)
        assert t.size() == n0 - int(full[iters * s:].sum().item()), "aging %s: size" % des
        if n_full:
            log("aging %s: %d of %d inserts ended FULL (both buckets full)" % (des, n_full, n0 + iters * s))
        res[des] = {"gops_mean": round(float(4 * s * iters / ms.sum() / 1e6), 3),
                    "gops_first10": round(float(g[:10].mean()), 3),
                    "gops_last100": round(float(g[-100:].mean()), 3),
                    "gops_min": round(float(g.min()), 3),
                    "gops_every100": [round(float(g[j: j + 100].mean()), 3) for j in range(0, iters, 100)],
                    "probe_cap": cap or None, "verified": True, "full_inserts": n_full}
        log("aging %s: mean %.2f Gops/s, first 10 %.2f, last 100 %.2f"
            % (des, res[des]["gops_mean"], res[des]["gops_first10"], res[des]["gops_last100"]))
        del t
        torch.cuda.empty_cache()
    del kd, nd
    torch.cuda.empty_cache()
    return {"workload": "aging: 2^%d slots filled to 0.85, %d iterations of one mixed launch (insert new 1%%, "
                        "erase oldest 1%%, query 1%% live + 1%% absent)" % (log2cap, iters),
            "ops_per_iteration": 4 * s, "designs": res}


def mixed_zipf_check(present, val, done, ops, r, vd, st, out):
    """Checks one mixed batch's outputs against the shadow model of the map (a
    present flag and a value per universe rank) and advances the model to the
    batch's end.  Queries must return the batch-start state, erases report
    presence, and of a key's upserts exactly one inserts (the key was absent) or
    none (present), the rest report EXISTED.  Returns a 0-dim tensor counting the
    mismatches.  Masks only, no boolean indexing, so nothing waits for the device
    between batches.  All of a rank's operations in a batch are of one kind, so
    the scatters below write one value per rank."""
    import torch
    q, u, e = ops == 0, ops == 2, ops == 3
    pr = present[r]
    vr = val[r]
    zero = torch.zeros_like(vr)
    bad = ((st != pr.to(torch.uint8)) & (q | e)).sum()
    bad += ((out != torch.where(pr, vr, zero)) & q).sum()
    bad += ((st != 1) & (st != 2) & u).sum()
    done.zero_()
    done.index_add_(0, r, ((st == 1) & u).to(torch.int32))
    bad += ((done[r] != (~pr).to(torch.int32)) & u).sum()
    # an absent key's upserts start from 0 (wrapping 64-bit sums); erased keys leave
    val.scatter_(0, r, torch.where(u & ~pr, zero, vr))
    val.index_add_(0, r, torch.where(u, vd, torch.zeros_like(vd)))
    present.scatter_(0, r, (pr | u) & ~e)
    return bad


def bench_mixed_zipf(n_batches=256, log2cap=27, universe_log2=26, design="DOUBLE_M", n_unmerged=8):
    """The mixed concurrent workload: a 2^log2cap-slot table preloaded with a 2^universe_log2-key
    universe (load 0.5, v = 3k+1), then `n_batches` shuffled mixed batches of 2^20
    operations (50% query, 30% SUM upsert, 20% erase; Zipf 0.99 keys drawn
    interleaved, so hot keys fall to every kind; erase and upsert keys disjoint,
    queries avoid both).  The table merges each call's upserts by key
    (HWAVE_F_MERGE_MIXED).  Per-batch latency from events around the call.
    Every output is checked on the device against a shadow model of the map
    indexed by universe rank (present flag, value): queries return the
    batch-start state, erases report presence, and of a key's upserts exactly one
    inserts (the key was absent) or none (present), the rest report EXISTED;
    after the last batch the table's size and its sum of values equal the
    model's.  Then the first `n_unmerged` batches again on a table without
    merging (same preload, same checks): every upsert of a hot key waits in its
    bucket's lock queue."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    t0 = time.time()
    U = 1 << universe_log2
    uk = w.universe_keys(U, workload_id=3)
    batches = list(w.mixed_batches(U, 1 << 20, n_batches, workload_id=3, ukeys=uk))
    shares = np.array([w.hottest_upsert_share(bt) for bt in batches])
    log("mixed Zipf workload: %d batches of 2^20 ops over a 2^%d-key universe generated in %.1f s; "
        "hottest upsert key: median %.3f, max %.3f of a batch's upserts"
        % (n_batches, universe_log2, time.time() - t0, float(np.median(shares)), float(shares.max())))
    n = 1 << 20
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    # every batch is resident in HBM before the first launch (~26 MB each), so no
    # host copy sits between two batches' kernels
    staged = [(torch.from_numpy(bt["ops"]).cuda(), to_dev(bt["keys"]), to_dev(bt["vals"]),
               torch.from_numpy(bt["ranks"]).cuda()) for bt in batches]
    del batches

    def run(flags, count):
        t = hw.Table(1 << log2cap, design, flags=flags)
        ukd = to_dev(uk)
        pre = t.insert(ukd, ukd * 3 + 1)
        assert bool((pre == 1).all()), "mixed Zipf workload: preload"
        present = torch.ones(U, dtype=torch.bool, device="cuda")
        val = ukd * 3 + 1
        del ukd
        bad = torch.zeros((), dtype=torch.int64, device="cuda")
        done = torch.zeros(U, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        ev = []
        for ops, kd, vd, r in staged[:count]:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            t.mixed(ops, kd, vd, combine="sum", out=out, status=st)
            b.record()
            ev.append((a, b))
            bad += mixed_zipf_check(present, val, done, ops, r, vd, st, out)
        torch.cuda.synchronize()
        nbad = int(bad.item())
        assert nbad == 0, "mixed Zipf workload: %d outputs differ from the shadow model" % nbad
        assert t.size() == int(present.sum().item()), "mixed Zipf workload: size"
        _, tv = t.export()
        assert int(tv.sum().item()) == int(val[present].sum().item()), "mixed Zipf workload: sum of values"
        del t, present, val, done, tv
        torch.cuda.empty_cache()
        return np.array([a.elapsed_time(b) for a, b in ev])

    ms = run(hw.F_MERGE_MIXED, len(staged))
    ms_plain = run(0, min(n_unmerged, len(staged))) if n_unmerged else None
    res = {"workload": "%s, 2^%d slots, 2^%d-key universe preloaded (load 0.5), %d shuffled batches of 2^20 ops "
                       "(50%% query / 30%% SUM upsert / 20%% erase, Zipf 0.99, interleaved draws), upserts merged "
                       "by key per call" % (design, log2cap, universe_log2, n_batches),
           "p50_batch_ms": round(float(np.percentile(ms, 50)), 4), "p99_batch_ms": round(float(np.percentile(ms, 99)), 4),
           "mean_gops": round(float(n * len(ms) / ms.sum() / 1e6), 3), "verified": True,
           "hottest_upsert_key_share": {"median": round(float(np.median(shares)), 4),
                                        "max": round(float(shares.max()), 4)}}
    if ms_plain is not None:
        res["unmerged_first_batches"] = {
            "batches": len(ms_plain), "p50_batch_ms": round(float(np.percentile(ms_plain, 50)), 4),
            "max_batch_ms": round(float(ms_plain.max()), 4), "merged_p50_same_batches_ms":
                round(float(np.percentile(ms[:len(ms_plain)], 50)), 4), "verified": True}
    log("mixed Zipf workload: p50 %.3f ms, p99 %.3f ms per 2^20-op batch (%.2f Gops/s), all outputs verified%s"
        % (res["p50_batch_ms"], res["p99_batch_ms"], res["mean_gops"],
           "" if ms_plain is None else "; unmerged p50 %.3f ms over the first %d" % (
               res["unmerged_first_batches"]["p50_batch_ms"], len(ms_plain))))
    del staged
    torch.cuda.empty_cache()
    return res


def one_config(alls, ops_of):
    """The one configuration with the least estimated time over a whole batch:
    alls[e] lists the tuner's results for capacity class e (dicts with design,
    bucket, tile, gops and full_ops), ops_of[e] the batch's operations on tables
    of class e.  The estimate is the sum over classes of ops / rate; a
    configuration that left an operation FULL in any class, or was not timed in
    every class, is never chosen.  Returns (design, bucket, tile)."""
    key = lambda a: (a["design"], a["bucket"], a["tile"])
    est, seen = {}, {}
    for e, rows in alls.items():
        for a in rows:
            k = key(a)
            seen[k] = seen.get(k, 0) + 1
            if a["full_ops"] or a["gops"] <= 0:
                est[k] = float("inf")
            else:
                est[k] = est.get(k, 0.0) + ops_of[e] / (a["gops"] * 1e9)
    ok = [k for k in est if seen[k] == len(alls) and est[k] != float("inf")]
    if not ok:
        raise ValueError("no configuration held every class")
    return min(ok, key=lambda k: est[k])


def bench_batched(n_tables=4096, e_min=10, e_max=22, load=0.85, reps=3, tune_reps=2, n_verify=16):
    """The batched form: n_tables uint32 tables with capacities 2^e,
    e uniform in [e_min, e_max], each receiving a group-by SUM-upsert batch that
    fills it to `load`.  Times one persistent multi-table launch (configuration
    autotuned per capacity class) against one plain launch per table (same
    configurations) and against one persistent launch with a fixed default
    configuration.  A group of one configuration runs on that configuration's own
    kernel, a group of several on the menu's; so when the classes chose different
    configurations, one launch with the single configuration of least estimated
    time (from the tuner's rates) is timed too, and the faster group is the
    batched result.  Verifies every table's size and, on a sample of tables, every
    key and value against the group-by sums computed directly with numpy."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    t0 = time.time()
    exps = w.table_exponents(n_tables, e_min, e_max, workload_id=4)
    offsets, keys, vals = w.groupby_tables(exps, load, workload_id=4)
    n_ops = int(offsets[-1])
    log("batched: %d tables, %d ops generated in %.1f s" % (n_tables, n_ops, time.time() - t0))
    t0 = time.time()
    classes = sorted(set(int(e) for e in exps))
    tuned, rejected, tuned_ne, alls_ne = {}, {}, {}, {}
    for e in classes:
        tuned[e], rejected[e] = hw.autotune(32, 1 << e, load=load, reps=tune_reps)
        tuned_ne[e], alls_ne[e] = hw.autotune(32, 1 << e, load=load, reps=tune_reps, flags=hw.F_NO_ERASE)
    log("batched: autotuned %d classes (locking and erase-free tables) in %.1f s" % (len(classes), time.time() - t0))
    kd = torch.from_numpy(keys.view(np.int32)).cuda()
    vd = torch.from_numpy(vals.view(np.int32)).cuda()
    st = torch.empty(n_ops, dtype=torch.uint8, device="cuda")

    def make(cfg_of, flags=0):
        tabs = []
        for e in exps:
            d, b, t = cfg_of(int(e))
            tabs.append(hw.Table(1 << int(e), d, kv_bits=32, bucket=b, tile=t, flags=flags))
        return tabs, hw.Multi(tabs)

    def timed(fn, clear):
        ms = []
        for r in range(reps + 1):
            clear()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        return float(np.median(ms))

    ds = (offsets[1:] - offsets[:-1]) // 2
    pick = w.sample_without_replacement(w.stream_seed(4, 9), n_tables, min(n_verify, n_tables))

    def verify(tabs):
        """Sizes of all tables; on a sample, the exported pairs equal the group-by
        (distinct keys, wrapping 32-bit sums of their values)."""
        sizes = [t.size() for t in tabs]
        assert sizes == [int(x) for x in ds], "table sizes"
        for i in pick.tolist():
            a, b = int(offsets[i]), int(offsets[i + 1])
            uk, inv = np.unique(keys[a:b], return_inverse=True)
            sums = np.zeros(len(uk), dtype=np.uint64)
            np.add.at(sums, inv, vals[a:b].astype(np.uint64))
            k, v = tabs[i].export()
            k = k.cpu().numpy().view(np.uint32)
            v = v.cpu().numpy().view(np.uint32)
            o = np.argsort(k)
            assert np.array_equal(k[o], uk), "table %d: key set" % i
            assert np.array_equal(v[o], (sums & np.uint64(0xFFFFFFFF)).astype(np.uint32)), "table %d: sums" % i

    def batched_and_plain(cfg, flags):
        tabs, m = make(lambda e: (cfg[e]["design"], cfg[e]["bucket"], cfg[e]["tile"]), flags)
        ms_b = timed(lambda: m.upsert(offsets, kd, vd, status=st), m.clear)
        verify(tabs)  # the batched run's final state

        def plain():
            for i, t in enumerate(tabs):
                a, b = int(offsets[i]), int(offsets[i + 1])
                t.upsert(kd[a:b], vd[a:b], status=st[a:b])
        ms_p = timed(plain, m.clear)
        verify(tabs)  # the plain run's
        del m, tabs
        torch.cuda.empty_cache()
        return ms_b, ms_p

    ops_of = {e: int(sum(offsets[i + 1] - offsets[i] for i in range(n_tables) if exps[i] == e)) for e in classes}
    one_cfg = lambda alls: one_config(alls, ops_of)

    def uniform_group(best_of, alls, flags):
        """Per-class choices that differ put the group on the full menu's kernel; a
        group of one configuration runs on that configuration's own.  Returns the
        one-configuration alternative's (configuration, ms), or None when the
        per-class choices already agree."""
        if len({(v["design"], v["bucket"], v["tile"]) for v in best_of.values()}) == 1:
            return None
        try:
            c = one_cfg(alls)
        except ValueError:  # no configuration held every class
            return None
        tabs, m = make(lambda e: c, flags)
        assert m.kernel()[0] == "solo"
        ms = timed(lambda: m.upsert(offsets, kd, vd, status=st), m.clear)
        verify(tabs)
        del m, tabs
        torch.cuda.empty_cache()
        return c, ms

    ms_batched, ms_plain = batched_and_plain(tuned, 0)
    uni = uniform_group(tuned, rejected, 0)
    log("batched: verified sizes of all tables and %d tables against their group-by sums" % len(pick))
    # group-by tables never erase: declared so, a repeated key is summed without its lock
    ms_batched_ne, ms_plain_ne = batched_and_plain(tuned_ne, hw.F_NO_ERASE)
    uni_ne = uniform_group(tuned_ne, alls_ne, hw.F_NO_ERASE)
    log("batched: erase-free tables %.2f Gops/s in one launch (per-class configurations) vs %.2f Gops/s plain "
        "(verified)"
        % (n_ops / ms_batched_ne / 1e6, n_ops / ms_plain_ne / 1e6))
    tabs_d, m_d = make(lambda e: ("P2_M", 32, 4))
    ms_default = timed(lambda: m_d.upsert(offsets, kd, vd, status=st), m_d.clear)
    del m_d, tabs_d, kd, vd, st
    torch.cuda.empty_cache()
    gops = lambda ms: round(n_ops / ms / 1e6, 3)
    kernel_of = lambda cfg: "solo" if len({(v["design"], v["bucket"], v["tile"]) for v in cfg.values()}) == 1 else "menu"
    one = lambda u: None if u is None else {"config": "%s/b%d/t%d" % u[0], "batched_ms": round(u[1], 3),
                                            "batched_gops": gops(u[1])}
    for name, u in (("locking", uni), ("erase-free", uni_ne)):
        if u is not None:
            log("batched (%s): the classes chose different configurations; one configuration (%s/b%d/t%d) for all "
                "tables: %.2f Gops/s" % ((name,) + u[0] + (n_ops / u[1] / 1e6,)))
    # the group step of the tuning: of the two groups timed, the faster is the
    # batched form's result (per-class choices on the menu's kernel, or one
    # configuration on its own kernel)
    best = lambda ms, u: (ms, "per-class configurations") if u is None or ms <= u[1] else \
        (u[1], "one configuration, %s/b%d/t%d" % u[0])
    ms_best, policy = best(ms_batched, uni)
    ms_best_ne, policy_ne = best(ms_batched_ne, uni_ne)
    return {"workload": "%d uint32 tables, capacities 2^e (e uniform %d..%d), group-by SUM upserts to %.2f load"
                        % (n_tables, e_min, e_max, load),
            "ops": n_ops, "slots": int((1 << exps.astype(np.int64)).sum()),
            "batched_ms": round(ms_best, 3), "batched_gops": gops(ms_best), "group": policy,
            "per_class_ms": round(ms_batched, 3), "per_class_gops": gops(ms_batched),
            "plain_ms": round(ms_plain, 3), "plain_gops": gops(ms_plain),
            "default_cfg_batched_ms": round(ms_default, 3), "default_cfg_batched_gops": gops(ms_default),
            "speedup_vs_plain": round(ms_plain / ms_best, 3),
            "per_class_kernel": kernel_of(tuned), "one_config": one(uni),
            "erase_free": {"batched_ms": round(ms_best_ne, 3), "batched_gops": gops(ms_best_ne), "group": policy_ne,
                           "per_class_ms": round(ms_batched_ne, 3), "per_class_gops": gops(ms_batched_ne),
                           "plain_ms": round(ms_plain_ne, 3), "plain_gops": gops(ms_plain_ne),
                           "per_class_kernel": kernel_of(tuned_ne), "one_config": one(uni_ne),
                           "tuning": {str(e): "%s/b%d/t%d %.2f" % (v["design"], v["bucket"], v["tile"], v["gops"])
                                      for e, v in tuned_ne.items()}},
            "tuning": {str(e): "%s/b%d/t%d %.2f" % (v["design"], v["bucket"], v["tile"], v["gops"])
                       for e, v in tuned.items()},
            "rejected_full": {str(e): ["%s/b%d/t%d" % (a["design"], a["bucket"], a["tile"])
                                       for a in rej if a["full_ops"]] for e, rej in rejected.items()}}


def bench_served(n_tables=64, log2cap=26, n_req=2000, rate=20000.0, slots=3, sweep_rates=(14000.0, 20000.0, 26000.0),
                 sweep_s=10.0):
    """The served form: n_tables resident, erase-free P2HT(M) tables of 2^log2cap
    slots, preloaded with half of a Zipf universe of floor(0.85 * capacity) keys;
    n_req requests arriving as a Poisson process at `rate`/s (query / upsert /
    insert 50/30/20, sizes 2^U, U ~ U[8, 20], Zipf 0.99 keys).  The same stream is
    replayed through the batched server and through plain one-request launches on
    identical tables; latency = completion - arrival."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    cap = 1 << log2cap
    universe = int(0.85 * cap)
    t0 = time.time()
    reqs = list(w.served_requests(n_tables, universe, n_req, rate, workload_id=5))
    n_ops = sum(len(r["keys"]) for r in reqs)
    log("served: %d requests, %d ops generated in %.1f s" % (n_req, n_ops, time.time() - t0))
    OP = {"query": hw.OPS["query"], "insert": hw.OPS["insert"],
          "upsert": hw.OPS["upsert"] | (hw.COMBINES["sum"] << 8)}
    # pinned request buffers, reused by both runs
    bufs = []
    for r in reqs:
        k = torch.from_numpy(r["keys"].view(np.int64)).pin_memory()
        v = None if r["vals"] is None else torch.from_numpy(r["vals"].view(np.int64)).pin_memory()
        o = torch.empty(len(r["keys"]), dtype=torch.int64).pin_memory()
        st = torch.empty(len(r["keys"]), dtype=torch.uint8).pin_memory()
        bufs.append((k, v, o, st))
    offs = [r["t"] for r in reqs]

    def run(mode, arrivals=None):
        # the served kinds never erase: the tables are declared erase-free, so
        # present keys are combined without the lock, and merge duplicate keys
        # per window, so a Zipf-hot key reaches its value word once per window
        tabs = [hw.Table(cap, "P2_M", flags=hw.F_NO_ERASE | hw.F_AGGREGATE) for _ in range(n_tables)]
        pre_n = universe // 2
        for t in range(n_tables):
            pre = w.splitmix64(w.stream_seed(5, 100 + t), 0, pre_n)
            kk = torch.from_numpy(pre.view(np.int64)).cuda()
            tabs[t].insert(kk, kk * 3 + 1)
            del kk
        torch.cuda.synchronize()
        srv = hw.Server(tabs, mode=mode, slots=slots, slot_ops=1 << 22)
        rs = [hw.Server.request(r["table"], OP[r["kind"]], *b) for r, b in zip(reqs, bufs)]
        srv.replay(rs, offs if arrivals is None else arrivals)
        srv.drain()
        st = srv.stats()
        srv.close()
        res = [(b[2].numpy().copy() if r["kind"] == "query" else None, b[3].numpy().copy())
               for r, b in zip(reqs, bufs)]
        del tabs
        torch.cuda.empty_cache()
        return st, res

    st_b, res_b = run("batched")
    log("served batched: %.2f Gops/s, p50 %.2f ms, p99 %.2f ms, %.1f requests/launch"
        % (st_b["ops"] / st_b["wall_s"] / 1e9, st_b["p50_ms"], st_b["p99_ms"], st_b["mean_requests_per_batch"]))
    st_p, res_p = run("plain")
    log("served plain: %.2f Gops/s, p50 %.2f ms, p99 %.2f ms"
        % (st_p["ops"] / st_p["wall_s"] / 1e9, st_p["p50_ms"], st_p["p99_ms"]))
    # closed loop: every request submitted at once, the batched form's saturation
    st_c, res_c = run("batched", [0.0] * len(reqs))
    log("served closed loop (all requests at once): %.2f Gops/s, %.1f requests/launch"
        % (st_c["ops"] / st_c["wall_s"] / 1e9, st_c["mean_requests_per_batch"]))

    # each request's results alone (plain, serial) and in the mix (batched, at the
    # arrival rate and all at once) agree: query outputs exactly, write statuses as
    # per-key counts
    def same_as_plain(res):
        same = 0
        for r, (ob, sb), (op_, sp) in zip(reqs, res, res_p):
            if r["kind"] == "query":
                ok = np.array_equal(ob, op_) and np.array_equal(sb, sp)
            else:
                ok = all(np.array_equal(np.unique(r["keys"][sb == c]), np.unique(r["keys"][sp == c]))
                         and (sb == c).sum() == (sp == c).sum() for c in (1, 2))
            same += int(ok)
        return same == len(reqs)
    assert same_as_plain(res_b) and same_as_plain(res_c), "served results differ from the one-at-a-time replay"
    log("served: all %d requests equal alone (plain replay) and in the mix (at the rate and all at once)" % len(reqs))
    f = lambda st: {"gops": round(st["ops"] / st["wall_s"] / 1e9, 3), "p50_ms": round(st["p50_ms"], 3),
                    "p99_ms": round(st["p99_ms"], 3), "max_ms": round(st["max_ms"], 3),
                    "wall_s": round(st["wall_s"], 4), "requests_per_launch": round(st["mean_requests_per_batch"], 2)}
    offered = n_ops / offs[-1] / 1e9
    out = {"workload": "%d P2HT(M) tables x 2^%d slots, %d Poisson requests at %.0f/s, sizes 2^U (U~U[8,20]), "
                       "query/upsert/insert 50/30/20, Zipf 0.99" % (n_tables, log2cap, n_req, rate),
           "ops": n_ops, "offered_gops": round(offered, 3), "batched": f(st_b), "plain": f(st_p),
           "closed_loop_batched": f(st_c), "identical_results": True}
    if sweep_rates:
        out["sweep"] = served_sweep(reqs, bufs, n_tables, cap, universe, sweep_rates, sweep_s, slots, OP, f)
    return out


def served_sweep(reqs, bufs, n_tables, cap, universe, rates, seconds, slots, OP, f):
    """Long runs of the served form: at each arrival rate, `seconds` of Poisson
    arrivals whose requests cycle through the verified run's request payloads
    (table, kind, keys, values; outputs are overwritten and not checked), served
    batched and then plain on one set of resident tables.  Reports ops/s and
    p50/p99 latency per rate and mode, and the offered rate."""
    import torch
    import paper_2509_16407_amd as hw
    from paper_2509_16407_amd import workloads as w
    tabs = [hw.Table(cap, "P2_M", flags=hw.F_NO_ERASE | hw.F_AGGREGATE) for _ in range(n_tables)]
    pre_n = universe // 2
    for t in range(n_tables):
        pre = w.splitmix64(w.stream_seed(5, 100 + t), 0, pre_n)
        kk = torch.from_numpy(pre.view(np.int64)).cuda()
        tabs[t].insert(kk, kk * 3 + 1)
        del kk
    torch.cuda.synchronize()
    mean_ops = float(np.mean([len(r["keys"]) for r in reqs]))
    rows = []
    for i, rate in enumerate(rates):
        offs = w.poisson_arrivals(w.stream_seed(5, 7000 + i), rate, seconds)
        n = len(offs)
        row = {"rate_per_s": rate, "requests": n, "offered_gops": round(rate * mean_ops / 1e9, 3)}
        for mode in ("batched", "plain"):
            srv = hw.Server(tabs, mode=mode, slots=slots, slot_ops=1 << 22)
            P = len(reqs)
            rs = [hw.Server.request(reqs[j % P]["table"], OP[reqs[j % P]["kind"]], *bufs[j % P]) for j in range(n)]
            srv.replay(rs, list(offs))
            srv.drain()
            st = srv.stats()
            srv.close()
            row[mode] = f(st)
            log("served sweep: %.0f req/s (offered %.2f Gops/s), %s: %.2f Gops/s, p50 %.2f ms, p99 %.2f ms"
                % (rate, row["offered_gops"], mode, row[mode]["gops"], row[mode]["p50_ms"], row[mode]["p99_ms"]))
        rows.append(row)
    del tabs
    torch.cuda.empty_cache()
    return {"seconds_of_arrivals": seconds, "payloads_cycled": len(reqs), "rates": rows}


def _step_phases(d):
    """(kind, keys, values) of the load benchmark's step, in its order."""
    from paper_2509_16407_amd import workloads as w
    keys = d["keys"]
    vals = w.value_of(keys)
    ones = np.ones(len(d["qpos"]), np.uint64)
    b0, b1, b2 = d["bounds"]
    return [("insert", keys[:b0], vals[:b0]), ("insert", keys[b0:b1], vals[b0:b1]),
            ("insert", keys[b1:b2], vals[b1:b2]), ("query", d["qpos"], None), ("query", d["qneg"], None),
            ("upsert", d["qpos"], ones), ("erase", d["ekeys"], None), ("query", d["qpos"], None),
            ("query", d["qneg"], None)]


def _oracle_run(m, kind, k, v):
    if kind == "insert":
        m.insert(k, v)
    elif kind == "upsert":
        m.upsert(k, v)
    elif kind == "query":
        m.query(k)
    else:
        m.erase(k)


def cpu_baseline(d, cap_log2: int, single_log2: int = 24, max_threads: int = 16):
    """The CPU oracle on the benchmark's own step at the metric's size (the same
    inputs as the GPU step): T threads, the keys sharded by a hash of their own
    into T maps (one per thread), the phases in the step's order with a join
    between phases.  The oracle's map calls release the interpreter lock, so the
    shards run in parallel.  `value` is that rate, `cores` = T.  A one-thread,
    one-map run of the whole step at this size would take minutes, so
    `single_thread_value` runs the same recipe at 2^single_log2 slots."""
    import concurrent.futures as cf
    import oracle
    phases = _step_phases(d)
    n_ops = sum(len(k) for _, k, _ in phases)
    b2 = d["bounds"][-1]
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    T = max(1, min(max_threads, avail))
    parts = []
    with np.errstate(over="ignore"):
        for kind, k, v in phases:
            sh = (((k * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(40)) % np.uint64(T)).astype(np.uint8)
            order = np.argsort(sh, kind="stable")
            cuts = np.cumsum(np.bincount(sh, minlength=T))[:-1]
            ks = np.split(k[order], cuts)
            vs = [None] * T if v is None else np.split(v[order], cuts)
            parts.append([(kind, ks[i], vs[i]) for i in range(T)])
            del sh, order
    maps = [oracle.OracleMap() for _ in range(T)]
    with cf.ThreadPoolExecutor(T) as ex:
        t0 = time.perf_counter()
        for ph in parts:
            list(ex.map(lambda i: _oracle_run(maps[i], *ph[i]), range(T)))
        dtT = time.perf_counter() - t0
    assert sum(mm.size() for mm in maps) == b2 - len(d["ekeys"]), "sharded oracle size"
    del maps, parts
    ds = make_inputs(single_log2, 0, 0)
    sph = _step_phases(ds)
    n1 = sum(len(k) for _, k, _ in sph)
    m = oracle.OracleMap()
    t0 = time.perf_counter()
    for kind, k, v in sph:
        _oracle_run(m, kind, k, v)
    dt1 = time.perf_counter() - t0
    del m, ds
    return dict(value=n_ops / dtT / 1e9, unit="Gops/s", cores=T, kind="oracle",
                single_thread_value=n1 / dt1 / 1e9,
                sample="the benchmark's step at 2^%d slots (insert to 0.9, 2^%d positive and negative "
                       "queries, upserts, 50%% erase, re-queries; the GPU step's own inputs), "
                       "std::unordered_map: %d ops over %d key-hash shards on %d threads in %.2f s; "
                       "single_thread_value: one thread, one map, the same recipe at 2^%d slots "
                       "(%d ops in %.2f s)" % (cap_log2, cap_log2 - 1, n_ops, T, T, dtT, single_log2, n1, dt1))


KERNEL_OF = {"insert_0.5": "k_upsert", "insert_0.75": "k_upsert", "insert_0.9": "k_upsert",
             "upsert": "k_upsert", "query_pos": "k_query", "query_neg": "k_query",
             "requery_pos": "k_query", "requery_neg": "k_query", "erase": "k_erase",
             "mixed": "k_mixed"}


def algo_kind(phase: str) -> str:
    return "insert" if phase.startswith("insert") else phase


def load_traffic():
    """Measured HBM bytes per launch, per phase, from the committed rocprofv3 counter
    summary -- only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_p2m_2p28.txt")
    if not os.path.exists(path):
        return None
    rec, phases = {}, {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("phase "):
                parts = line.split()
                kv = dict(x.split("=", 1) for x in parts[3:])
                phases.setdefault(parts[1], float(kv["hbm_bytes"]))
            elif "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k] = v
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return phases


def load_requests():
    """Fabric requests (L2 -> memory) per launch, per phase, and the copy kernel's
    request rate, from the committed counter summary -- current sources only."""
    path = os.path.join(ROOT, "profiles", "fabric_requests_p2m_2p28.txt")
    if not os.path.exists(path):
        return None
    rec, phases = {}, {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("phase "):
                parts = line.split()
                kv = dict(x.split("=", 1) for x in parts[3:])
                phases.setdefault(parts[1], float(kv["rd_req"]) + float(kv["wr_req"]))
            elif "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k] = v
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return phases, float(rec["reference_greq_s"])


def roofline(phase_ms: dict, per_step_ops: dict, steps: int, traffic_by_phase):
    """Roofline object of the dominant kernel (largest total time per step):
    algorithmic bytes of all its launches in a step / their total time, against the
    8 TB/s HBM peak; `traffic` = measured HBM bytes per launch (or None)."""
    kern_ms, kern_bytes, kern_launch, kern_meas = {}, {}, {}, {}
    for ph, lst in phase_ms.items():
        k = KERNEL_OF[ph]
        kern_ms[k] = kern_ms.get(k, 0.0) + float(np.sum(lst)) / steps
        n_launch = len(lst) // steps
        kern_launch[k] = kern_launch.get(k, 0) + n_launch
        kern_bytes[k] = kern_bytes.get(k, 0.0) + ALGO_BYTES[algo_kind(ph)] * per_step_ops[ph] * n_launch
        if traffic_by_phase is not None and ph in traffic_by_phase:
            kern_meas[k] = kern_meas.get(k, 0.0) + traffic_by_phase[ph] * n_launch
    dom = max(kern_ms, key=kern_ms.get)
    avg_launch_ms = kern_ms[dom] / kern_launch[dom]
    bytes_per_launch = kern_bytes[dom] / kern_launch[dom]
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    traffic = None
    if traffic_by_phase is not None and dom in kern_meas:
        traffic = round(kern_meas[dom] / kern_launch[dom])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom, "launches_per_step": kern_launch[dom],
            "algo_bytes_per_launch": round(bytes_per_launch), "avg_launch_ms": round(avg_launch_ms, 4)}
    if traffic is not None:
        roof["traffic_GBps"] = round(traffic / (avg_launch_ms * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_GBps"] / HBM_PEAK_GBS, 4)
    req = load_requests()
    if req is not None:
        # random single-line accesses: the request rate, not the byte rate, is the ceiling
        by_phase, ref = req
        n_req = sum(by_phase[ph] * (len(lst) // steps) for ph, lst in phase_ms.items()
                    if KERNEL_OF[ph] == dom and ph in by_phase)
        per_launch = n_req / kern_launch[dom]
        g = per_launch / (avg_launch_ms * 1e-3) / 1e9
        roof["fabric_requests"] = {"per_launch": round(per_launch), "achieved_Greq_s": round(g, 2),
                                   "copy_kernel_Greq_s": ref, "frac_of_copy": round(g / ref, 4)}
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2cap", type=int, default=28)
    ap.add_argument("--design", default="P2_M")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--bucket", type=int, default=0)
    ap.add_argument("--mixed-batches", type=int, default=16)
    ap.add_argument("--zipf-batches", type=int, default=256,
                    help="2^20-op batches of the mixed Zipf workload (DOUBLE_M, 2^27 slots; 0 to skip)")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-probes", action="store_true", help="skip the GPU-counted probes (instrumented build)")
    ap.add_argument("--no-batched", action="store_true", help="skip the multi-table (batched) section")
    ap.add_argument("--no-served", action="store_true", help="skip the serving section")
    ap.add_argument("--served-sweep-s", type=float, default=10.0,
                    help="seconds of arrivals per rate in the served-form rate sweep (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-aging", action="store_true", help="skip the aging (churn) section")
    ap.add_argument("--compare", default="DOUBLE,DOUBLE_M,P2,ICEBERG,ICEBERG_M,CHAINING,CUCKOO",
                    help="other designs to run the same step on ('' to skip)")
    ap.add_argument("--cpu-single-log2cap", type=int, default=24,
                    help="table size of the one-thread CPU oracle figure")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB read + 1 GiB write elementwise kernel first "
                         "(reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: HashWave has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    t0 = time.time()
    log("generating inputs (2^%d slots)" % args.log2cap)
    d = make_inputs(args.log2cap, args.mixed_batches, 1 << 20)
    log("inputs ready in %.1f s" % (time.time() - t0))
    step = Step(d, args.design, args.tile, args.bucket)
    torch.cuda.synchronize()
    log("device inputs resident; table %s bucket %d tile %d" % (args.design, step.t.bucket_slots, step.t.tile))
    verify_full = None
    if not args.no_verify:
        verify_full = verify_step(step, d)
        log("full-size closed-form verification passed (%d FULL inserts, each legal)" % verify_full)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1, out=dst)  # reads 2^30 bytes, writes 2^30 bytes
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy done (1 GiB read, 1 GiB written)")

    for _ in range(args.warmup):
        step.run()
    torch.cuda.synchronize()
    log("warmup done")

    events = {}
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        step.run(events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    log("timed %d steps in %.3f s" % (args.steps, wall))

    ops_per_step = step.ops_per_step()
    value = ops_per_step * args.steps / wall / 1e9
    phase_ms = {k: [a.elapsed_time(b) for a, b in v] for k, v in events.items()}
    rates = {}
    for name in step.phase_names:
        ms = np.mean(phase_ms[name])
        rates[name] = {"ms": round(float(ms), 4), "gops": round(step.ops[name] / ms / 1e6, 3)}
    if "mixed" in phase_ms:
        mixed = np.array(phase_ms["mixed"])
        mb = step.mixed_ops // len(step.mixed)
        rates["mixed"] = {"ms": round(float(mixed.mean()), 4), "gops": round(mb / mixed.mean() / 1e6, 3)}
        p50, p99 = float(np.percentile(mixed, 50)), float(np.percentile(mixed, 99))
    else:
        p50 = p99 = None

    per_step_ops = dict(step.ops)
    if step.mixed:
        per_step_ops["mixed"] = step.mixed_ops // len(step.mixed)
    roof = roofline(phase_ms, per_step_ops, args.steps, load_traffic())
    rates["upsert_miss_0.9"] = upsert_miss(step)
    log("upsert misses 0.75 -> 0.9: %.2f Gops/s" % rates["upsert_miss_0.9"]["gops"])
    probes = None
    if not args.no_probes:
        probes = probe_counts(step, args.design)
        log("probes at 0.9 (GPU-counted lines per query): positive %.3f, negative %.3f"
            % (probes["positive_lines_per_query"], probes["negative_lines_per_query"]))
        probes["load_probes_all_designs"] = load_probes(["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG",
                                                         "ICEBERG_M", "CHAINING"])

    cfg = {"workload": "load benchmark at 2^%d slots on %s (bucket %d, tile %d): insert to "
                       "0.5/0.75/0.9, 2^%d pos+neg queries, 2^%d SUM upserts, erase 50%%, "
                       "re-query, %d mixed 2^20-op batches"
                       % (args.log2cap, args.design, step.t.bucket_slots, step.t.tile,
                          args.log2cap - 1, args.log2cap - 1, len(step.mixed)),
           "slots": step.t.capacity, "ops_per_step": ops_per_step, "key_bits": 64,
           "parallelism": "single GPU"}
    designs = None
    cmp_list = [x for x in args.compare.split(",") if x and x != args.design]
    if cmp_list:
        designs = bench_designs(step, d, cmp_list, verify=not args.no_verify)
        main_t = step.t
        designs[args.design] = {"bucket": step.t.bucket_slots, "tile": step.t.tile, "main": True,
                                "phase_gops": {k: v["gops"] for k, v in rates.items()}}
        step.t = None
        torch.cuda.empty_cache()
        designs[args.design]["phased"] = bench_phased(step, d, args.design, designs[args.design]["phase_gops"])
        step.t = main_t

    zipf = None
    if args.zipf_batches:
        zipf = bench_mixed_zipf(n_batches=args.zipf_batches)

    aging = None
    if not args.no_aging:
        aging = bench_aging(["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG", "ICEBERG_M", "CHAINING", "CUCKOO"])
        if not args.no_probes:
            aging["probes"] = aging_probes(["DOUBLE", "DOUBLE_M", "P2", "P2_M", "ICEBERG", "ICEBERG_M", "CHAINING"])

    batched = None
    if not args.no_batched:
        del step
        torch.cuda.empty_cache()
        batched = bench_batched()
        log("batched: %.2f Gops/s in one launch vs %.2f Gops/s plain" % (batched["batched_gops"], batched["plain_gops"]))

    served = None
    if not args.no_served:
        if args.no_batched:
            del step
        torch.cuda.empty_cache()
        served = bench_served(sweep_rates=(14000.0, 20000.0, 26000.0) if args.served_sweep_s > 0 else (),
                              sweep_s=args.served_sweep_s)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) at 2^%d" % args.log2cap)
        cpu = cpu_baseline(d, args.log2cap, args.cpu_single_log2cap)

    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gops/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": cfg,
        "phases": rates,
        "insert_0.9_gops": rates["insert_0.9"]["gops"], "query_gops": rates["query_pos"]["gops"],
        "upsert_gops": rates["upsert"]["gops"], "upsert_miss_gops": rates["upsert_miss_0.9"]["gops"],
        "p50_batch_ms": None if p50 is None else round(p50, 4),
        "p99_batch_ms": None if p99 is None else round(p99, 4),
        "roofline": roof, "probes": probes, "cpu_baseline": cpu, "designs": designs, "mixed_zipf": zipf,
        "aging": aging,
        "batched": batched,
        "served": served,
        # the paper's own numbers on an NVIDIA A40 (Section 6.3, Table 1), beside
        # this run's matching figures: context, not a baseline of this workload
        "paper_a40_context": {
            "p2m_query_at_0.9_gops": {"paper": 2.605, "here": rates["query_pos"]["gops"]},
            "p2m_query_concurrent_phased_mops": {"paper": [2903, 2909]},
            "p2_insert_peak_gops": {"paper": 2.037},
            "metadata_tables_delete_gops": {"paper": 1.17, "here_p2m_erase": rates["erase"]["gops"]},
        },
        "kernel_source_hash": kernel_source_hash(),
        # inserts of the verified fill that ended FULL with every bucket of the
        # key full (null when verification was skipped)
        "verify_full_inserts": verify_full,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

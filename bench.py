#!/usr/bin/env python3
"""HashWave benchmark: the load benchmark of the paper (Section 6.3) at 2^28 slots on
one MI355X, on the power-of-two-choice table with 16-bit tags.

One step = one pass of the whole hot path over one synthetic batch set:
  clear; insert distinct uniform keys to load 0.5, 0.75, 0.9 (v = 3k+1);
  2^27 positive and 2^27 negative queries; 2^27 SUM upserts on present keys;
  erase a seeded 50% of the keys; re-query the positive and negative sets;
  16 mixed batches of 2^20 ops (50% query / 30% SUM upsert / 20% erase, Zipf 0.99
  over the inserted keys).
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
# load; derivation in the design doc.
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
    keys, bounds = w.load_phases(cap, (0.5, 0.75, 0.9), config_id=2)
    n = bounds[-1]
    nq = min(1 << (cap_log2 - 1), n)  # 2^27 positive and 2^27 negative queries at 2^28
    pos_idx = w.sample_without_replacement(w.stream_seed(2, 3), n, nq)
    qpos = keys[pos_idx]
    qneg = w.distinct_keys(w.stream_seed(2, 1), nq, skip=n)
    er_idx = w.sample_without_replacement(w.stream_seed(2, 4), n, n // 2)
    ekeys = keys[er_idx]
    mixed = []
    if n_mixed:
        for b in w.mixed_batches(n, mixed_batch, n_mixed, config_id=2, ukeys=keys):
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
        self.t = hw.Table(d["cap"], design, bucket=bucket, tile=tile)
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


def verify_step(step: Step, d) -> None:
    """Closed-form checks of one full step at full size (no oracle needed): every
    insert DONE, positives return 3k+1 (3k+2 after the +1 upsert), negatives miss,
    erased keys miss, kept keys found, table size equals inserted - erased."""
    import torch
    from paper_2509_16407_amd import workloads as w
    t = step.t
    t.clear()
    b2 = step.bounds[-1]
    st = t.insert(step.keys, step.vals, status=step.st[:b2])
    assert bool((st == 1).all()), "insert statuses"
    f, v = t.query(step.qpos, out=step.out)
    assert bool((f == 1).all()), "positive queries"
    exp = to_dev(w.value_of(d["qpos"]))
    assert bool((v == exp).all()), "positive values"
    f, v = t.query(step.qneg, out=step.out)
    assert bool((f == 0).all()) and bool((v == 0).all()), "negative queries"
    st = t.upsert(step.qpos, step.ones, combine="sum")
    assert bool((st == 2).all()), "upsert statuses"
    f, v = t.query(step.qpos, out=step.out)
    assert bool((v == exp + 1).all()), "upserted values"
    st = t.erase(step.ekeys)
    assert bool((st == 1).all()), "erase statuses"
    assert t.size() == b2 - len(d["ekeys"]), "size after erase"
    erased = np.zeros(b2, dtype=bool)
    erased[d["er_idx"]] = True
    kept_mask = torch.from_numpy(~erased[d["pos_idx"]]).cuda()
    f, v = t.query(step.qpos, out=step.out)
    assert bool(((f == 1) == kept_mask).all()), "re-query membership"
    assert bool(torch.where(kept_mask, v == exp + 1, v == 0).all()), "re-query values"
    torch.cuda.synchronize()
    del exp


def cpu_baseline(cap_log2: int):
    """The CPU oracle (single thread) on the same step recipe at a smaller size."""
    import oracle
    from paper_2509_16407_amd import workloads as w
    d = make_inputs(cap_log2, 0, 0)
    m = oracle.OracleMap()
    keys = d["keys"]
    vals = w.value_of(keys)
    ones = np.ones(len(d["qpos"]), np.uint64)
    t0 = time.perf_counter()
    b0, b1, b2 = d["bounds"]
    m.insert(keys[:b0], vals[:b0])
    m.insert(keys[b0:b1], vals[b0:b1])
    m.insert(keys[b1:b2], vals[b1:b2])
    m.query(d["qpos"])
    m.query(d["qneg"])
    m.upsert(d["qpos"], ones)
    m.erase(d["ekeys"])
    m.query(d["qpos"])
    m.query(d["qneg"])
    dt = time.perf_counter() - t0
    n_ops = b2 + 5 * len(d["qpos"]) + len(d["ekeys"])  # inserts, 4 query sets + upserts, erases
    return dict(value=n_ops / dt / 1e9, unit="Gops/s", cores=1, kind="oracle",
                sample="same step recipe (insert to 0.9, 2^%d pos + neg queries, upserts, 50%% erase, "
                       "re-query) at 2^%d slots, std::unordered_map, 1 thread; %d ops in %.1f s"
                       % (cap_log2 - 1, cap_log2, n_ops, dt))


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
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-log2cap", type=int, default=24)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB read + 1 GiB write elementwise kernel first "
                         "(reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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
    if not args.no_verify:
        verify_step(step, d)
        log("full-size closed-form verification passed")

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

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) at 2^%d" % args.cpu_log2cap)
        cpu = cpu_baseline(args.cpu_log2cap)

    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gops/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "load benchmark at 2^%d slots on %s (bucket %d, tile %d): insert to "
                               "0.5/0.75/0.9, 2^%d pos+neg queries, 2^%d SUM upserts, erase 50%%, "
                               "re-query, %d mixed 2^20-op batches"
                               % (args.log2cap, args.design, step.t.bucket_slots, step.t.tile,
                                  args.log2cap - 1, args.log2cap - 1, len(step.mixed)),
                   "slots": step.t.capacity, "ops_per_step": ops_per_step, "key_bits": 64,
                   "parallelism": "single GPU"},
        "phases": rates,
        "insert_0.9_gops": rates["insert_0.9"]["gops"], "query_gops": rates["query_pos"]["gops"],
        "upsert_gops": rates["upsert"]["gops"],
        "p50_batch_ms": None if p50 is None else round(p50, 4),
        "p99_batch_ms": None if p99 is None else round(p99, 4),
        "roofline": roof, "cpu_baseline": cpu,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""The bench's on-device check of the mixed concurrent workload (mixed_zipf_check),
run on the CPU with the oracle standing in for the table: it must accept the
oracle's outputs batch after batch, keep the model's size and value sum equal to
the oracle's, and reject each kind of planted mistake.  Also the batched form's
choice of one configuration for a whole group (one_config)."""
import numpy as np
import pytest
import torch

import bench
import oracle
from paper_2509_16407_amd import workloads as w

U = 1 << 12


def _setup(n_batches=4, batch=1 << 10):
    uk = w.universe_keys(U, workload_id=3)
    om = oracle.OracleMap()
    om.insert(uk, 3 * uk + 1)
    present = torch.ones(U, dtype=torch.bool)
    val = torch.from_numpy((3 * uk + 1).view(np.int64).copy())
    done = torch.zeros(U, dtype=torch.int32)
    return uk, om, present, val, done, list(w.mixed_batches(U, batch, n_batches, workload_id=3, ukeys=uk))


def _run(om, bt):
    st, out = om.apply(bt["keys"], bt["vals"], ops=bt["ops"])
    return torch.from_numpy(st.copy()), torch.from_numpy(out.view(np.int64).copy())


def _args(bt):
    return (torch.from_numpy(bt["ops"].copy()), torch.from_numpy(bt["ranks"].astype(np.int64)),
            torch.from_numpy(bt["vals"].view(np.int64).copy()))


def test_mixed_zipf_check_accepts_the_oracle_batch_after_batch():
    uk, om, present, val, done, batches = _setup()
    for bt in batches:
        st, out = _run(om, bt)
        ops, r, vd = _args(bt)
        assert int(bench.mixed_zipf_check(present, val, done, ops, r, vd, st, out)) == 0
    assert int(present.sum()) == om.size()
    _, ov = om.dump()
    assert int(val[present].sum()) == int(ov.view(np.int64).sum())


@pytest.mark.parametrize("mistake", ["query_status", "query_value", "erase_status", "upsert_twice",
                                     "upsert_status"])
def test_mixed_zipf_check_rejects_planted_mistakes(mistake):
    uk, om, present, val, done, batches = _setup(n_batches=2)
    bt = batches[0]
    st, out = _run(om, bt)
    ops, r, vd = _args(bt)
    q = np.nonzero(bt["ops"] == 0)[0]
    e = np.nonzero(bt["ops"] == 3)[0]
    u = np.nonzero(bt["ops"] == 2)[0]
    if mistake == "query_status":
        st[q[0]] ^= 1
    elif mistake == "query_value":
        out[q[np.nonzero(st.numpy()[q] == 1)[0][0]]] += 1
    elif mistake == "erase_status":
        st[e[0]] ^= 1
    elif mistake == "upsert_twice":
        # a key upserted more than once whose first upsert inserted: a second DONE
        ranks = bt["ranks"][u]
        vals, counts = np.unique(ranks, return_counts=True)
        multi = set(vals[counts > 1].tolist())
        cand = [i for i in u if bt["ranks"][i] in multi and st[i] == 2]
        st[cand[0]] = 1
    else:
        st[u[0]] = 3  # FULL is never a valid outcome here
    assert int(bench.mixed_zipf_check(present, val, done, ops, r, vd, st, out)) > 0


def _row(design, bucket, tile, gops, full=0):
    return {"design": design, "bucket": bucket, "tile": tile, "gops": gops, "full_ops": full}


def test_one_config_minimises_the_estimated_batch_time():
    """The batched form's group step: the one configuration with the least sum over
    classes of ops / rate, never one that left an op FULL in some class or was not
    timed in every class."""
    ops = {10: 1_000_000, 20: 100_000_000}
    alls = {10: [_row("DOUBLE", 16, 4, 6.0), _row("DOUBLE", 16, 8, 9.0), _row("P2_M", 16, 4, 20.0, full=3)],
            20: [_row("DOUBLE", 16, 4, 8.0), _row("DOUBLE", 16, 8, 7.9), _row("P2_M", 16, 4, 30.0)]}
    # per class, t8 wins class 10 and t4 class 20; over the batch, class 20 dominates
    assert bench.one_config(alls, ops) == ("DOUBLE", 16, 4)
    ops = {10: 100_000_000, 20: 1_000_000}
    assert bench.one_config(alls, ops) == ("DOUBLE", 16, 8)
    # a configuration timed in only one class is not a candidate
    alls[20].append(_row("DOUBLE_M", 32, 4, 50.0))
    assert bench.one_config(alls, ops) == ("DOUBLE", 16, 8)
    # FULL anywhere excludes a configuration, even when it is fastest elsewhere
    alls[10].append(_row("DOUBLE_M", 32, 4, 50.0, full=1))
    assert bench.one_config(alls, ops) == ("DOUBLE", 16, 8)
    with pytest.raises(ValueError):
        bench.one_config({10: [_row("P2_M", 16, 4, 9.0, full=1)]}, {10: 1})

"""The allocation-free entry point (hwave_mixed_noalloc) against the entry point
it is a variant of (hwave_mixed on a table created with HWAVE_F_MERGE_MIXED),
through the C-ABI: two calls in a row, the second smaller, each compared
element by element (statuses, query values) and by the dump afterwards.  Both
merge every key's upserts under its smallest index, so outputs are identical.
Also the size limit (2^18 operations): a larger call is refused with
HWAVE_ETOOBIG and leaves the table untouched."""
import numpy as np
import pytest
import torch

import paper_2509_16407_amd as hw
from paper_2509_16407_amd import workloads as w
from gpu_util import dev, host, u8

pytestmark = pytest.mark.gpu


def _dump(t):
    k, v = t.export()
    k, v = host(k), host(v)
    o = np.argsort(k)
    return k[o], v[o]


@pytest.mark.parametrize("design", ["P2_M", "DOUBLE_M"])
def test_noalloc_equals_merged_mixed(design):
    universe = 1 << 20
    uk = w.universe_keys(universe, workload_id=13)
    ref = hw.Table(1 << 21, design, flags=hw.F_MERGE_MIXED)
    new = hw.Table(1 << 21, design)  # no workspace of its own
    for t in (ref, new):
        assert bool((t.insert(dev(uk), dev(w.value_of(uk))) == hw.ST_DONE).all())
    sizes = [1 << 18, 50000]  # the limit itself, then a smaller call
    for bt, n in zip(w.mixed_batches(universe, 1 << 18, 2, workload_id=13, ukeys=uk), sizes):
        ops = torch.from_numpy(bt["ops"][:n]).cuda()
        kd, vd = dev(bt["keys"][:n]), dev(bt["vals"][:n])
        s0, v0 = ref.mixed(ops, kd, vd, combine="sum")
        s1, v1 = new.mixed_noalloc(ops, kd, vd, combine="sum")
        assert np.array_equal(u8(s0), u8(s1))
        assert np.array_equal(host(v0), host(v1))
        a, b = _dump(ref), _dump(new)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_noalloc_rejects_a_batch_over_its_limit():
    t = hw.Table(1 << 16, "P2_M")
    n = (1 << 18) + 1
    keys = w.distinct_keys(w.stream_seed(84, 1), n)
    ops = torch.full((n,), 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(hw.HashWaveError, match="fixed workspace"):
        t.mixed_noalloc(ops, dev(keys), dev(keys), combine="sum")
    torch.cuda.synchronize()
    assert t.size() == 0

"""The C-ABI library (CPU only): it loads, exports every function the header
declares, and its host-only calls (sizes, defaults, error text) behave.  No
kernel is launched here."""
import ctypes
import os
import re

import pytest

import paper_2509_16407_amd as hw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hashwave.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hwave_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    so = ctypes.CDLL(hw.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def _bytes(capacity, design, kv_bits=64, bucket=0, tile=0, flags=0):
    c = hw._Config(kv_bits, bucket, tile, 0, flags, 0)
    b = ctypes.c_uint64()
    rc = hw.lib().hwave_table_bytes(capacity, design, ctypes.byref(c), ctypes.byref(b))
    return rc, b.value


@pytest.mark.parametrize("design,per_slot,bucket", [(0, 16, 8), (1, 18, 32), (2, 16, 32), (3, 18, 32),
                                                    (4, 16, 32), (5, 18, 32)])
def test_space_per_slot_matches_section_6_1(design, per_slot, bucket):
    """16 bytes per key-value slot, plus 2 bytes of tag in the metadata designs
    (Section 6.1); on top, one lock byte per bucket (Section 5.1 keeps one lock
    bit per bucket in an external array) at a stride of clamp(2^23 / buckets, 1,
    8) bytes, 2^14 eight-byte lock queues and a 256-byte control word."""
    slots = 1 << 28
    rc, b = _bytes(slots, design)
    assert rc == 0
    nb = slots // bucket
    stride = max(1, min(8, (1 << 23) // nb))
    assert b == slots * per_slot + nb * stride + 8 * (1 << 14) + 256


@pytest.mark.parametrize("log2nb,stride", [(10, 8), (20, 8), (21, 4), (22, 2), (23, 1), (26, 1)])
def test_lock_stride_spreads_locks_within_8_mib(log2nb, stride):
    """The lock array: buckets x stride bytes, the stride the largest power of two
    <= 8 that keeps the array within 2^23 bytes (P2HT(M), bucket 32; tags 2 bytes
    per slot; queues min(2^14, buckets) words)."""
    nb = 1 << log2nb
    rc, b = _bytes(nb * 32, 3)
    assert rc == 0
    r256 = lambda x: -(-x // 256) * 256
    assert b == nb * 32 * 18 + r256(nb * stride) + r256(8 * min(nb, 1 << 14)) + 256


def test_chaining_space():
    """Chaining: ceil(capacity / 7) bucket nodes and twice as many pool nodes, 128
    bytes each (7 pairs and a link, Section 5), one lock byte per bucket (at a
    stride of 8 bytes in a table this small), lock
    queues (the largest power of two <= the bucket count, 8 bytes each), and
    1024 pool-partition counters, one per 128-byte line."""
    rc, b = _bytes(7 * 1000, 6)
    assert rc == 0
    nb, pool = 1000, 2000
    node_bytes = -(-(nb + pool) * 128 // 256) * 256
    lock_bytes = -(-(8 * nb) // 256) * 256 + 512 * 8  # stride 8: 1000 buckets << 2^23
    assert b == node_bytes + lock_bytes + 256 + 1024 * 128
    assert _bytes(7 * 1000, 6, kv_bits=32)[0] == -4  # 64-bit keys only


@pytest.mark.parametrize("design", range(8))
def test_merge_workspace_size(design):
    """HWAVE_F_MERGE_MIXED adds the merge workspace: 2 * 2^20 entries of an 8-byte
    key word and 16 bytes, and a 4-byte word per operation of a 2^20-operation
    chunk (rounded to 256 bytes)."""
    rc0, plain = _bytes(1 << 16, design)
    rc1, merged = _bytes(1 << 16, design, flags=hw.F_MERGE_MIXED)
    assert rc0 == rc1 == 0
    assert merged - plain == (2 << 20) * 24 + (1 << 20) * 4


@pytest.mark.parametrize("design", range(8))
def test_hot_key_accumulators_only_for_merging_erase_free_tables(design):
    """32 x 128 entries of two 8-byte words (64 KiB) are added exactly when a
    table merges duplicates and never erases, and not for cuckoo (it moves keys)
    or the phased variant."""
    both = hw.F_AGGREGATE | hw.F_NO_ERASE
    rc0, plain = _bytes(1 << 16, design)
    assert rc0 == 0
    for flags in (hw.F_AGGREGATE, hw.F_NO_ERASE):
        assert _bytes(1 << 16, design, flags=flags) == (0, plain)
    extra = 0 if design == 7 else 32 * 128 * 16
    assert _bytes(1 << 16, design, flags=both) == (0, plain + extra)
    if design != 7 and design != 6:  # the phased variant: default bucket and tile only
        assert _bytes(1 << 16, design, flags=both | hw.F_BSP) == (0, plain)


def test_capacity_rounds_up_to_power_of_two_buckets():
    rc, b1 = _bytes(1000, 0)
    rc2, b2 = _bytes(1024, 0)
    assert rc == rc2 == 0 and b1 == b2  # 1000 slots -> 128 buckets of 8
    rc3, b3 = _bytes(1025, 0)
    assert b3 > b2


def test_iceberg_has_a_bucket_in_each_yard():
    """The smallest iceberg table holds two buckets: one front yard, one backyard."""
    rc, b1 = _bytes(1, 4)
    rc2, b2 = _bytes(64, 4)
    assert rc == rc2 == 0 and b1 == b2
    rc3, b3 = _bytes(65, 4)
    assert b3 > b2


def test_bad_arguments_rejected_on_host():
    L = hw.lib()
    assert _bytes(0, 0)[0] == -1                      # capacity 0
    assert _bytes(1024, 8)[0] == -1                   # no such design
    assert _bytes(1024, 0, kv_bits=16)[0] == -1       # key width
    assert _bytes(1024, 0, bucket=8, tile=16)[0] == -4  # no kernel instance
    b = ctypes.c_uint64()
    for limit, rc in ((40000000, 0), (40000001, -1)):    # lock time limit, microseconds
        c = hw._Config(64, 0, 0, 0, 0, limit)
        assert L.hwave_table_bytes(1024, 0, ctypes.byref(c), ctypes.byref(b)) == rc
    assert L.hwave_table_bytes(1024, 0, None, None) == -1
    c = hw._Config()
    assert L.hwave_config_default(9, ctypes.byref(c)) == -1
    assert L.hwave_config_default(3, ctypes.byref(c)) == 0
    assert (c.kv_bits, c.bucket_slots, c.tile) == (64, 32, 4)
    assert L.hwave_num_buckets(None) == 0 and L.hwave_capacity(None) == 0
    assert L.hwave_destroy(None) == -1
    k, wv = ctypes.c_uint32(7), ctypes.c_uint32(7)
    assert L.hwave_multi_kernel(None, ctypes.byref(k), ctypes.byref(wv)) == -1
    assert (k.value, wv.value) == (7, 7)                # untouched on error
    assert L.hwave_multi_destroy(None) == -1
    for code in (0, -1, -2, -3, -4):
        assert L.hwave_strerror(code)


def test_paper_default_configurations():
    """Section 5: double hashing bucket 8 / tile 8; its metadata variant bucket 32 /
    tile 4; power-of-two-choice bucket 32 / tile 8; its metadata variant 32 / 4;
    iceberg bucket 32 / tile 8; its metadata variant 32 / 4."""
    L = hw.lib()
    expect = {0: (8, 8), 1: (32, 4), 2: (32, 8), 3: (32, 4), 4: (32, 8), 5: (32, 4), 6: (7, 8), 7: (8, 4)}
    for d, (b, t) in expect.items():
        c = hw._Config()
        assert L.hwave_config_default(d, ctypes.byref(c)) == 0
        assert (c.bucket_slots, c.tile) == (b, t)


def test_tuning_file_round_trip(tmp_path):
    """hwave_tune_save / hwave_tune_load: every field survives, the text format is
    the documented one, and classes come back in the saved order."""
    table = {10: {"design": "DOUBLE", "bucket": 16, "tile": 4, "kv_bits": 32, "gops": 7.25, "full_ops": 0,
                  "load": 0.85, "flags": 0},
             22: {"design": "DOUBLE_M", "bucket": 32, "tile": 4, "kv_bits": 32, "gops": 6.125, "full_ops": 3,
                  "load": 0.9, "flags": hw.F_NO_ERASE},
             14: {"design": "P2_M", "bucket": 64, "tile": 8, "kv_bits": 64, "gops": 1e-3, "full_ops": 0,
                  "load": 0.5, "flags": hw.F_AGGREGATE | hw.F_NO_ERASE}}
    path = tmp_path / "tune.txt"
    hw.save_tuning(str(path), table)
    lines = path.read_text().splitlines()
    assert lines[0] == "hwave-tune 2"
    assert lines[1].split()[:7] == ["10", "0.84999999999999998", "0", "32", str(hw.DESIGNS["DOUBLE"]), "16", "4"]
    back = hw.load_tuning(str(path))
    assert back == table
    assert list(back) == [10, 14, 22]


@pytest.mark.parametrize("body", [
    "hwave-tune 1\n10 32 0 16 4 7.0 0\n",                # the earlier format, without load and flags
    "hwave-tune 2\n10 0.85 0 32 0 16 4 7.0\n",           # a field missing
    "hwave-tune 2\n10 0.85 0 32 0 16 4 7.0 0 extra\n",   # trailing text
    "hwave-tune 2\n10 0.85 0 48 0 16 4 7.0 0\n",         # key width
    "hwave-tune 2\n10 0.85 0 32 9 16 4 7.0 0\n",         # design
    "hwave-tune 2\n10 0.85 0 32 0 16 0 7.0 0\n",         # tile
    "hwave-tune 2\n10 0 0 32 0 16 4 7.0 0\n",            # load 0
    "hwave-tune 2\n10 1.5 0 32 0 16 4 7.0 0\n",          # load above 1
    "hwave-tune 2\n10 0.85 16 32 0 16 4 7.0 0\n",        # unknown flag
    "hwave-tune 2\n10 nan 0 32 0 16 4 7.0 0\n",           # load not a number
])
def test_tuning_file_rejects_malformed(tmp_path, body):
    path = tmp_path / "bad.txt"
    path.write_text(body)
    with pytest.raises(hw.HashWaveError):
        hw.load_tuning(str(path))


def test_tuning_file_errors(tmp_path):
    L = hw.lib()
    n = ctypes.c_uint32()
    assert L.hwave_tune_load(str(tmp_path / "missing.txt").encode(), None, None, 0, ctypes.byref(n)) == -5
    path = tmp_path / "two.txt"
    path.write_text("hwave-tune 2\n10 0.85 0 32 0 16 4 7.0 0\n11 0.85 0 32 0 16 4 7.0 0\n")
    caps = (ctypes.c_uint32 * 1)()
    arr = (hw._Tune * 1)()
    assert L.hwave_tune_load(str(path).encode(), caps, arr, 1, ctypes.byref(n)) == -5  # more classes than room
    assert n.value == 0
    assert L.hwave_tune_save(None, None, None, 0) == -1
    assert L.hwave_strerror(-5).startswith(b"file")


def test_documented_configurations_have_instances():
    """Every (kv_bits, design, bucket, tile) the header lists sizes a table (an
    instance exists); a few unlisted ones report EUNSUPPORTED."""
    import re
    text = open(os.path.join(os.path.dirname(hw.LIB_PATH), "..", "include", "hashwave.h")).read()
    block = text[text.index("Supported (kv_bits, design, bucket/tile)"): text.index("Reserved key patterns")]
    bits = None
    seen = 0
    for line in block.splitlines():
        if "64-bit keys/values" in line:
            bits = 64
        elif "32-bit keys/values" in line:
            bits = 32
        for name, cfgs in re.findall(r"\b(DOUBLE_M|DOUBLE|P2_M|P2|ICEBERG_M|ICEBERG)\s+((?:b\d+/t\d+\s*)+)", line):
            for b, t in re.findall(r"b(\d+)/t(\d+)", cfgs):
                rc, _ = _bytes(1 << 12, hw.DESIGNS[name], kv_bits=bits, bucket=int(b), tile=int(t))
                assert rc == 0, (bits, name, b, t)
                seen += 1
    assert seen >= 40
    assert _bytes(1 << 12, hw.DESIGNS["P2_M"], bucket=32, tile=64)[0] == -4
    assert _bytes(1 << 12, hw.DESIGNS["CUCKOO"], kv_bits=32)[0] == -4

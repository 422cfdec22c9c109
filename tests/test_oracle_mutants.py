"""Strength of the oracle's pins: each planted mistake (a dropped wrap-around,
an off-by-one sentinel set, an erase that keeps the key, a capacity check off by
one, KEEP acting as REPLACE, an even double-hashing step, a 1/2 shortcut
threshold, ties sent to the alternate bucket, a wrong tag remap, a wrong probe
count, a checker blind to duplicates, a query returning the key, a 90/10 iceberg
split, backyard ties sent to the second choice, erase without tombstones in
the aging simulator, chaining that only looks for room in a chain's first
node, cuckoo that never looks past a key's first bucket, an insert that counts
the alternate bucket as visited under the shortcut) is built into a
copy of the oracle, and the oracle's own pin tests must fail against it."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MUTANTS = list(range(1, 19))


def _killed(k, tmp):
    lib = os.path.join(tmp, "mutant%d.so" % k)
    oracle.build(extra_flags=("-DORC_MUTANT=%d" % k,), out=lib)
    env = dict(os.environ, HW_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode != 0


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 2)) as ex:
            killed = dict(zip(MUTANTS, ex.map(lambda k: _killed(k, tmp), MUTANTS)))
    survivors = [k for k, v in killed.items() if not v]
    assert not survivors, "mutants not caught by any pin: %s" % survivors


def test_unmutated_oracle_passes_its_pins():
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "clean.so")
        oracle.build(out=lib)
        env = dict(os.environ, HW_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:]

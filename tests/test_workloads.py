"""Seeded input generators (CPU only): each checked against an independent
restatement of its published definition or a property that must hold."""
import numpy as np

from paper_2509_16407_amd import workloads as w

MASK = (1 << 64) - 1


def _splitmix_py(seed, n):
    """splitmix64 with Python integers (Steele, Lea, Flood 2014)."""
    s = seed
    out = []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_matches_integer_definition():
    for seed in (0, 1, 1234567, w.stream_seed(2, 1), MASK):
        assert w.splitmix64(seed, 0, 50).tolist() == _splitmix_py(seed, 50)
    # offset access equals the tail of a longer draw
    assert w.splitmix64(99, 17, 10).tolist() == _splitmix_py(99, 27)[17:]
    # the compiled path (long draws) agrees with the definition too
    long = w.splitmix64(12345, 100, 6000)
    assert long.tolist() == _splitmix_py(12345, 6100)[100:]


def test_distinct_keys_and_continuation_disjoint():
    a = w.distinct_keys(w.stream_seed(1, 1), 200000)
    b = w.distinct_keys(w.stream_seed(1, 1), 200000, skip=200000)
    assert len(np.unique(a)) == len(a) == 200000
    assert len(np.intersect1d(a, b)) == 0
    assert (a <= np.uint64(MASK - 3)).all()
    both = w.distinct_keys(w.stream_seed(1, 1), 400000)
    assert (both[:200000] == a).all() and (both[200000:] == b).all()


def test_distinct_keys_32():
    k = w.distinct_keys(77, 300000, key_bits=32)
    assert len(np.unique(k)) == len(k) == 300000
    assert (k <= np.uint64(0xFFFFFFFF - 3)).all()


def test_permutation_is_a_permutation():
    for n in (0, 1, 2, 1000, 300001):
        p = w.permutation(5, n)
        assert np.array_equal(np.sort(p), np.arange(n))
    assert not np.array_equal(w.permutation(5, 1000), np.arange(1000))
    assert np.array_equal(w.permutation(5, 300001), w.permutation(5, 300001))


def test_zipf_rank_frequencies():
    """P(rank r) of Zipf(theta) over n ranks is (r+1)^-theta / zeta(n)."""
    n, theta = 1 << 16, 0.99
    z = w.Zipf(n, theta)
    r = z.ranks(123, 0, 2_000_000)
    assert r.min() >= 0 and r.max() < n
    zeta = np.sum(np.arange(1, n + 1, dtype=np.float64) ** -theta)
    for rank in (0, 1):
        p = (rank + 1) ** -theta / zeta
        obs = np.mean(r == rank)
        assert abs(obs - p) < 5 * np.sqrt(p * (1 - p) / len(r)), (rank, obs, p)


def test_mixed_batches_are_deterministic_and_disjoint():
    gen = w.mixed_batches(1 << 14, 1 << 12, 2, workload_id=3)
    for b in gen:
        ops, keys = b["ops"], b["keys"]
        er = keys[ops == 3]
        up = keys[ops == 2]
        q = keys[ops == 0]
        assert len(np.unique(er)) == len(er) == int(0.2 * 4096)
        assert len(up) == int(0.3 * 4096)
        assert len(np.intersect1d(er, up)) == 0
        assert len(np.intersect1d(q, np.concatenate([er, up]))) == 0
    g1 = next(w.mixed_batches(1 << 14, 1 << 12, 1, workload_id=3))
    g2 = next(w.mixed_batches(1 << 14, 1 << 12, 1, workload_id=3))
    assert all(np.array_equal(g1[k], g2[k]) for k in g1)


def test_mixed_batches_give_hot_ranks_to_every_kind():
    """Draws are interleaved: a rank belongs, for one batch, to the kind of its
    first candidate, so the hottest ranks fall to queries, upserts and erases in
    proportion to their shares instead of all going to erases.  Over 40 batches
    the hottest rank (p ~ 4.9% of Zipf 0.99 draws over 2^16 ranks) is an upsert
    key in some batch and a query key in another, and in a batch where it is
    an upsert key it takes a large share of the upserts."""
    kinds, shares = set(), []
    for b in w.mixed_batches(1 << 16, 1 << 12, 40, workload_id=11):
        r0 = b["ranks"] == 0
        if r0.any():
            kinds.add(int(b["ops"][r0][0]))
            if b["ops"][r0][0] == 2:
                shares.append(w.hottest_upsert_share(b))
    assert {0, 2} <= kinds
    assert max(shares) > 0.05


def test_selection_sample_exact_size_and_uniform():
    """Algorithm S returns exactly k distinct increasing indices; every index is
    taken with probability k/n (checked on per-decile counts)."""
    n, k = 1_000_000, 300_000
    idx = w.sample_without_replacement(7, n, k)
    assert len(idx) == k and np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < n
    counts = np.bincount(idx * 10 // n, minlength=10)
    exp = k / 10
    assert np.all(np.abs(counts - exp) < 5 * np.sqrt(exp))
    assert len(w.sample_without_replacement(7, 10, 10)) == 10
    assert len(w.sample_without_replacement(7, 10, 0)) == 0


def test_aging_plan_slices():
    """Aging recipe (Section 6.5): every positive slice lies in the keys live through
    its iteration and misses that iteration's erase slice; negatives were never
    inserted; all keys are distinct."""
    p = w.aging_plan(1 << 14, iters=300)
    n0, s = p["n0"], p["s"]
    assert n0 == int(0.85 * (1 << 14)) and s == int(0.01 * n0)
    assert len(p["keys"]) == n0 + 300 * s and len(p["negs"]) == 300 * s
    assert len(np.unique(np.concatenate([p["keys"], p["negs"]]))) == len(p["keys"]) + len(p["negs"])
    for i, ps in enumerate(p["pos_start"].tolist()):
        assert (i + 1) * s <= ps and ps + s <= n0 + i * s

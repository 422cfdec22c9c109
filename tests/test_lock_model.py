"""The bucket-lock hand-off under a same-bucket storm, on the CPU (lock_model.py).

The storm: 2^16 tiles, each with one SUM upsert of one of 16 keys that share a
primary bucket, all resident at once, so all 2^16 wait on one lock word.  One
address of MI355X memory serves ~80 M requests per second.

* With test-and-set waiting (an atomic OR per attempt, with or without back-off)
  and with test-and-test-and-set waiting (coherent loads between atomics), the
  waiters keep one request each queued at the word, and every release waits
  behind them: ~0.8 ms per hand-off, tens of seconds per 2^16 batch (growing
  with the square of the waiters), which is the storm test that never finished.
* The ticket lock with proportional back-off keeps the queue short: the batch
  takes ~0.3 s, one critical section plus a few hundred nanoseconds per hand-off,
  whatever the number of waiters.
* The kernels' lock -- a byte per bucket, taken with one atomic when free, and a
  ticket queue for tiles that find it held -- hands off as fast as the ticket
  lock, with one poller per queue.

The old protocols are simulated at 2^16 / 128 waiters with the service rate
divided by 128 as well: while waiters keep requests queued, a hand-off costs
(queued requests) / rate, which this scaling preserves, so the full batch takes
128 times the scaled one (checked against the closed form).
"""
import pytest

import lock_model as lm

W = 1 << 16
MU = 80e6
SCALE = 128


@pytest.mark.parametrize("proto", ["spin", "spin_bo", "poll"])
def test_waiting_protocols_serialise_for_tens_of_seconds(proto):
    r = lm.simulate(proto, W // SCALE, mu=MU / SCALE)
    full = r.total_s * SCALE
    closed = lm.saturated_total(W, mu=MU)
    # each release queues behind the waiters' requests: ~W/mu per hand-off
    assert r.mean_handoff_s > 0.35 * (W / SCALE) / (MU / SCALE)
    assert full > 20.0, "a 2^16-op storm should take tens of seconds, got %.1f s" % full
    assert full > 0.9 * closed


def test_load_polling_is_no_better_than_atomic_spinning():
    spin = lm.simulate("spin", W // SCALE, mu=MU / SCALE)
    poll = lm.simulate("poll", W // SCALE, mu=MU / SCALE)
    # polls served at the same address rate queue exactly like the atomics did
    assert poll.total_s >= 0.9 * spin.total_s


def test_handoff_grows_with_waiters_for_test_and_set():
    small = lm.simulate("spin", 256)
    large = lm.simulate("spin", 2048)
    assert large.mean_handoff_s > 2.5 * small.mean_handoff_s


def test_ticket_lock_bounds_the_storm():
    r = lm.simulate("ticket", W, mu=MU)
    per = r.mean_handoff_s
    # one critical section (3 us) plus a round trip and a short poll delay
    assert per < 3e-6 + 2 * 0.5e-6 + 1.5e-6, per
    assert r.total_s < 0.5, r.total_s
    # FIFO: the longest wait is the whole queue once, never more
    assert r.max_wait_s <= r.total_s
    # the polls leave the address mostly idle (requests per second << mu)
    assert r.requests / r.total_s < 0.25 * MU


def test_ticket_handoff_does_not_depend_on_waiters():
    a = lm.simulate("ticket", 1 << 10)
    b = lm.simulate("ticket", 1 << 14)
    assert abs(a.mean_handoff_s - b.mean_handoff_s) < 0.1 * a.mean_handoff_s


@pytest.mark.parametrize("cs", [1e-6, 10e-6])
def test_ticket_handoff_tracks_the_critical_section(cs):
    r = lm.simulate("ticket", 1 << 12, cs=cs)
    assert cs < r.mean_handoff_s < cs + 2.5e-6


def test_grid_stride_tiles_each_hold_one_ticket_at_a_time():
    # 2^12 tiles with 4 operations each: FIFO per operation, 2^14 hand-offs
    r = lm.simulate("ticket", 1 << 12, ops_per_waiter=4)
    assert r.handoffs == 1 << 14
    assert r.mean_handoff_s < 3e-6 + 2.5e-6


def test_queued_lock_bounds_the_storm():
    """The kernels' lock (byte plus ticket queue) in a 2^14-tile storm: a
    hand-off costs one critical section plus about a round trip, as in the ticket
    lock, and the two words see far fewer requests than they could serve."""
    w = 1 << 14
    r = lm.simulate("queued", w, mu=MU)
    assert r.handoffs == w
    assert r.mean_handoff_s < 3e-6 + 2 * 0.5e-6 + 1.5e-6, r.mean_handoff_s
    assert r.requests / r.total_s < 0.25 * MU
    t = lm.simulate("ticket", w, mu=MU)
    assert abs(r.mean_handoff_s - t.mean_handoff_s) < 0.1 * t.mean_handoff_s


def test_queued_lock_uncontended_costs_one_atomic_and_one_store():
    r = lm.simulate("queued", 1)
    assert r.handoffs == 1 and r.requests == 2
    # a second tile arriving while the first holds the byte retries, then gets it
    r = lm.simulate("queued", 2, cs=1e-6)
    assert r.handoffs == 2


def test_queued_lock_without_retries_still_bounded():
    r = lm.simulate("queued", 1 << 12, spins=0)
    assert r.mean_handoff_s < 3e-6 + 2.5e-6

"""Discrete-event model of a bucket lock handed between many waiting tiles.

Test infrastructure (CPU only): it models how long a batch of same-bucket write
operations takes when every one of them must hold the bucket's lock (Section 4.1:
writers of one key are serialised by the lock of its primary bucket), under the
lock protocols the kernels have used.  The memory system is reduced to what
decides the outcome:

* every request to the lock word -- atomic read-modify-write, coherent load or
  store -- is served at the word's address one at a time, first come first
  served, `mu` requests per second (MI355X serves one address at ~80 M atomics/s);
* a request travels `lat` seconds to the address and its answer `lat` back;
* the holder spends `cs` seconds in the critical section (its bucket reads,
  combine and completion wait touch other addresses) and then stores the release.

Protocols (`proto`):

* "spin"     -- test-and-set: an atomic OR per attempt, retried at once;
* "spin_bo"  -- the same with a pause before each retry, doubling from 128 to
                8192 cycles (2.4 GHz);
* "poll"     -- test-and-test-and-set: after a failed attempt, pause as above,
                then read the word and try the atomic only when it reads free,
                or unconditionally on every 256th attempt;
* "ticket"   -- ticket lock with proportional back-off (Mellor-Crummey and
                Scott, ACM TOCS 9(1), 1991): one atomic add takes a ticket;
                the waiter whose ticket is d places behind the one being served
                reads the serving counter again after (d - 1) * unit + first
                seconds (at most max_gap + first); the release stores
                serving + 1.  Waiters never issue a
                read-modify-write while waiting.
* "queued"   -- the kernels' lock: a lock byte per bucket plus a ticket queue
                on a second word.  An atomic OR on the byte; when it finds the
                byte held, up to `spins` retries (pause as in "poll", a load,
                the OR when the load reads clear); then a ticket of the queue,
                waited for as in "ticket"; at the head of the queue, the OR
                every `first` seconds until it finds the byte clear (one
                tile per queue does this).  A tile that took the byte through
                the queue stores serving + 1 into the queue word at once, so
                the next head polls during its critical section; the release
                is a store to the byte.  The two words are separate addresses,
                each with its own service queue.

In the first three the waiters' own requests queue at the address ahead of the
holder's release, so each hand-off costs about (requests in the queue) / mu; in
the ticket lock the polls spread out in time and the queue stays short.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass

CLOCK_HZ = 2.4e9
PAUSE_CYCLES = 128      # one back-off step
PAUSE_MAX_STEPS = 64    # back-off ceiling: 64 steps = 8192 cycles
FORCE_EVERY = 256       # "poll": unconditional atomic every 256th attempt


@dataclass
class Result:
    total_s: float          # time until the last operation released the lock
    handoffs: int           # lock acquisitions
    mean_handoff_s: float   # total_s / handoffs
    requests: int           # requests served at the lock word
    max_wait_s: float       # longest wait of one operation for the lock
    peak_queue: int         # most requests waiting at the address at once


def simulate(proto: str, waiters: int, ops_per_waiter: int = 1, mu: float = 80e6, lat: float = 0.5e-6,
             cs: float = 3e-6, unit: float = 1e-6, first: float = 0.25e-6, max_gap: float = 10.48576e-3,
             spins: int = 4) -> Result:
    """Runs `waiters` tiles, each doing `ops_per_waiter` locked operations on one
    lock, all starting at time 0, and returns what it took."""
    assert proto in ("spin", "spin_bo", "poll", "ticket", "queued")
    svc = 1.0 / mu
    ev: list = []            # (time, seq, kind, tile, value)
    seq = 0
    server_free = {"byte": 0.0, "queue": 0.0}
    # lock word state, as the address sees it
    held = False
    ticket = 0
    serving = 0
    # per tile
    left = [ops_per_waiter] * waiters
    steps = [0] * waiters       # back-off steps
    attempt = [0] * waiters
    my_ticket = [0] * waiters
    wait_from = [0.0] * waiters
    via_queue = [False] * waiters
    # queue-length bookkeeping: completion times of requests in service order
    in_queue = {"byte": [], "queue": []}
    peak = 0
    served = 0
    acquisitions = 0
    last_release = 0.0
    max_wait = 0.0

    def push(t, kind, tile, value=0):
        nonlocal seq
        heapq.heappush(ev, (t, seq, kind, tile, value))
        seq += 1

    def request(t_issue, op, tile, value=0):
        # the request reaches the address at t_issue + lat
        push(t_issue + lat, "arrive:" + op, tile, value)

    def pause_of(tile):
        return steps[tile] * PAUSE_CYCLES / CLOCK_HZ

    def grow(tile):
        s = steps[tile]
        steps[tile] = 1 if s == 0 else min(2 * s, PAUSE_MAX_STEPS)

    def start_op(t, tile):
        steps[tile] = 0
        attempt[tile] = 0
        wait_from[tile] = t
        via_queue[tile] = False
        if proto == "ticket":
            request(t, "take", tile)
        else:
            attempt[tile] = 1
            request(t, "or", tile)

    def acquired(t, tile):
        nonlocal acquisitions, max_wait
        acquisitions += 1
        max_wait = max(max_wait, t - wait_from[tile])
        # a tile that came through the queue passes it on at once: the next
        # head then polls the byte during this critical section
        if proto == "queued" and via_queue[tile]:
            request(t, "pass", tile, my_ticket[tile] + 1)
        # critical section, then the release store
        request(t + cs, "release", tile, my_ticket[tile] + 1)

    for i in range(waiters):
        start_op(0.0, i)

    while ev:
        t, _, kind, tile, value = heapq.heappop(ev)
        if kind.startswith("arrive:"):
            op = kind[7:]
            addr = "queue" if (proto == "queued" and op in ("take", "poll", "pass")) else "byte"
            start = max(t, server_free[addr])
            server_free[addr] = start + svc
            served += 1
            iq = in_queue[addr]
            while iq and iq[0] <= t:
                heapq.heappop(iq)
            heapq.heappush(iq, server_free[addr])
            peak = max(peak, len(iq))
            done = server_free[addr]
            # the effect happens in service order, which is arrival order
            if op in ("or", "hor"):
                old = held
                held = True
                push(done + lat, "ans:" + op, tile, int(old))
            elif op in ("load", "hload"):
                push(done + lat, "ans:" + op, tile, int(held))
            elif op == "pass":
                serving = value
            elif op == "take":
                my_ticket[tile] = ticket
                ticket += 1
                push(done + lat, "ans:take", tile, serving)
            elif op == "poll":
                push(done + lat, "ans:poll", tile, serving)
            elif op == "release":
                if proto == "ticket":
                    serving = value
                else:
                    held = False
                last_release = max(last_release, done)
                left[tile] -= 1
                if left[tile] > 0:
                    # the tile's next operation starts once its release is issued;
                    # model it as issued right after the store
                    push(t - lat, "next", tile)
            continue
        if kind == "next":
            start_op(t, tile)
            continue
        if proto == "queued":
            if kind in ("ans:or", "ans:load"):
                if kind == "ans:or" and value == 0:
                    acquired(t, tile)
                elif kind == "ans:load" and value == 0:
                    request(t, "or", tile)
                elif attempt[tile] > spins:
                    request(t, "take", tile)
                else:
                    attempt[tile] += 1
                    grow(tile)
                    request(t + pause_of(tile), "load", tile)
            elif kind in ("ans:take", "ans:poll"):
                d = my_ticket[tile] - value
                if d == 0:
                    request(t, "hor", tile)
                else:
                    request(t + min((d - 1) * unit, max_gap) + first, "poll", tile)
            elif kind == "ans:hor":
                if value == 0:
                    via_queue[tile] = True
                    acquired(t, tile)
                else:
                    request(t + first, "hor", tile)
            continue
        if proto in ("spin", "spin_bo", "poll"):
            if kind == "ans:or":
                if value == 0:
                    acquired(t, tile)
                    continue
                if proto == "spin":
                    attempt[tile] += 1
                    request(t, "or", tile)
                    continue
                grow(tile)
                t_next = t + pause_of(tile)
                if proto == "spin_bo":
                    attempt[tile] += 1
                    request(t_next, "or", tile)
                else:
                    if attempt[tile] % FORCE_EVERY == 0:
                        attempt[tile] += 1
                        request(t_next, "or", tile)
                    else:
                        request(t_next, "load", tile)
            elif kind == "ans:load":
                if value == 0:
                    attempt[tile] += 1
                    request(t, "or", tile)
                else:
                    attempt[tile] += 1
                    grow(tile)
                    t_next = t + pause_of(tile)
                    if attempt[tile] % FORCE_EVERY == 0:
                        attempt[tile] += 1
                        request(t_next, "or", tile)
                    else:
                        request(t_next, "load", tile)
        else:
            if kind in ("ans:take", "ans:poll"):
                d = (my_ticket[tile] - value)
                if d == 0:
                    acquired(t, tile)
                else:
                    request(t + min((d - 1) * unit, max_gap) + first, "poll", tile)
    handoffs = acquisitions
    return Result(total_s=last_release, handoffs=handoffs,
                  mean_handoff_s=last_release / max(handoffs, 1), requests=served,
                  max_wait_s=max_wait, peak_queue=peak)


def saturated_total(waiters: int, mu: float = 80e6, lat: float = 0.5e-6, cs: float = 3e-6) -> float:
    """Closed form for the protocols whose waiters keep a request queued at the
    word: the k-th release waits behind the (waiters - k) requests of the tiles
    still waiting, so the batch takes sum_k ((waiters - k) / mu + cs + 2 lat)."""
    return sum((waiters - k) / mu + cs + 2 * lat for k in range(1, waiters + 1))

// Device primitives of HashWave for gfx950 (CDNA4, wave64).
//
//  * reserved key patterns and the tag rule (Section 5.1: a tag is the low 16
//    bits of the key);
//  * the hash rule: MurmurHash3's 64-bit finaliser of (key XOR salt).  The paper
//    only says double hashing uses two hash functions and power-of-two-choice two
//    candidate buckets (Section 2.2); one 64-bit mix supplies both here: its low
//    32 bits give the primary bucket, its high 32 bits the second hash;
//  * sub-wave tiles: T consecutive lanes of a 64-lane wave cooperate on one
//    operation (the paper's tiles, Section 3.2), with 64-bit ballots masked down
//    to the tile;
//  * coherent memory access.  The paper makes lock-free reads safe with
//    "morally strong" acquire loads and 128-bit release stores (Sections 3.1
//    and 4.2).  gfx950 keeps one L2 per XCD and these are not coherent with each
//    other for ordinary accesses; agent-scope atomic accesses (the `sc1` cache
//    policy) are.  Every access to table memory that can race is therefore an
//    agent-scope atomic access, and ordering between two of them is obtained by
//    waiting for the first to complete (`s_waitcnt vmcnt(0)`) before issuing the
//    second, instead of the full-L2 write-back / invalidate that a C++ release /
//    acquire fence costs on this chip (measured 3x slower for publishes).
//    Building with -DHW_STRICT_ORDER adds those fences back (for comparison);
//  * the lock of a bucket (Section 5.1: one lock per bucket in an external
//    array), a ticket lock taken by the tile's leader lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hw {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ patterns

template <typename K> struct Keys;
template <> struct Keys<uint64_t> {
  static constexpr uint64_t EMPTY = ~0ull;
  static constexpr uint64_t TOMB = ~0ull - 1;
  static constexpr uint64_t RESERVED = ~0ull - 2;  // slot claimed, key not yet published
  static constexpr uint64_t FIRST_INVALID = RESERVED;
};
template <> struct Keys<uint32_t> {
  // 32-bit slots publish key and value with one 64-bit operation, so no
  // reservation marker is needed.
  static constexpr uint32_t EMPTY = 0xFFFFFFFFu;
  static constexpr uint32_t TOMB = 0xFFFFFFFEu;
  static constexpr uint32_t RESERVED = 0xFFFFFFFEu;  // never written
  static constexpr uint32_t FIRST_INVALID = TOMB;
};

constexpr uint32_t TAG_EMPTY = 0xFFFF;
constexpr uint32_t TAG_TOMB = 0xFFFE;

__device__ __forceinline__ uint32_t tag_of(uint64_t key) {
  uint32_t t = (uint32_t)key & 0xFFFFu;
  return t >= TAG_TOMB ? t - 2 : t;
}

// ------------------------------------------------------------------ hashing

constexpr uint64_t HASH_SALT = 0x6a09e667f3bcc909ull;

__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

struct Hashed {
  uint32_t b1;  // primary bucket
  uint32_t h2;  // second hash (double-hashing step / alternate bucket)
};

__device__ __forceinline__ Hashed hash_key(uint64_t key, uint32_t bucket_mask) {
  uint64_t h = fmix64(key ^ HASH_SALT);
  return Hashed{(uint32_t)h & bucket_mask, (uint32_t)(h >> 32)};
}

// Iceberg hashing (Section 2.2, split of Section 5): buckets [0, nf) are the
// front yard, [nf, nf + nback) the backyard.  A 32-bit hash x is mapped to
// [0, n) as floor(x * n / 2^32) (one multiply-high), so neither region has to
// be a power of two.  The second backyard choice comes from an independently
// salted hash.
constexpr uint64_t HASH_SALT_B = 0xbb67ae8584caa73bull;

struct Yard {
  uint32_t front, back1, back2;
};

__device__ __forceinline__ uint32_t front_bucket(uint64_t key, uint32_t nf) {
  return __umulhi((uint32_t)fmix64(key ^ HASH_SALT), nf);
}

__device__ __forceinline__ Yard yard_of(uint64_t key, uint32_t nf, uint32_t nback) {
  const uint64_t h = fmix64(key ^ HASH_SALT);
  const uint64_t g = fmix64(key ^ HASH_SALT_B);
  return Yard{__umulhi((uint32_t)h, nf), nf + __umulhi((uint32_t)(h >> 32), nback),
              nf + __umulhi((uint32_t)g, nback)};
}

// ------------------------------------------------------------------ tiles

template <int T>
struct Tile {
  static_assert(T == 2 || T == 4 || T == 8 || T == 16 || T == 32 || T == 64, "tile");
  static constexpr uint64_t MASK = T == 64 ? ~0ull : ((1ull << T) - 1);
  uint32_t tl;  // lane within the tile
  uint32_t tb;  // first wave lane of the tile
  __device__ __forceinline__ Tile() {
    uint32_t lane = __lane_id();
    tl = lane & (T - 1);
    tb = lane & ~(uint32_t)(T - 1);
  }
  // Tile-local ballot: bit j set when lane j of this tile has p true.
  __device__ __forceinline__ uint64_t ballot(bool p) const { return (__ballot(p) >> tb) & MASK; }
  template <typename X>
  __device__ __forceinline__ X bcast(X x, uint32_t src) const {
    return __shfl(x, (int)(tb + src), 64);
  }
  __device__ __forceinline__ bool leader() const { return tl == 0; }
};

__device__ __forceinline__ int ffs64(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// ------------------------------------------------------------------ coherent access

// Waits until every earlier memory operation of this wave has completed.
__device__ __forceinline__ void wait_mem() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters untouched
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// 16-byte agent-coherent load (one global_load_dwordx4 with the sc1 policy).  A
// single 16-byte aligned access is served from one cache line in one request,
// so it returns a snapshot of the whole slot.
__device__ __forceinline__ u32x4 ld16(const void* p) {
  u32x4 r;
  asm volatile("global_load_dwordx4 %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" : "=v"(r) : "v"(p) : "memory");
  return r;
}

// 16-byte agent-coherent store (one global_store_dwordx4 with the sc1 policy):
// publishes a whole (key, value) slot in one request, the counterpart of the
// paper's 128-bit release store (Section 4.2).  Completion is awaited by the
// caller's next wait_mem().
__device__ __forceinline__ void st16(void* p, uint64_t lo, uint64_t hi) {
  u32x4 v;
  v.x = (uint32_t)lo;
  v.y = (uint32_t)(lo >> 32);
  v.z = (uint32_t)hi;
  v.w = (uint32_t)(hi >> 32);
  asm volatile("global_store_dwordx4 %0, %1, off sc1" : : "v"(p), "v"(v) : "memory");
}

template <typename X>
__device__ __forceinline__ X ld(const X* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename X>
__device__ __forceinline__ void st(X* p, X v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename X>
__device__ __forceinline__ X cas(X* p, X expected, X desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found (== the argument on success)
}

// Threads per block of every kernel that operates on a table (the per-tile
// lock-wait state below is sized by it).
constexpr int BLOCK = 256;

// ------------------------------------------------------------------ locks
//
// One lock byte per bucket in an external array (the paper keeps one lock bit
// per bucket there, Section 5.1; a byte makes the release a plain store): byte
// b % 4 of 32-bit word b / 4, nonzero while held.  The array is small (1 byte
// per 32 slots at bucket size 32: 8 MB for 2^28 slots), so most of it stays in
// the last-level cache between operations; per-bucket 64-bit ticket words would
// take 8 bytes per bucket and cost ~8% of a write-heavy batch's time in lock
// misses.
//
//  * Uncontended acquire: one atomic OR of the bucket's bit pattern into its
//    word.  It returns the word as it was: the byte was clear, so the lock is
//    ours.  Release: a byte store of 0, after every write of the critical
//    section has completed.
//  * Contended acquire (the OR found the byte set): the tile retries a few
//    times (LOCK_SPINS), each after a growing pause and only when the byte
//    reads clear -- a lock held by one other tile is usually free within a
//    critical section.  Then it queues on one of the table's lock queues,
//    ticket locks with proportional back-off
//    (Mellor-Crummey and Scott, ACM TOCS 9(1), 1991) in 64-bit words (high
//    half: next ticket; low half: ticket being served), queue b mod the queue
//    count.  A waiter d tickets behind the one being served reads the serving
//    half again after about d - 1 critical sections.  When its turn comes it is
//    the only queued tile of that queue: it tries the OR on its bucket's byte
//    every LOCK_FIRST_TICKS until the byte was clear, and then passes the queue
//    on at once (stores its ticket + 1), so that the next tile in line polls
//    during its critical section and takes the byte soon after the release.
//
// Why queue at all: one address of MI355X memory serves ~80 M requests per
// second.  If every waiter kept retrying the byte (test-and-set, even with
// back-off), its requests would queue at the lock word ahead of each release:
// with 2^16 tiles on one bucket a hand-off costs ~0.8 ms.  Queued waiters
// issue no read-modify-write and poll rarely; one tile per queue polls the
// byte, so a hand-off costs one critical section plus a short poll delay, in
// arrival order (new arrivals may take a free byte ahead of the queue during
// their few retries).
//
// A ticket cannot be given back, so a queued waiter never leaves the queue --
// except when its wait exceeds the table's time limit, a failure that the lock
// protocol itself never produces (a wait is bounded by the waiters ahead of it
// times one critical section).  Such an operation reports ST_TIMEOUT and sets
// the table's failure flag; every waiter that sees the flag gives up too, so the
// kernel still ends.  The abandoned ticket blocks its queue until the table is
// cleared; the lock bytes themselves are never abandoned (a tile holds one only
// inside its critical section).

// Wall clock of the chip: 100 MHz (s_memrealtime), low 32 bits.  They wrap
// every ~43 s; waits are compared as differences, and a wait never exceeds
// the time limit (at most 40 s).
__device__ __forceinline__ uint32_t now_ticks() { return (uint32_t)__builtin_amdgcn_s_memrealtime(); }

// Whether tick `t` has been reached at `now` (within 2^31 ticks of it).
__device__ __forceinline__ bool ticks_reached(uint32_t now, uint32_t t) { return (int32_t)(now - t) >= 0; }

constexpr uint32_t LOCK_UNIT_TICKS = 100;   // 1 us: assumed critical section per ticket ahead
constexpr uint32_t LOCK_FIRST_TICKS = 25;   // 0.25 us: the head of a queue tries its byte this often
constexpr uint32_t LOCK_FLAG_WORD = 32;     // ctrl word of the failure flag (its own 128-byte line)
constexpr uint32_t LOCK_QUEUES_MAX = 1u << 14;  // lock queues of a large table (128 KB)
constexpr uint32_t LOCK_SPINS = 4;               // retries of a held byte before queueing

// The lock array: bucket b's lock byte is byte b << shift of `words`.  The
// table picks the stride (1 << shift bytes, 1 to 8) so that the locks spread
// over at least 2^16 lines of 128 bytes while the array stays within 8 MiB,
// small enough to live mostly in the last-level cache: stride =
// clamp(2^23 / buckets, 1, 8).  Atomics on one line are served one after
// another at the memory side, so a small table whose lock bytes shared few
// lines made its writers queue there: at 2^26 slots (2^21 buckets, stride 4)
// the aging launches run 6% faster than with bytes, while 2^28-slot tables
// keep bytes (an 8-byte stride, 64 MiB, made their write phases 8% slower).
struct LockArray {
  uint32_t* words;
  uint32_t shift;
};

__device__ __forceinline__ uint64_t lock_at(const LockArray& L, uint32_t b) { return (uint64_t)b << L.shift; }
__device__ __forceinline__ uint32_t lock_pattern(uint64_t at) { return 1u << ((uint32_t)(at & 3u) * 8u); }

// Leader lane ORs bucket b's lock byte; every lane learns whether it was clear
// (then the tile holds the lock).
template <int T>
__device__ __forceinline__ bool try_lock(const LockArray& L, uint32_t b, const Tile<T>& tile) {
  const uint64_t at = lock_at(L, b);
  uint32_t old = 0;
  if (tile.leader()) {
#ifdef HW_STRICT_ORDER
    old = __hip_atomic_fetch_or(L.words + (at >> 2), lock_pattern(at), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
#else
    old = __hip_atomic_fetch_or(L.words + (at >> 2), lock_pattern(at), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#endif
  }
  return (tile.bcast(old, 0) & lock_pattern(at)) == 0;
}

// Whether bucket b's lock byte currently reads clear (a coherent load; no atomic).
template <int T>
__device__ __forceinline__ bool lock_looks_free(const LockArray& L, uint32_t b, const Tile<T>& tile) {
  uint32_t v = 0;
  if (tile.leader()) v = ld((const uint8_t*)L.words + lock_at(L, b));
  return tile.bcast(v, 0) == 0;
}

// Leader lane clears bucket b's lock byte.  The caller has waited for the
// critical section's writes (wait_mem), or uses the strict-order build.
__device__ __forceinline__ void release_try_lock(const LockArray& L, uint32_t b) {
#ifdef HW_STRICT_ORDER
  __hip_atomic_store((uint8_t*)L.words + lock_at(L, b), (uint8_t)0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
#else
  st((uint8_t*)L.words + lock_at(L, b), (uint8_t)0);
#endif
}

// Leader lane takes a ticket of lock queue q; every lane of the tile gets the
// word as it was (high half: our ticket; low half: the ticket being served).
template <int T>
__device__ __forceinline__ uint64_t take_ticket(uint64_t* queues, uint32_t q, const Tile<T>& tile) {
  uint64_t old = 0;
  if (tile.leader())
    old = __hip_atomic_fetch_add(queues + q, (uint64_t)1 << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return tile.bcast(old, 0);
}

// The ticket queue q is serving now (a coherent load; no atomic).
template <int T>
__device__ __forceinline__ uint32_t read_serving(uint64_t* queues, uint32_t q, const Tile<T>& tile) {
  uint32_t s = 0;
  if (tile.leader()) s = ld((const uint32_t*)(queues + q));
  return tile.bcast(s, 0);
}

// Passes queue q on to the ticket after `mine` (leader lane).
__device__ __forceinline__ void pass_queue(uint64_t* queues, uint32_t q, uint32_t mine) {
  st((uint32_t*)(queues + q), mine + 1);
}

// When a waiter d tickets behind should look again: after d - 1 assumed
// critical sections, but at least every LOCK_MAX_GAP_TICKS, so that the time
// limit is checked even far back in a long queue.
constexpr uint32_t LOCK_MAX_GAP_TICKS = 1u << 20;  // ~10 ms
__device__ __forceinline__ uint32_t next_look(uint32_t now, uint32_t d) {
  const uint32_t ahead = d - 1;
  const uint32_t gap = ahead < LOCK_MAX_GAP_TICKS / LOCK_UNIT_TICKS ? ahead * LOCK_UNIT_TICKS : LOCK_MAX_GAP_TICKS;
  return now + gap + LOCK_FIRST_TICKS;
}

// Cuckoo operations hold all three of their buckets' locks at once and take
// them with try_lock alone (no queue), so a tile that misses one releases the
// others and never waits while holding a lock.  A waiting tile reads the bytes
// first and tries the atomics only when they read clear (or on every 256th
// attempt).

// Back-off between failed try-lock attempts: a pause that doubles from 128
// cycles up to ~3.4 us (64 x 128 cycles).
struct Backoff {
  uint32_t n = 0;
  __device__ __forceinline__ void pause() {
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(2);
  }
  __device__ __forceinline__ void grow() { n = n ? (n < 64 ? 2 * n : 64) : 1; }
};

}  // namespace hw

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

// ------------------------------------------------------------------ locks
//
// One lock per bucket (the paper keeps one lock bit per bucket in an external
// array, Section 5.1), here a ticket lock with proportional back-off
// (Mellor-Crummey and Scott, ACM TOCS 9(1), 1991) in one 64-bit word per bucket:
// the high half is the next ticket, the low half the ticket being served, and
// the lock is free when the two are equal.
//
//  * Taking the lock is one 64-bit atomic add of 2^32: it returns the word as it
//    was, so an uncontended acquire costs one atomic, as a test-and-set would.
//    Carries out of the high half fall off the word; they never reach the low one.
//  * Releasing it is a 32-bit store of (own ticket + 1) into the low half, after
//    every write of the critical section has completed.  Only the holder writes
//    the low half.
//  * A waiter d tickets behind the one being served reads the low half again
//    after about d - 1 critical sections, so the waiters' reads stay spread out.
//
// Why not test-and-set: one address of MI355X memory serves ~80 M requests per
// second.  With test-and-set every waiter keeps an atomic (or, polling, a load)
// queued at the lock word, and each release waits behind all of them: with 2^16
// tiles on one bucket a hand-off costs ~0.8 ms.  Ticket waiters issue no
// read-modify-write and poll rarely, so a hand-off costs one critical section
// plus a short poll delay, and service is first come first served.
//
// A ticket cannot be given back, so a waiter never leaves the queue -- except
// when its wait exceeds the table's time limit, a failure that the lock protocol
// itself never produces (FIFO service bounds every wait by the waiters ahead of
// it times one critical section).  Such an operation reports ST_TIMEOUT and sets
// the table's failure flag; every waiter that sees the flag gives up too, so the
// kernel still ends.  The table's lock state is then undefined.

// Wall clock of the chip: 100 MHz (s_memrealtime).
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

constexpr uint32_t LOCK_UNIT_TICKS = 100;  // 1 us: assumed critical section per ticket ahead
constexpr uint32_t LOCK_FIRST_TICKS = 25;  // 0.25 us: next in line polls this often
constexpr uint32_t LOCK_FLAG_WORD = 32;    // ctrl word of the failure flag (its own 128-byte line)

__device__ __forceinline__ uint32_t* serving_of(uint64_t* locks, uint32_t b) { return (uint32_t*)(locks + b); }

// Leader lane takes a ticket for bucket b; every lane of the tile gets the
// word as it was (high half: our ticket; low half: the ticket being served).
template <int T>
__device__ __forceinline__ uint64_t take_ticket(uint64_t* locks, uint32_t b, const Tile<T>& tile) {
  uint64_t old = 0;
  if (tile.leader()) {
#ifdef HW_STRICT_ORDER
    old = __hip_atomic_fetch_add(locks + b, (uint64_t)1 << 32, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
#else
    old = __hip_atomic_fetch_add(locks + b, (uint64_t)1 << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#endif
  }
  return tile.bcast(old, 0);
}

// The ticket bucket b is serving now (a coherent load; no atomic).
template <int T>
__device__ __forceinline__ uint32_t read_serving(uint64_t* locks, uint32_t b, const Tile<T>& tile) {
  uint32_t s = 0;
  if (tile.leader()) {
#ifdef HW_STRICT_ORDER
    s = __hip_atomic_load(serving_of(locks, b), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
#else
    s = ld(serving_of(locks, b));
#endif
  }
  return tile.bcast(s, 0);
}

// When a waiter d tickets behind should look again: after d - 1 assumed
// critical sections, but at least every LOCK_MAX_GAP_TICKS, so that the time
// limit is checked even far back in a long queue.
constexpr uint64_t LOCK_MAX_GAP_TICKS = 1u << 20;  // ~10 ms
__device__ __forceinline__ uint64_t next_look(uint64_t now, uint32_t d) {
  const uint64_t gap = (uint64_t)(d - 1) * LOCK_UNIT_TICKS;
  return now + (gap < LOCK_MAX_GAP_TICKS ? gap : LOCK_MAX_GAP_TICKS) + LOCK_FIRST_TICKS;
}

// Releases bucket b, held with ticket `mine`, after every write of the critical
// section has completed.
template <int T>
__device__ __forceinline__ void unlock(uint64_t* locks, uint32_t b, uint32_t mine, const Tile<T>& tile) {
#ifdef HW_STRICT_ORDER
  if (tile.leader())
    __hip_atomic_store(serving_of(locks, b), mine + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
#else
  wait_mem();
  if (tile.leader()) st(serving_of(locks, b), mine + 1);
#endif
}

// Cuckoo operations hold all three of their buckets' locks at once and take
// them with try-locks (test-and-set on the low half of the lock word: bit 0 set
// = held; the high half stays 0), so a tile that misses one releases the others
// and never waits while holding a lock.  A waiting tile reads the word first and
// tries the atomic only when it reads free (or on every 256th attempt).

// Leader lane sets bucket b's lock bit; every lane learns whether it was free.
template <int T>
__device__ __forceinline__ bool try_lock(uint64_t* locks, uint32_t b, const Tile<T>& tile) {
  uint32_t old = 0;
  if (tile.leader())
    old = __hip_atomic_fetch_or(serving_of(locks, b), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (tile.bcast(old, 0) & 1u) == 0;
}

// Whether bucket b's try-lock currently reads free (a coherent load; no atomic).
template <int T>
__device__ __forceinline__ bool lock_looks_free(uint64_t* locks, uint32_t b, const Tile<T>& tile) {
  uint32_t w = 0;
  if (tile.leader()) w = ld(serving_of(locks, b));
  return tile.bcast(w, 0) == 0;
}

// Releases a try-lock (leader lane), after the caller has waited for the
// critical section's writes.
__device__ __forceinline__ void release_try_lock(uint64_t* locks, uint32_t b) { st(serving_of(locks, b), 0u); }

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

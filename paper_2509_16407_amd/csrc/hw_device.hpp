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
//  * the lock bit of a bucket (Section 5.1: one bit per bucket in an external
//    array), taken by the tile's leader lane with an atomic OR.
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
// One lock byte per bucket (the paper keeps one lock bit per bucket in an
// external array, Section 5.1).  Taking the lock is an atomic OR of the bucket's
// bit 0 on the 32-bit word holding four buckets' bytes; releasing it is a plain
// agent-coherent store of the byte, which cannot disturb the neighbours' bytes.
// A byte per bucket thus saves the atomic AND a bit-packed release needs: on this
// chip the atomic unit, not HBM bandwidth, bounds the write operations.

__device__ __forceinline__ uint32_t lock_bit(uint32_t b) { return 1u << ((b & 3) * 8); }

// Leader lane sets bucket b's lock; every lane of the tile learns whether the
// lock was free.  On success the caller owns the bucket until unlock().
template <int T>
__device__ __forceinline__ bool try_lock(uint32_t* locks, uint32_t b, const Tile<T>& tile) {
  const uint32_t bit = lock_bit(b);
  uint32_t old = 0;
  if (tile.leader()) {
#ifdef HW_STRICT_ORDER
    old = __hip_atomic_fetch_or(locks + (b >> 2), bit, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
#else
    old = __hip_atomic_fetch_or(locks + (b >> 2), bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#endif
  }
  old = tile.bcast(old, 0);
  return (old & bit) == 0;
}

// Backoff between failed lock attempts: a pause that doubles from 128 cycles up
// to ~3.4 us (64 x 128 cycles), about one critical section.  Waiters poll the
// lock with loads between attempts, so short pauses cost no atomics; long pauses
// would leave a released lock idle while its waiters sleep.
struct Backoff {
  uint32_t n = 0;
  __device__ __forceinline__ void pause() {
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(2);
  }
  __device__ __forceinline__ void grow() { n = n ? (n < 64 ? 2 * n : 64) : 1; }
};

// Whether bucket b's lock currently reads clear (a coherent load; no atomic).
// Waiting tiles poll with this and only try the atomic when it looks clear, so
// the lock word's atomic unit -- which serves one address at ~80 M operations/s
// on MI355X -- is left to the holders.
template <int T>
__device__ __forceinline__ bool lock_looks_free(const uint32_t* locks, uint32_t b, const Tile<T>& tile) {
  uint32_t w = 0;
  if (tile.leader()) w = ld((const uint8_t*)locks + b);
  return tile.bcast(w, 0) == 0;
}

// Releases bucket b after every write of the critical section has completed.
template <int T>
__device__ __forceinline__ void unlock(uint32_t* locks, uint32_t b, const Tile<T>& tile) {
#ifdef HW_STRICT_ORDER
  if (tile.leader())
    __hip_atomic_fetch_and(locks + (b >> 2), ~lock_bit(b), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
#else
  wait_mem();
  if (tile.leader()) st((uint8_t*)locks + b, (uint8_t)0);
#endif
}

}  // namespace hw

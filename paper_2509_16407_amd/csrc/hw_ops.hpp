// Per-operation device logic of the four open-addressing designs.
//
// One operation is carried out by one tile of T lanes (Section 3.2).  Upsert and
// erase hold the lock bit of the key's primary bucket for their whole critical
// section (Section 4.1: with associativity above one, two writers of the same
// key must be serialised or the key can be duplicated).  Query takes no lock
// (Section 4.2).  A new key's slot is first claimed atomically -- by a
// compare-and-swap of its key word to the reservation marker, or of its tag in
// the fingerprint designs (the tag is written first, Section 4.3, Fig. 3) -- then
// the value is stored and the key is published last.  A reader that matches the
// key therefore also sees its value.  Keys never move once stored (stability,
// Section 2.1), which makes the in-place combine of an upsert safe.
//
// Probing (Section 2.2):
//  * double hashing visits buckets b1, b1+s, b1+2s, ... (s odd) and stops at the
//    first bucket holding an empty slot: the empty pattern never comes back,
//    because erase leaves a tombstone, so a key is never stored past such a
//    bucket.  Inserts take the first free (empty or tombstone) slot on the way;
//  * power-of-two-choice inserts into the less loaded of its two buckets (ties
//    to the primary), or straight into the primary while that holds fewer than
//    3/4 of its slots ("shortcutting").  Erase returns slots to empty.
//  * iceberg hashing keeps a key in its single front-yard bucket while that has
//    a free slot, and otherwise in the less loaded of its two backyard buckets
//    (ties to the first).  The front bucket's lock serialises the key's writers;
//    front-yard slots are only ever claimed under that lock.  Erase returns
//    slots to empty.
//
// Shortcut safety (a reading; the paper is silent): after an erase, a key can sit
// in its alternate bucket while its primary has dropped below 3/4, and the
// shortcut would then insert a second copy.  A per-table flag records that an
// erase has happened; the shortcut is used only while it is clear.  An erase
// sets it (and waits for the store) before removing anything; an insert reads it
// after reading the primary bucket, so whoever observes a removal also observes
// the flag.  Iceberg uses the same flag: until an erase, a front bucket's fill
// only grows, so a key was placed in the backyard only while its front bucket
// was full and stays full; an insert that finds a free front slot claims it
// without looking at the backyard, and a query that finds one stops there.
#pragma once

#include "hw_device.hpp"

namespace hw {

enum : uint8_t { ST_MISS = 0, ST_DONE = 1, ST_EXISTED = 2, ST_FULL = 3, ST_INVALID = 4, ST_TIMEOUT = 5 };
enum : int { C_SUM = 0, C_KEEP = 1, C_REPLACE = 2, C_MIN = 3, C_MAX = 4 };
enum : int { OP_QUERY = 0, OP_INSERT = 1, OP_UPSERT = 2, OP_ERASE = 3 };
// Chaining's overflow pool is split into this many partitions, each with its own
// allocation counter in a 128-byte line of its own (POOL_CTR_STRIDE 32-bit
// words apart): atomics to one line are served one after another, so counters
// sharing lines would serialise the allocations.  Bucket b draws from
// partition b mod POOL_PARTS first.
constexpr uint32_t POOL_PARTS = 1024;
constexpr uint32_t POOL_CTR_STRIDE = 32;

// Striped accumulators of hot keys (tables that merge duplicates and never
// erase).  A key that a merge window saw more than once is combined into one
// of HOT_ROWS rows (chosen by the wave) of HOT_M entries, keyed by the key's
// slot, instead of into its value word; a flush after the launch folds every
// entry into the table.  A hot key thus costs one atomic per row and launch at
// its value word instead of one per window.  Entry: tag word (slot + 1, the
// combine in bits 56..63; 0 = free) and accumulator word, in two arrays.
constexpr uint32_t HOT_ROWS = 32;
constexpr uint32_t HOT_M = 128;
constexpr uint32_t HOT_N = HOT_ROWS * HOT_M;
constexpr int HOT_PROBE = 8;

enum : int { D_DOUBLE = 0, D_DOUBLE_M = 1, D_P2 = 2, D_P2_M = 3, D_ICEBERG = 4, D_ICEBERG_M = 5, D_CHAINING = 6,
             D_CUCKOO = 7 };

// Device view of one table (passed by value to kernels).
struct TableDev {
  void* slots;           // (key, value) pairs, bucket-major
  uint32_t* tagw;        // 16-bit tags viewed as 32-bit words; null without tags
  LockArray locks;       // one lock byte per bucket, at a stride (hw_device.hpp)
  uint64_t* lockq;       // lock queues: lockq_mask + 1 ticket words
  uint32_t* ctrl;        // ctrl[0]: an erase has happened (power-of-two-choice, iceberg);
                         // ctrl[LOCK_FLAG_WORD]: a lock wait timed out
  uint32_t bucket_mask;  // buckets - 1 (a power of two minus one)
  uint32_t nb_front;     // iceberg: front-yard buckets [0, nb_front); chaining: buckets
  uint32_t nb_back;      // iceberg: backyard buckets [nb_front, nb_front + nb_back)
  uint32_t pool_nodes;   // chaining: overflow nodes after the buckets' first nodes
  uint32_t* pool_ctr;    // chaining: POOL_PARTS allocation counters, one per line
  uint32_t probe_cap;    // double hashing: most buckets visited
  uint32_t shortcut;     // power-of-two-choice shortcut enabled
  uint32_t no_erase;     // table never erases: present keys are combined without the lock
  uint32_t aggregate;    // merge duplicate keys of a write batch first (hw_agg.hpp)
  uint32_t lock_limit;   // longest wait for a bucket lock, in 100 MHz ticks
  uint32_t lockq_mask;   // lock queues - 1 (a power of two minus one); bucket b queues on b & lockq_mask
  uint64_t* hot_tag;     // HOT_N entry tags, or null (see HOT_ROWS)
  uint64_t* hot_acc;     // HOT_N accumulators
  unsigned long long* probe_ctr;  // instrumented builds: PROBE_STRIPES query probe counters; else null
};

// Query probe counters of instrumented builds (-DHW_INSTRUMENT): PROBE_STRIPES
// stripes of 16 words, one 128-byte line each, picked by wave; word PC_BUCKET
// counts the unique 128-byte lines of buckets, tag buckets and chain nodes a
// query reads, PC_SLOT the key/value slots it reads after a tag match, PC_QUERY
// the queries; PC_WRITE the upserts that search under the lock and PC_VISIT the
// buckets those searches look at before deciding (rescans after a lost claim
// not counted).  Other builds compile the counting out.
constexpr uint32_t PROBE_STRIPES = 64;
enum : int { PC_BUCKET = 0, PC_SLOT = 1, PC_QUERY = 2, PC_WRITE = 3, PC_VISIT = 4 };

__device__ __forceinline__ void probe_add(const TableDev& tv, int word, uint64_t n) {
#ifdef HW_INSTRUMENT
  if (!tv.probe_ctr || n == 0) return;
  const uint32_t stripe = (blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) % PROBE_STRIPES;
  __hip_atomic_fetch_add(tv.probe_ctr + stripe * 16 + word, (unsigned long long)n, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
#else
  (void)tv; (void)word; (void)n;
#endif
}

// BSP_: the phased (bulk-synchronous) variant used to measure what concurrency
// costs (Section 6.4): writes take no lock and queries read with plain cacheable
// loads.  Correct only for phased use: the writes of one launch are to distinct
// keys and no launch mixes writes and reads of one key.
template <typename K_, int DESIGN_, int B_, int T_, bool BSP_ = false>
struct Cfg {
  using K = K_;
  static constexpr int DESIGN = DESIGN_;
  static constexpr bool BSP = BSP_;
  static constexpr bool TAGS = DESIGN == D_DOUBLE_M || DESIGN == D_P2_M || DESIGN == D_ICEBERG_M;
  static constexpr bool DOUBLE = DESIGN == D_DOUBLE || DESIGN == D_DOUBLE_M;
  static constexpr bool ICEBERG = DESIGN == D_ICEBERG || DESIGN == D_ICEBERG_M;
  static constexpr bool CHAIN = DESIGN == D_CHAINING;  // B = 7 slots per node, T = 8
  static constexpr bool CUCKOO = DESIGN == D_CUCKOO;   // three candidate buckets
  static constexpr int B = B_;
  static constexpr int T = T_;
  static constexpr int SLOT_BYTES = 2 * (int)sizeof(K);
  static constexpr int SPL = 16 / SLOT_BYTES;   // slots per lane per 16-byte load
  static constexpr int STEPS = B / (T * SPL);   // slot loads per bucket (no tags)
  static constexpr int TPL = B / T;             // tags per lane (tag designs)
  static_assert(CHAIN || TAGS || (B % (T * SPL) == 0 && STEPS >= 1), "bucket must be a multiple of the tile's load");
  static_assert(!CHAIN || (B == 7 && T == 8 && sizeof(K_) == 8), "chain node: 7 slots and a link, one per lane");
  static_assert(!TAGS || TPL == 1 || TPL == 2 || TPL == 4 || TPL == 8 || TPL == 16, "tags per lane");
};

template <typename K>
struct BucketScan {
  int32_t hit;         // slot (within the bucket) holding the key, -1 if none
  int32_t free;        // first free slot (empty or tombstone), -1 if none
  uint32_t fill;       // slots not free (valid only when hit < 0)
  bool has_empty;      // bucket holds an empty slot
  K val;               // value at `hit`
  uint64_t free_word;  // as read: the free slot's tag word (tag designs), its key
                       // (64-bit slots) or its whole slot (32-bit slots); the
                       // expected value of the claiming compare-and-swap
};

template <class C>
struct Ops {
  using K = typename C::K;
  static constexpr int B = C::B, T = C::T, SPL = C::SPL, TPL = C::TPL;
  static constexpr K EMPTY = Keys<K>::EMPTY;
  static constexpr K TOMB = Keys<K>::TOMB;

  __device__ static __forceinline__ K* key_ptr(const TableDev& tv, uint64_t s) {
    return (K*)tv.slots + 2 * s;
  }
  __device__ static __forceinline__ K* val_ptr(const TableDev& tv, uint64_t s) {
    return (K*)tv.slots + 2 * s + 1;
  }

  // Loads: agent-coherent, or plain cacheable ones (PLAIN: queries of the phased
  // variant only -- they never retry, so a stale line cannot hold them up).
  template <bool PLAIN>
  __device__ static __forceinline__ u32x4 rd16(const void* p) {
    if constexpr (PLAIN) return *(const u32x4*)p;
    else return ld16(p);
  }
  template <bool PLAIN, typename X>
  __device__ static __forceinline__ X rd(const X* p) {
    if constexpr (PLAIN) return *p;
    else return ld(p);
  }

  // Read of one whole slot in one access.
  template <bool PLAIN = false>
  __device__ static __forceinline__ void load_slot(const TableDev& tv, uint64_t s, K& k, K& v) {
    if constexpr (sizeof(K) == 8) {
      u32x4 w = rd16<PLAIN>(key_ptr(tv, s));
      k = (uint64_t)w.x | ((uint64_t)w.y << 32);
      v = (uint64_t)w.z | ((uint64_t)w.w << 32);
    } else {
      uint64_t w = rd<PLAIN>((const uint64_t*)key_ptr(tv, s));
      k = (uint32_t)w;
      v = (uint32_t)(w >> 32);
    }
  }

  // Unique 128-byte lines of a slot bucket read in its first `steps` tile-width
  // steps (buckets start on a line).
  static constexpr uint32_t lines_after(int steps) {
    return (uint32_t)(((uint64_t)steps * T * SPL * 2 * sizeof(K) + 127) / 128);
  }

  // Sum over the tile of a per-lane count.
  __device__ static __forceinline__ uint32_t tile_sum(uint32_t x) {
#pragma unroll
    for (int o = 1; o < T; o <<= 1) x += __shfl_xor(x, o, 64);
    return x;
  }

  // ---------------------------------------------------------------- scans

  // Scans bucket b for `key` (FIND) and gathers its free/empty/fill state.
  // Slot designs read the bucket one tile-width at a time and stop at a hit;
  // tag designs read the tag bucket once and check each tag match against the
  // full key (tags are lossy, Section 4.3).
  // COUNT: a query's scan, counted by instrumented builds (probe_add).
  template <bool FIND, bool PLAIN = false, bool COUNT = false>
  __device__ static BucketScan<K> scan(const TableDev& tv, const Tile<T>& tile, uint32_t b, K key,
                                       uint32_t tag) {
    BucketScan<K> r;
    r.hit = -1;
    r.free = -1;
    r.fill = 0;
    r.has_empty = false;
    r.val = 0;
    r.free_word = 0;
    const uint64_t base = (uint64_t)b * B;
    if constexpr (!C::TAGS) {
      uint32_t occ = 0;
#pragma unroll 1
      for (int s = 0; s < C::STEPS; ++s) {
        const uint64_t first = base + (uint64_t)s * T * SPL + (uint64_t)tile.tl * SPL;
        K k[SPL], v[SPL];
        if constexpr (SPL == 1) {
          load_slot<PLAIN>(tv, first, k[0], v[0]);
        } else {
          u32x4 w = rd16<PLAIN>(key_ptr(tv, first));
          k[0] = (K)w.x; v[0] = (K)w.y; k[1] = (K)w.z; v[1] = (K)w.w;
        }
        uint32_t m_hit = 0, m_free = 0, m_empty = 0;
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
          m_hit |= (uint32_t)(FIND && k[j] == key) << j;
          m_free |= (uint32_t)(k[j] == EMPTY || k[j] == TOMB) << j;
          m_empty |= (uint32_t)(k[j] == EMPTY) << j;
        }
        if constexpr (FIND) {
          uint64_t lh = tile.ballot(m_hit != 0);
          if (lh) {
            int src = ffs64(lh);
            uint32_t mm = tile.bcast(m_hit, src);
            int j = __ffs(mm) - 1;
            K vv = v[0];
            if constexpr (SPL == 2) vv = j ? v[1] : v[0];
            r.val = tile.bcast(vv, src);
            r.hit = s * T * SPL + src * SPL + j;
            if constexpr (COUNT) {
              if (tile.leader()) probe_add(tv, PC_BUCKET, lines_after(s + 1));
            }
            return r;
          }
        }
        if (r.free < 0) {
          uint64_t lanes = tile.ballot(m_free != 0);
          if (lanes) {
            int src = ffs64(lanes);
            int j = __ffs(tile.bcast(m_free, src)) - 1;
            uint64_t word;
            if constexpr (SPL == 1) word = (uint64_t)k[0];
            else word = j ? ((uint64_t)k[1] | ((uint64_t)v[1] << 32)) : ((uint64_t)k[0] | ((uint64_t)v[0] << 32));
            r.free_word = tile.bcast(word, src);
            r.free = s * T * SPL + src * SPL + j;
          }
        }
        r.has_empty |= tile.ballot(m_empty != 0) != 0;
        occ += (uint32_t)__popc(~m_free & ((1u << SPL) - 1));
      }
      r.fill = tile_sum(occ);
      if constexpr (COUNT) {
        if (tile.leader()) probe_add(tv, PC_BUCKET, lines_after(C::STEPS));
      }
    } else {
      uint32_t tw[(TPL + 1) / 2];
      const uint32_t* tp = tv.tagw + (base + (uint64_t)tile.tl * TPL) / 2;
      if constexpr (TPL == 16) {
        u32x4 a = rd16<PLAIN>(tp), c = rd16<PLAIN>(tp + 4);
        tw[0] = a.x; tw[1] = a.y; tw[2] = a.z; tw[3] = a.w;
        tw[4] = c.x; tw[5] = c.y; tw[6] = c.z; tw[7] = c.w;
      } else if constexpr (TPL == 8) {
        u32x4 a = rd16<PLAIN>(tp);
        tw[0] = a.x; tw[1] = a.y; tw[2] = a.z; tw[3] = a.w;
      } else if constexpr (TPL == 4) {
        uint64_t a = rd<PLAIN>((const uint64_t*)tp);
        tw[0] = (uint32_t)a; tw[1] = (uint32_t)(a >> 32);
      } else if constexpr (TPL == 2) {
        tw[0] = rd<PLAIN>(tp);
      } else {
        tw[0] = rd<PLAIN>((const uint16_t*)tv.tagw + base + tile.tl);
      }
      if constexpr (COUNT) {
        if (tile.leader()) probe_add(tv, PC_BUCKET, (2 * B + 127) / 128);
      }
      uint32_t m_hit = 0, m_free = 0, m_empty = 0;
#pragma unroll
      for (int i = 0; i < TPL; ++i) {
        uint32_t t = (tw[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
        m_hit |= (uint32_t)(t == tag) << i;
        m_free |= (uint32_t)(t >= TAG_TOMB) << i;
        m_empty |= (uint32_t)(t == TAG_EMPTY) << i;
      }
      if constexpr (FIND) {
        uint64_t lanes = tile.ballot(m_hit != 0);
        while (lanes) {
          int src = ffs64(lanes);
          lanes &= lanes - 1;
          uint32_t mm = tile.bcast(m_hit, src);
          while (mm) {
            int j = __ffs(mm) - 1;
            mm &= mm - 1;
            K k, v;
            load_slot<PLAIN>(tv, base + src * TPL + j, k, v);
            if constexpr (COUNT) {
              if (tile.leader()) probe_add(tv, PC_SLOT, 1);
            }
            if (k == key) {
              r.hit = src * TPL + j;
              r.val = v;
              return r;
            }
          }
        }
      }
      {
        uint64_t lanes = tile.ballot(m_free != 0);
        if (lanes) {
          int src = ffs64(lanes);
          int j = __ffs(tile.bcast(m_free, src)) - 1;
          uint32_t word = tw[0];
#pragma unroll
          for (int i = 1; i < (TPL + 1) / 2; ++i)
            if ((j >> 1) == i) word = tw[i];
          if constexpr (TPL == 1) {
            // one tag per lane: the 32-bit word pairs this lane's tag with its neighbour's
            const uint32_t other = __shfl_xor(tw[0], 1, 64) & 0xFFFFu;
            word = (tile.tl & 1) ? ((tw[0] & 0xFFFFu) << 16) | other : (other << 16) | (tw[0] & 0xFFFFu);
          }
          r.free_word = tile.bcast(word, src);
          r.free = src * TPL + j;
        }
      }
      r.has_empty = tile.ballot(m_empty != 0) != 0;
      constexpr uint32_t lane_bits = TPL == 32 ? 0xFFFFFFFFu : ((1u << TPL) - 1);
      r.fill = tile_sum((uint32_t)__popc(~m_free & lane_bits));
    }
    return r;
  }

  // ---------------------------------------------------------------- writes

  // Claims slot s for a new key and publishes (key, value).  `seen` is the
  // free slot's word as the scan read it (see BucketScan::free_word): the
  // compare-and-swap expects it, and retries with whatever it finds for as
  // long as the slot stays free.  `excl`: the slot's bucket is written only by
  // holders of the lock this operation holds (an iceberg front-yard bucket), so
  // the slot stays free and is taken with plain stores -- tag first, then the
  // slot -- without the compare-and-swap.  Leader lane only touches memory;
  // the result is broadcast.
  __device__ static bool claim(const TableDev& tv, const Tile<T>& tile, uint64_t s, uint64_t seen,
                               K key, K val, uint32_t tag, bool excl = false) {
    bool ok = false;
    if (excl) {
      if (tile.leader()) {
        if constexpr (C::TAGS) st((uint16_t*)tv.tagw + s, (uint16_t)tag);
        publish(tv, s, key, val);
      }
      return true;
    }
    if (tile.leader()) {
      if constexpr (C::TAGS) {
        uint32_t* wp = tv.tagw + (s >> 1);
        const uint32_t sh = (uint32_t)(s & 1) * 16;
        uint32_t cur = (uint32_t)seen;
        while (((cur >> sh) & 0xFFFFu) >= TAG_TOMB) {
          uint32_t want = (cur & ~(0xFFFFu << sh)) | (tag << sh);
          uint32_t old = cas(wp, cur, want);
          if (old == cur) { ok = true; break; }
          cur = old;
        }
        if (ok) publish(tv, s, key, val);
      } else if constexpr (sizeof(K) == 8) {
        K* kp = key_ptr(tv, s);
        K cur = (K)seen;
        while (cur == EMPTY || cur == TOMB) {
          K old = cas(kp, cur, (K)Keys<K>::RESERVED);
          if (old == cur) { ok = true; break; }
          cur = old;
        }
        if (ok) publish(tv, s, key, val);
      } else {
        uint64_t* sp = (uint64_t*)key_ptr(tv, s);
        uint64_t cur = seen;
        const uint64_t want = (uint64_t)key | ((uint64_t)val << 32);
        while ((K)cur == EMPTY || (K)cur == TOMB) {
          uint64_t old = cas(sp, cur, want);
          if (old == cur) { ok = true; break; }
          cur = old;
        }
      }
    }
    return tile.bcast((uint32_t)ok, 0) != 0;
  }

  // Writes (key, value) into a slot this operation has claimed.  64-bit slots:
  // one 16-byte store, or with -DHW_SPLIT_PUBLISH the value first and the key
  // once the value store has completed.  32-bit slots (tag designs): one 8-byte
  // store.
  __device__ static __forceinline__ void publish(const TableDev& tv, uint64_t s, K key, K val) {
    if constexpr (sizeof(K) == 8) {
#ifdef HW_SPLIT_PUBLISH
      st(val_ptr(tv, s), val);
      wait_mem();
      st(key_ptr(tv, s), key);
#else
      st16(key_ptr(tv, s), (uint64_t)key, (uint64_t)val);
#endif
    } else {
      st((uint64_t*)key_ptr(tv, s), (uint64_t)key | ((uint64_t)val << 32));
    }
  }

  // Upsert callback applied to a present key (Section 5.1).
  __device__ static void combine_at(const TableDev& tv, const Tile<T>& tile, uint64_t s, K val,
                                    int combine) {
    if (tile.leader()) {
      K* vp = val_ptr(tv, s);
      switch (combine) {
        case C_SUM: __hip_atomic_fetch_add(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
        case C_REPLACE: st(vp, val); break;
        case C_MIN: __hip_atomic_fetch_min(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
        case C_MAX: __hip_atomic_fetch_max(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
        default: break;
      }
    }
  }

  // Removes the key in slot s: the key word first (the linearisation point),
  // then, once that store has completed, the tag (a reading; the paper does not
  // state the erase order).  The tag is freed with a 16-bit store: it leaves the
  // other tag of its 32-bit word alone, and an inserter's compare-and-swap on that
  // word that races with it simply fails and retries.
  __device__ static void remove(const TableDev& tv, const Tile<T>& tile, uint64_t s, uint32_t tag) {
    if (tile.leader()) {
      st(key_ptr(tv, s), C::DOUBLE ? TOMB : EMPTY);
      if constexpr (C::TAGS) {
        wait_mem();
        st((uint16_t*)tv.tagw + s, (uint16_t)(C::DOUBLE ? TAG_TOMB : TAG_EMPTY));
      }
    }
  }

  // Claims the first free slot of bucket b (as found by scan `r`), rescanning
  // after lost races.  Returns the slot or -1 when the bucket is full.
  __device__ static int64_t claim_in_bucket(const TableDev& tv, const Tile<T>& tile, uint32_t b,
                                            BucketScan<K> r, K key, K val, uint32_t tag,
                                            bool excl = false) {
    while (r.free >= 0) {
      const uint64_t s = (uint64_t)b * B + r.free;
      if (claim(tv, tile, s, r.free_word, key, val, tag, excl)) return (int64_t)s;
      r = scan<false>(tv, tile, b, key, tag);
    }
    return -1;
  }

  // ---------------------------------------------------------------- operations

  // A key's buckets.  b1 is the bucket whose lock guards the key (primary; the
  // front bucket for iceberg); h2 the second hash (double-hashing step,
  // power-of-two-choice alternate) or, for iceberg, the first backyard choice;
  // b3 the second backyard choice.
  struct Home {
    uint32_t b1, h2, b3;
  };

  __device__ static __forceinline__ Home home_of(const TableDev& tv, K key) {
    if constexpr (C::CHAIN) {
      return Home{front_bucket((uint64_t)key, tv.nb_front), 0u, 0u};
    } else if constexpr (C::CUCKOO) {
      const Hashed h = hash_key((uint64_t)key, tv.bucket_mask);
      const uint32_t g = (uint32_t)fmix64((uint64_t)key ^ HASH_SALT_B);
      return Home{h.b1, h.h2 & tv.bucket_mask, g & tv.bucket_mask};
    } else if constexpr (C::ICEBERG) {
      const Yard y = yard_of((uint64_t)key, tv.nb_front, tv.nb_back);
      return Home{y.front, y.back1, y.back2};
    } else {
      const Hashed h = hash_key((uint64_t)key, tv.bucket_mask);
      return Home{h.b1, h.h2, 0u};
    }
  }

  // The erase flag, read by the leader and broadcast.
  __device__ static __forceinline__ bool erased(const TableDev& tv, const Tile<T>& tile) {
    const uint32_t e = tile.leader() ? ld(tv.ctrl) : 0u;
    return tile.bcast(e, 0) != 0;
  }

  __device__ static __forceinline__ uint32_t step_of(const TableDev& tv, const Home& h) {
    return (h.h2 & tv.bucket_mask) | 1u;
  }

  // ---------------------------------------------------------------- cuckoo
  //
  // Three-way bucketed cuckoo hashing (Sections 2.2 and 5; concurrent insertion
  // after libcuckoo): a key lives in one of three buckets, and keys move between
  // their buckets to make room, so the table is not stable and every operation,
  // queries included, holds the locks of all its key's buckets (Section 6.4
  // notes CuckooHT's locked queries).  Locks are taken in ascending bucket order
  // with try-locks only: a tile that misses one releases what it holds and backs
  // off, so no tile waits while holding a lock (no deadlock, and no waiting on
  // a tile of its own wave).  Every write to a bucket happens under its lock,
  // so slots are written with plain stores.
  //
  // Making room: with the locks released, a random walk looks for a path of
  // displacements ending in a bucket with an empty slot (reads only); the path
  // is then carried out backwards, each move under the locks of its two buckets
  // after checking that nothing changed: the key is copied into the empty slot,
  // the copy completes, then the old slot is emptied.  Any failed check drops the
  // path and the insert starts over; after CUCKOO_MAX_ROUNDS fruitless rounds it
  // reports FULL.
  static constexpr int CUCKOO_MAX_PATH = 6;
  static constexpr uint32_t CUCKOO_MAX_ROUNDS = 64;

  struct Cands {
    uint32_t c[3];  // distinct candidate buckets, in hash order
    uint32_t s[3];  // the same, ascending (lock order)
    uint32_t n;
  };

  __device__ static Cands cuckoo_cands(const Home& h) {
    Cands r;
    r.c[0] = h.b1;
    r.n = 1;
    if (h.h2 != h.b1) r.c[r.n++] = h.h2;
    if (h.b3 != h.b1 && h.b3 != h.h2) r.c[r.n++] = h.b3;
    r.s[0] = r.c[0];
    r.s[1] = r.c[1];
    r.s[2] = r.c[2];
    for (uint32_t i = 1; i < r.n; ++i)
      for (uint32_t j = i; j > 0 && r.s[j - 1] > r.s[j]; --j) {
        const uint32_t t = r.s[j];
        r.s[j] = r.s[j - 1];
        r.s[j - 1] = t;
      }
    return r;
  }

  __device__ static __forceinline__ void release(const TableDev& tv, uint32_t b, const Tile<T>& tile) {
    if (tile.leader()) release_try_lock(tv.locks, b);
  }

  __device__ static bool try_lock_all(const TableDev& tv, const Tile<T>& tile, const Cands& c) {
    for (uint32_t i = 0; i < c.n; ++i) {
      if (!try_lock(tv.locks, c.s[i], tile)) {
        for (uint32_t j = 0; j < i; ++j) release(tv, c.s[j], tile);
        return false;
      }
    }
    return true;
  }

  __device__ static bool all_look_free(const TableDev& tv, const Tile<T>& tile, const Cands& c) {
    bool f = true;
    for (uint32_t i = 0; i < c.n; ++i) f &= lock_looks_free(tv.locks, c.s[i], tile);
    return f;
  }

  // Releases all of c's locks; after writes, once those have completed.
  __device__ static void unlock_all(const TableDev& tv, const Tile<T>& tile, const Cands& c, bool wrote) {
    if (wrote) wait_mem();
    for (uint32_t i = 0; i < c.n; ++i) release(tv, c.s[i], tile);
  }

  __device__ static __forceinline__ uint64_t next_rand(uint64_t& st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }

  // Moves key x from slot j of bucket `from` to an empty slot of bucket `to`
  // (two of x's buckets) under both locks; false if a lock was busy or the
  // buckets changed since the path was found.
  __device__ static bool cuckoo_move(const TableDev& tv, const Tile<T>& tile, uint32_t from, uint32_t j, K x,
                                     uint32_t to) {
    const uint32_t lo = from < to ? from : to, hi = from < to ? to : from;
    if (!try_lock(tv.locks, lo, tile)) return false;
    if (!try_lock(tv.locks, hi, tile)) {
      release(tv, lo, tile);
      return false;
    }
    K k, v;
    load_slot(tv, (uint64_t)from * B + j, k, v);
    const BucketScan<K> r = scan<false>(tv, tile, to, x, 0u);
    const bool ok = k == x && r.free >= 0;
    if (ok && tile.leader()) {
      publish(tv, (uint64_t)to * B + r.free, x, v);
      wait_mem();  // the copy is complete before the original goes
      st(key_ptr(tv, (uint64_t)from * B + j), EMPTY);
    }
    if (ok) wait_mem();
    release(tv, hi, tile);
    release(tv, lo, tile);
    return ok;
  }

  // One attempt at freeing a slot in one of c's buckets (see above).
  __device__ static void cuckoo_make_room(const TableDev& tv, const Tile<T>& tile, const Cands& c, uint64_t& rng) {
    uint32_t pb[CUCKOO_MAX_PATH + 1], pj[CUCKOO_MAX_PATH];
    K px[CUCKOO_MAX_PATH];
    uint32_t b = c.c[next_rand(rng) % c.n];
    int len = -1;
    for (int d = 0; d < CUCKOO_MAX_PATH; ++d) {
      pb[d] = b;
      const uint32_t j = (uint32_t)(next_rand(rng) % B);
      K x, v;
      load_slot(tv, (uint64_t)b * B + j, x, v);
      if (x >= Keys<K>::FIRST_INVALID) return;  // a free (or changing) slot: retry the insert
      const Cands cx = cuckoo_cands(home_of(tv, x));
      if (cx.n < 2) return;
      uint32_t alt = cx.c[next_rand(rng) % cx.n];
      if (alt == b) alt = cx.c[(alt == cx.c[0]) ? 1 : 0];
      pj[d] = j;
      px[d] = x;
      const BucketScan<K> r = scan<false>(tv, tile, alt, x, 0u);
      if (r.free >= 0) {
        pb[d + 1] = alt;
        len = d + 1;
        break;
      }
      b = alt;
    }
    for (int i = len - 1; i >= 0; --i)
      if (!cuckoo_move(tv, tile, pb[i], pj[i], px[i], pb[i + 1])) return;
  }

  __device__ static uint8_t cuckoo_upsert(const TableDev& tv, const Tile<T>& tile, K key, K val, int combine) {
    const Cands c = cuckoo_cands(home_of(tv, key));
    uint64_t rng = (uint64_t)key ^ 0x2545F4914F6CDD1Dull;
    uint8_t status = ST_FULL;
    bool done = false;
    uint32_t rounds = 0, attempt = 0;
    Backoff bo;
    while (!done) {
      bo.pause();
      const bool go = (attempt & 255) == 0 || all_look_free(tv, tile, c);
      ++attempt;
      int outcome = 0;  // 0: locks busy, 1: finished, 2: all buckets full
      if (go && try_lock_all(tv, tile, c)) {
        int64_t free_slot = -1;
        bool wrote = false;
        for (uint32_t i = 0; i < c.n && outcome == 0; ++i) {
          const BucketScan<K> r = scan<true>(tv, tile, c.c[i], key, 0u);
          if (r.hit >= 0) {
            combine_at(tv, tile, (uint64_t)c.c[i] * B + r.hit, val, combine);
            wrote = combine != C_KEEP;
            status = ST_EXISTED;
            outcome = 1;
          } else if (free_slot < 0 && r.free >= 0) {
            free_slot = (int64_t)c.c[i] * B + r.free;
          }
        }
        if (outcome == 0) {
          if (free_slot >= 0) {
            if (tile.leader()) publish(tv, (uint64_t)free_slot, key, val);
            wrote = true;
            status = ST_DONE;
            outcome = 1;
          } else {
            outcome = 2;
          }
        }
        unlock_all(tv, tile, c, wrote);
      }
      if (outcome == 1) {
        done = true;
      } else if (outcome == 2) {
        if (++rounds > CUCKOO_MAX_ROUNDS) done = true;  // status stays FULL
        else cuckoo_make_room(tv, tile, c, rng);
      } else {
        bo.grow();
      }
    }
    return status;
  }

  // Locked search (cuckoo queries and erases): the key's slot or -1.
  __device__ static uint8_t cuckoo_locked(const TableDev& tv, const Tile<T>& tile, K key, bool erase, K* out) {
    const Cands c = cuckoo_cands(home_of(tv, key));
    Backoff bo;
    uint32_t attempt = 0;
    while (true) {
      bo.pause();
      const bool go = (attempt & 255) == 0 || all_look_free(tv, tile, c);
      ++attempt;
      if (go && try_lock_all(tv, tile, c)) {
        uint8_t st_ = ST_MISS;
        for (uint32_t i = 0; i < c.n; ++i) {
          const BucketScan<K> r = scan<true>(tv, tile, c.c[i], key, 0u);
          if (r.hit >= 0) {
            if (erase) remove(tv, tile, (uint64_t)c.c[i] * B + r.hit, 0u);
            else *out = r.val;
            st_ = ST_DONE;
            break;
          }
        }
        unlock_all(tv, tile, c, erase && st_ == ST_DONE);
        return st_;
      }
      bo.grow();
    }
  }

  // ---------------------------------------------------------------- chaining
  //
  // A chain node is one 128-byte line (Section 5): lanes 0..6 of the 8-lane tile
  // read one (key, value) slot each, lane 7 the link unit, whose value word holds
  // the next node's index (all-ones: none).  Nodes 0 .. nb-1 are the buckets'
  // first nodes; the overflow pool follows.  Every write into a chain happens
  // under its bucket's lock, so slots are taken with plain stores; a new node is
  // filled before the link to it is published, so lock-free readers never see a
  // half-built node.
  static constexpr uint64_t NIL = ~0ull;

  struct NodeScan {
    int32_t hit, free;  // slot of the key / first empty slot in this node, or -1
    uint64_t next;      // next node, or NIL
    K val;
  };

  template <bool PLAIN = false>
  __device__ static __forceinline__ NodeScan scan_node(const TableDev& tv, const Tile<T>& tile, uint64_t node,
                                                       K key) {
    const u32x4 w = rd16<PLAIN>((const uint64_t*)tv.slots + 16 * node + 2 * tile.tl);
    const uint64_t k = (uint64_t)w.x | ((uint64_t)w.y << 32);
    const uint64_t v = (uint64_t)w.z | ((uint64_t)w.w << 32);
    const bool slot = tile.tl < 7;
    const uint64_t mh = tile.ballot(slot && k == (uint64_t)key);
    const uint64_t mf = tile.ballot(slot && k == (uint64_t)EMPTY);
    NodeScan r;
    r.hit = mh ? ffs64(mh) : -1;
    r.free = mf ? ffs64(mf) : -1;
    r.next = tile.bcast(v, 7);
    r.val = r.hit >= 0 ? (K)tile.bcast(v, (uint32_t)r.hit) : (K)0;
    return r;
  }

  // Most nodes a chain can have: a walk that reaches this many has found a cycle,
  // which the table never builds; the bound only keeps a damaged image from
  // holding a tile forever.
  __device__ static __forceinline__ uint32_t max_chain(const TableDev& tv) { return tv.pool_nodes + 1; }

  template <bool COUNT = false>
  __device__ static int64_t chain_find(const TableDev& tv, const Tile<T>& tile, uint32_t b, K key, K* val) {
    uint64_t node = b;
    for (uint32_t i = 0; i < max_chain(tv) && node != NIL; ++i) {
      const NodeScan r = scan_node<C::BSP>(tv, tile, node, key);
      if constexpr (COUNT) {
        if (tile.leader()) probe_add(tv, PC_BUCKET, 1);
      }
      if (r.hit >= 0) { *val = r.val; return (int64_t)(node * 8 + r.hit); }
      node = r.next;
    }
    return -1;
  }

  // Takes a node from the overflow pool for bucket b.  The pool is split into
  // POOL_PARTS partitions with a counter each, and bucket b draws from partition
  // b mod POOL_PARTS first: allocations spread over a thousand lines instead of
  // funnelling through one (a single line serves tens of millions of atomics
  // per second).  A spent partition sends the tile on to the next ones;
  // a counter is read before its atomic, so spent partitions cost no atomics.
  // NIL when the whole pool is spent.
  __device__ static uint64_t alloc_node(const TableDev& tv, const Tile<T>& tile, uint32_t b) {
    uint64_t got = NIL;
    if (tile.leader()) {
      const uint32_t psz = (tv.pool_nodes + POOL_PARTS - 1) / POOL_PARTS;
      for (uint32_t q = 0; q < POOL_PARTS; ++q) {
        const uint32_t p = (b + q) % POOL_PARTS;
        const uint32_t lo = p * psz;
        const uint32_t hi = lo + psz < tv.pool_nodes ? lo + psz : tv.pool_nodes;
        uint32_t* ctr = tv.pool_ctr + p * POOL_CTR_STRIDE;
        if (lo >= hi || ld(ctr) >= hi - lo) continue;
        const uint32_t i = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (i < hi - lo) { got = (uint64_t)tv.nb_front + lo + i; break; }
      }
    }
    return tile.bcast(got, 0);
  }

  __device__ static uint8_t upsert_chain_locked(const TableDev& tv, const Tile<T>& tile, const Home& h, K key,
                                                K val, int combine) {
    uint64_t node = h.b1, last = h.b1, free_slot = NIL;
    for (uint32_t i = 0; i < max_chain(tv) && node != NIL; ++i) {
      const NodeScan r = scan_node(tv, tile, node, key);
      if (r.hit >= 0) {
        combine_at(tv, tile, node * 8 + r.hit, val, combine);
        return ST_EXISTED;
      }
      if (free_slot == NIL && r.free >= 0) free_slot = node * 8 + r.free;
      last = node;
      node = r.next;
    }
    if (free_slot != NIL) {
      if (tile.leader()) publish(tv, free_slot, key, val);
      return ST_DONE;
    }
    const uint64_t fresh = alloc_node(tv, tile, h.b1);
    if (fresh == NIL) return ST_FULL;
    if (tile.leader()) {
      publish(tv, fresh * 8, key, val);  // the pool node is empty: slot 0
      wait_mem();                        // node content before the link to it
      st((uint64_t*)tv.slots + 16 * last + 15, fresh);
    }
    return ST_DONE;
  }

  __device__ static uint8_t erase_chain_locked(const TableDev& tv, const Tile<T>& tile, const Home& h, K key) {
    uint64_t node = h.b1;
    for (uint32_t i = 0; i < max_chain(tv) && node != NIL; ++i) {
      const NodeScan r = scan_node(tv, tile, node, key);
      if (r.hit >= 0) {
        if (tile.leader()) st(key_ptr(tv, node * 8 + r.hit), EMPTY);
        return ST_DONE;
      }
      node = r.next;
    }
    return ST_MISS;
  }

  // Lock-free search (Section 4.2): the slot holding `key`, or -1.  Value in *val.
  template <bool COUNT = false>
  __device__ static int64_t find(const TableDev& tv, const Tile<T>& tile, const Home& h, K key,
                                 uint32_t tag, K* val) {
    if constexpr (C::CHAIN) {
      return chain_find<COUNT>(tv, tile, h.b1, key, val);
    } else if constexpr (C::ICEBERG) {
      BucketScan<K> r = scan<true, C::BSP, COUNT>(tv, tile, h.b1, key, tag);
      if (r.hit >= 0) { *val = r.val; return (int64_t)h.b1 * B + r.hit; }
      // The flag is read after the front bucket: a free slot seen there that an
      // erase made is seen together with the flag the erase set first.
      if (r.free >= 0 && !erased(tv, tile)) return -1;
      r = scan<true, C::BSP, COUNT>(tv, tile, h.h2, key, tag);
      if (r.hit >= 0) { *val = r.val; return (int64_t)h.h2 * B + r.hit; }
      if (h.b3 != h.h2) {
        r = scan<true, C::BSP, COUNT>(tv, tile, h.b3, key, tag);
        if (r.hit >= 0) { *val = r.val; return (int64_t)h.b3 * B + r.hit; }
      }
      return -1;
    } else if constexpr (C::DOUBLE) {
      const uint32_t step = step_of(tv, h);
      uint32_t b = h.b1;
      for (uint32_t i = 0; i < tv.probe_cap; ++i, b = (b + step) & tv.bucket_mask) {
        BucketScan<K> r = scan<true, C::BSP, COUNT>(tv, tile, b, key, tag);
        if (r.hit >= 0) { *val = r.val; return (int64_t)b * B + r.hit; }
        if (r.has_empty) break;
      }
      return -1;
    } else {
      BucketScan<K> r = scan<true, C::BSP, COUNT>(tv, tile, h.b1, key, tag);
      if (r.hit >= 0) { *val = r.val; return (int64_t)h.b1 * B + r.hit; }
      const uint32_t b2 = h.h2 & tv.bucket_mask;
      if (b2 != h.b1) {
        r = scan<true, C::BSP, COUNT>(tv, tile, b2, key, tag);
        if (r.hit >= 0) { *val = r.val; return (int64_t)b2 * B + r.hit; }
      }
      return -1;
    }
  }

  // Combines val into the hot-key accumulator of slot s in row `row` (leader lane
  // only): the entry whose tag is (s + 1, combine), claimed by a compare-and-swap
  // if free; after HOT_PROBE taken entries, into the value word directly.  An
  // accumulator starts at 0, which every combine accepts as its identity: sums
  // add, maxima keep the largest value, minima keep the largest complement.
  __device__ static void hot_add(const TableDev& tv, uint64_t s, K val, int combine, uint32_t row) {
    const uint64_t tagged = (s + 1) | ((uint64_t)combine << 56);
    uint64_t* trow = tv.hot_tag + (uint64_t)row * HOT_M;
    uint64_t* arow = tv.hot_acc + (uint64_t)row * HOT_M;
    uint32_t j = (uint32_t)fmix64(s);
    for (int p = 0; p < HOT_PROBE; ++p, ++j) {
      const uint32_t i = j & (HOT_M - 1);
      uint64_t cur = ld(trow + i);
      if (cur == 0) cur = cas(trow + i, (uint64_t)0, tagged);  // 0: claimed
      if (cur != 0 && cur != tagged) continue;
      if (combine == C_SUM)
        __hip_atomic_fetch_add(arow + i, (uint64_t)val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else if (combine == C_MAX)
        __hip_atomic_fetch_max(arow + i, (uint64_t)val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_max(arow + i, (uint64_t)(K)~val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    K* vp = val_ptr(tv, s);
    if (combine == C_SUM) __hip_atomic_fetch_add(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (combine == C_MAX) __hip_atomic_fetch_max(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_fetch_min(vp, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // Runs cs() under bucket b's lock (hw_device.hpp) and returns its status, or
  // ST_TIMEOUT when the wait outlasted the table's limit or another waiter of
  // the table reported such a failure (checked on every 16th look).
  //
  // The tile tries the lock byte; if it is held, it retries up to LOCK_SPINS
  // times, each after a growing pause and only when the byte reads clear (a
  // lock held by one other tile is usually free again within a critical
  // section).  Then it takes a ticket of the bucket's lock queue, looks at the
  // serving counter at times spaced by its place in the queue, and once at the
  // head tries the byte until it takes it, then passes the queue on.
  //
  // Lanes of a wave run in lockstep, so every tile of the wave goes round this
  // loop until the last one is done.  The critical section comes first in each
  // round: a tile that holds the lock runs it and releases before any waiting
  // step of the round, so its lock is not held across other tiles' pauses and
  // round trips (the retries, the most common wait, come last in the round),
  // and tiles of one wave that wait on each other cannot deadlock.
  template <class F>
  __device__ static uint8_t locked(const TableDev& tv, const Tile<T>& tile, uint32_t b, F&& cs) {
    // The waiting state (ticket, start of the wait, next look, retries or
    // looks) lives in LDS, one slot per tile of the block: it is touched only
    // while waiting, and kept out of registers it leaves them to the critical
    // section inlined below.  Every lane of a tile writes the same values.
    __shared__ uint32_t wait_lds[4 * (BLOCK / T)];
    uint32_t* const ws = wait_lds + 4 * (threadIdx.x / T);
    enum : uint32_t { HAVE = 0, RETRY = 1, QUEUED = 2, HEAD = 3, DONE = 4 };
    uint32_t stage = try_lock(tv.locks, b, tile) ? HAVE : RETRY;
    if (stage == RETRY) ws[3] = 0;
    uint8_t status = ST_TIMEOUT;
    while (stage != DONE) {
      if (stage == HAVE) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // critical-section accesses after the lock's
        status = cs();
#ifndef HW_STRICT_ORDER
        wait_mem();  // every write of the critical section has completed
#endif
        if (tile.leader()) release_try_lock(tv.locks, b);
        stage = DONE;
      } else if (stage != RETRY) {
        const uint32_t now = now_ticks();
        if (ticks_reached(now, ws[2])) {
          const uint32_t mine = ws[0];
          uint32_t look = ws[2];
          if (stage == QUEUED) {
            const uint32_t served = read_serving(tv.lockq, b & tv.lockq_mask, tile);
            if (served == mine) stage = HEAD;
            else look = next_look(now, mine - served);
          }
          if (stage == HEAD) {
            if (try_lock(tv.locks, b, tile)) {
              stage = HAVE;
              if (tile.leader()) pass_queue(tv.lockq, b & tv.lockq_mask, mine);  // the next head polls during our section
            } else {
              look = now + LOCK_FIRST_TICKS;
            }
          }
          const uint32_t looks = ws[3] + 1;
          if (stage != HAVE && (now - ws[1] > tv.lock_limit || ((looks & 15) == 0 && lock_failed(tv, tile)))) {
            if (tile.leader()) st(tv.ctrl + LOCK_FLAG_WORD, 1u);
            stage = DONE;  // status stays ST_TIMEOUT
          }
          ws[2] = look;
          ws[3] = looks;
        } else {
          __builtin_amdgcn_s_sleep(2);
        }
      } else {
        // retry: a pause of 2^retries steps of 128 cycles, then a look at the
        // byte and the OR if it reads clear
        const uint32_t retries = ws[3];
        for (uint32_t i = 0; i < (1u << retries); ++i) __builtin_amdgcn_s_sleep(2);
        if (lock_looks_free(tv.locks, b, tile) && try_lock(tv.locks, b, tile)) {
          stage = HAVE;
        } else if (retries + 1 == LOCK_SPINS) {
          const uint64_t w = take_ticket(tv.lockq, b & tv.lockq_mask, tile);
          const uint32_t mine = (uint32_t)(w >> 32), since = now_ticks();
          stage = (uint32_t)w == mine ? HEAD : QUEUED;
          ws[0] = mine;
          ws[1] = since;
          ws[2] = stage == HEAD ? since : next_look(since, mine - (uint32_t)w);
          ws[3] = 0;
        } else {
          ws[3] = retries + 1;
        }
      }
    }
    return status;
  }

  // Whether a lock wait of this table has timed out (leader reads, broadcast).
  __device__ static __forceinline__ bool lock_failed(const TableDev& tv, const Tile<T>& tile) {
    const uint32_t f = tile.leader() ? ld(tv.ctrl + LOCK_FLAG_WORD) : 0u;
    return tile.bcast(f, 0) != 0;
  }

  // Upsert: lock primary, find or insert, unlock.  Status per hwave.h.
  //
  // In a table that never erases, a slot once filled keeps its key for good
  // (stability, Section 2.1), so a present key is combined in place without the
  // lock (as the paper does for sparse tensor contraction, Section 6.7); only an
  // absent key queues for the lock, whose holder then finds or inserts it.
  // hot_row >= 0 (a key that a merge window met more than once): in a table with
  // hot-key accumulators, where a present key's slot is fixed for good, a
  // SUM/MIN/MAX combine of a present key goes to row hot_row of the accumulators
  // instead of the value word.
  __device__ static uint8_t upsert(const TableDev& tv, const Tile<T>& tile, K key, K val,
                                   int combine, int hot_row = -1) {
    return write(tv, tile, key, val, combine, false, hot_row);
  }

  // Upsert (erase false) or erase (erase true) of one key: the write path both
  // share.  Callers pass a constant `erase`, so the other kind's code folds
  // away.
  __device__ static uint8_t write(const TableDev& tv, const Tile<T>& tile, K key, K val, int combine, bool erase,
                                  int hot_row = -1) {
    if (key >= Keys<K>::FIRST_INVALID || (erase && tv.no_erase)) return ST_INVALID;
    if constexpr (C::CUCKOO) {
      K unused;
      return erase ? cuckoo_locked(tv, tile, key, true, &unused) : cuckoo_upsert(tv, tile, key, val, combine);
    }
    const Home h = home_of(tv, key);
    const uint32_t tag = C::TAGS ? tag_of((uint64_t)key) : 0u;
    if constexpr (!C::DOUBLE) {
      // an erase marks the table first: the two-choice shortcut and iceberg's
      // front-yard rule hold only while nothing was ever erased
      if (erase && tile.leader() && ld(tv.ctrl) == 0) {
        st(tv.ctrl, 1u);
        wait_mem();
      }
    }
    // Phased chaining keeps its write locks: appending a node is not safe for
    // two writers of one chain (only its queries differ, Table 1's phased column).
    if constexpr (C::BSP && !C::CHAIN) {
      if (erase) return erase_locked(tv, tile, h, key, tag);
      if constexpr (C::ICEBERG)
        return upsert_iceberg_locked(tv, tile, h, key, val, tag, combine);
      else if constexpr (C::DOUBLE)
        return upsert_double_locked(tv, tile, h, key, val, tag, combine);
      else
        return upsert_p2_locked(tv, tile, h, key, val, tag, combine);
    }
    if (!erase && tv.no_erase) {
      K cur;
      const int64_t s = find(tv, tile, h, key, tag, &cur);
      if (s >= 0) {
        if (hot_row >= 0 && tv.hot_tag && (combine == C_SUM || combine == C_MIN || combine == C_MAX)) {
          if (tile.leader()) hot_add(tv, (uint64_t)s, val, combine, (uint32_t)hot_row);
        } else {
          combine_at(tv, tile, (uint64_t)s, val, combine);
        }
        return ST_EXISTED;
      }
    }
    return locked(tv, tile, h.b1, [&]() -> uint8_t {
      if (erase) return erase_locked(tv, tile, h, key, tag);
      if constexpr (C::CHAIN)
        return upsert_chain_locked(tv, tile, h, key, val, combine);
      else if constexpr (C::ICEBERG)
        return upsert_iceberg_locked(tv, tile, h, key, val, tag, combine);
      else if constexpr (C::DOUBLE)
        return upsert_double_locked(tv, tile, h, key, val, tag, combine);
      else
        return upsert_p2_locked(tv, tile, h, key, val, tag, combine);
    });
  }

  __device__ static uint8_t upsert_double_locked(const TableDev& tv, const Tile<T>& tile,
                                                 const Home& h, K key, K val, uint32_t tag,
                                                 int combine) {
    const uint32_t step = step_of(tv, h);
    BucketScan<K> first_free;
    first_free.free = -1;
    uint32_t free_i = 0, free_b = 0;
    uint32_t b = h.b1;
    if (tile.leader()) probe_add(tv, PC_WRITE, 1);
    for (uint32_t i = 0; i < tv.probe_cap; ++i, b = (b + step) & tv.bucket_mask) {
      BucketScan<K> r = scan<true>(tv, tile, b, key, tag);
      if (tile.leader()) probe_add(tv, PC_VISIT, 1);
      if (r.hit >= 0) {
        combine_at(tv, tile, (uint64_t)b * B + r.hit, val, combine);
        return ST_EXISTED;
      }
      if (first_free.free < 0 && r.free >= 0) {
        first_free = r;
        free_i = i;
        free_b = b;
      }
      if (r.has_empty) break;
    }
    // Absent: claim the first free slot met, moving on along the sequence when
    // other writers take the free slots first.
    if (first_free.free < 0) return ST_FULL;
    b = free_b;
    BucketScan<K> r = first_free;
    for (uint32_t i = free_i; i < tv.probe_cap; ++i, b = (b + step) & tv.bucket_mask) {
      if (i != free_i) r = scan<false>(tv, tile, b, key, tag);
      if (claim_in_bucket(tv, tile, b, r, key, val, tag) >= 0) return ST_DONE;
    }
    return ST_FULL;
  }

  __device__ static uint8_t upsert_p2_locked(const TableDev& tv, const Tile<T>& tile,
                                             const Home& h, K key, K val, uint32_t tag,
                                             int combine) {
    const uint32_t b1 = h.b1;
    const uint32_t b2 = h.h2 & tv.bucket_mask;
    if (tile.leader()) probe_add(tv, PC_WRITE, 1);
    BucketScan<K> r1 = scan<true>(tv, tile, b1, key, tag);
    if (tile.leader()) probe_add(tv, PC_VISIT, 1);
    if (r1.hit >= 0) {
      combine_at(tv, tile, (uint64_t)b1 * B + r1.hit, val, combine);
      return ST_EXISTED;
    }
    if (tv.shortcut && 4 * r1.fill < 3 * (uint32_t)B && !erased(tv, tile)) {
      // After a lost race the shortcut is judged again on the bucket as it now
      // is: concurrent claims may have taken it past 3/4.
      while (4 * r1.fill < 3 * (uint32_t)B && r1.free >= 0) {
        if (claim(tv, tile, (uint64_t)b1 * B + r1.free, r1.free_word, key, val, tag)) return ST_DONE;
        r1 = scan<false>(tv, tile, b1, key, tag);
      }
    }
    if (b2 == b1) {
      return claim_in_bucket(tv, tile, b1, r1, key, val, tag) >= 0 ? ST_DONE : ST_FULL;
    }
    BucketScan<K> r2 = scan<true>(tv, tile, b2, key, tag);
    if (tile.leader()) probe_add(tv, PC_VISIT, 1);
    if (r2.hit >= 0) {
      combine_at(tv, tile, (uint64_t)b2 * B + r2.hit, val, combine);
      return ST_EXISTED;
    }
    return claim_less_loaded(tv, tile, b1, r1, b2, r2, key, val, tag);
  }

  // Claims a slot in the less loaded of buckets ba and bb (ties to ba), judging
  // the choice again after every lost race, so that operations deciding at the
  // same moment on the same pair do not all pile into one bucket.  ST_FULL when
  // both are full.
  __device__ static uint8_t claim_less_loaded(const TableDev& tv, const Tile<T>& tile, uint32_t ba,
                                              BucketScan<K> ra, uint32_t bb, BucketScan<K> rb, K key,
                                              K val, uint32_t tag) {
    for (;;) {
      const bool second = rb.fill < ra.fill;
      BucketScan<K>& rp = second ? rb : ra;
      BucketScan<K>& ro = second ? ra : rb;
      const uint32_t bp = second ? bb : ba, bo = second ? ba : bb;
      if (rp.free >= 0) {
        if (claim(tv, tile, (uint64_t)bp * B + rp.free, rp.free_word, key, val, tag)) return ST_DONE;
        rp = scan<false>(tv, tile, bp, key, tag);
      } else if (ro.free >= 0) {
        if (claim(tv, tile, (uint64_t)bo * B + ro.free, ro.free_word, key, val, tag)) return ST_DONE;
        ro = scan<false>(tv, tile, bo, key, tag);
      } else {
        return ST_FULL;
      }
    }
  }

  // Iceberg insert under the front bucket's lock: the front bucket if it has a
  // free slot (after checking the backyard for the key once an erase has
  // happened), else the less loaded backyard choice, ties to the first.
  __device__ static uint8_t upsert_iceberg_locked(const TableDev& tv, const Tile<T>& tile,
                                                  const Home& h, K key, K val, uint32_t tag,
                                                  int combine) {
    if (tile.leader()) probe_add(tv, PC_WRITE, 1);
    BucketScan<K> rf = scan<true>(tv, tile, h.b1, key, tag);
    if (tile.leader()) probe_add(tv, PC_VISIT, 1);
    if (rf.hit >= 0) {
      combine_at(tv, tile, (uint64_t)h.b1 * B + rf.hit, val, combine);
      return ST_EXISTED;
    }
    // Front-yard slots are claimed only under this lock: plain stores suffice
    // (not in the phased variant, which takes no lock).
    if (rf.free >= 0 && !erased(tv, tile)) {
      if (claim_in_bucket(tv, tile, h.b1, rf, key, val, tag, !C::BSP) >= 0) return ST_DONE;
      rf = scan<false>(tv, tile, h.b1, key, tag);  // phased variant: lost the slot to another key
    }
    BucketScan<K> r1 = scan<true>(tv, tile, h.h2, key, tag);
    if (tile.leader()) probe_add(tv, PC_VISIT, 1);
    if (r1.hit >= 0) {
      combine_at(tv, tile, (uint64_t)h.h2 * B + r1.hit, val, combine);
      return ST_EXISTED;
    }
    BucketScan<K> r2 = r1;
    if (h.b3 != h.h2) {
      r2 = scan<true>(tv, tile, h.b3, key, tag);
      if (tile.leader()) probe_add(tv, PC_VISIT, 1);
      if (r2.hit >= 0) {
        combine_at(tv, tile, (uint64_t)h.b3 * B + r2.hit, val, combine);
        return ST_EXISTED;
      }
    }
    if (rf.free >= 0 && claim_in_bucket(tv, tile, h.b1, rf, key, val, tag, !C::BSP) >= 0) return ST_DONE;
    if (h.b3 == h.h2) return claim_in_bucket(tv, tile, h.h2, r1, key, val, tag) >= 0 ? ST_DONE : ST_FULL;
    return claim_less_loaded(tv, tile, h.h2, r1, h.b3, r2, key, val, tag);
  }

  // Lock-free query (Section 4.2).  Returns ST_DONE/ST_MISS/ST_INVALID, value in *out.
  __device__ static uint8_t query(const TableDev& tv, const Tile<T>& tile, K key, K* out) {
    *out = 0;
    if (key >= Keys<K>::FIRST_INVALID) return ST_INVALID;
    if constexpr (C::CUCKOO) {
      if constexpr (C::BSP) {
        // phased: no locks, plain loads over the three buckets (no writer runs)
        const Cands c = cuckoo_cands(home_of(tv, key));
        for (uint32_t i = 0; i < c.n; ++i) {
          const BucketScan<K> r = scan<true, true>(tv, tile, c.c[i], key, 0u);
          if (r.hit >= 0) {
            *out = r.val;
            return ST_DONE;
          }
        }
        return ST_MISS;
      } else {
        return cuckoo_locked(tv, tile, key, false, out);
      }
    }
    const Home h = home_of(tv, key);
    const uint32_t tag = C::TAGS ? tag_of((uint64_t)key) : 0u;
#ifdef HW_INSTRUMENT
    if (tile.leader()) probe_add(tv, PC_QUERY, 1);
    return find<true>(tv, tile, h, key, tag, out) >= 0 ? ST_DONE : ST_MISS;
#else
    return find(tv, tile, h, key, tag, out) >= 0 ? ST_DONE : ST_MISS;
#endif
  }

  // Erase under the primary lock (none in the phased variant).  ST_DONE if
  // removed, ST_MISS if absent.
  __device__ static uint8_t erase(const TableDev& tv, const Tile<T>& tile, K key) {
    return write(tv, tile, key, K(0), C_KEEP, true);
  }

  // Finds and removes `key` among its candidate buckets.
  __device__ static uint8_t erase_locked(const TableDev& tv, const Tile<T>& tile, const Home& h, K key,
                                         uint32_t tag) {
    if constexpr (C::CHAIN) {
      return erase_chain_locked(tv, tile, h, key);
    } else if constexpr (C::ICEBERG) {
      const uint32_t cand[3] = {h.b1, h.h2, h.b3};
#pragma unroll 1
      for (int i = 0; i < 3; ++i) {
        if (i == 2 && h.b3 == h.h2) break;
        BucketScan<K> r = scan<true>(tv, tile, cand[i], key, tag);
        if (r.hit >= 0) {
          remove(tv, tile, (uint64_t)cand[i] * B + r.hit, tag);
          return ST_DONE;
        }
      }
    } else if constexpr (C::DOUBLE) {
      const uint32_t step = step_of(tv, h);
      uint32_t b = h.b1;
      for (uint32_t i = 0; i < tv.probe_cap; ++i, b = (b + step) & tv.bucket_mask) {
        BucketScan<K> r = scan<true>(tv, tile, b, key, tag);
        if (r.hit >= 0) {
          remove(tv, tile, (uint64_t)b * B + r.hit, tag);
          return ST_DONE;
        }
        if (r.has_empty) break;
      }
    } else {
      BucketScan<K> r = scan<true>(tv, tile, h.b1, key, tag);
      if (r.hit >= 0) {
        remove(tv, tile, (uint64_t)h.b1 * B + r.hit, tag);
        return ST_DONE;
      }
      const uint32_t b2 = h.h2 & tv.bucket_mask;
      if (b2 != h.b1) {
        r = scan<true>(tv, tile, b2, key, tag);
        if (r.hit >= 0) {
          remove(tv, tile, (uint64_t)b2 * B + r.hit, tag);
          return ST_DONE;
        }
      }
    }
    return ST_MISS;
  }
};

}  // namespace hw

// HashWave CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the package smoke check and the benchmark's CPU-baseline
// leg may load this library.  The GPU library never links, loads or calls it, and
// this file includes nothing from the GPU library: every rule below is written
// out again here from the paper and from the documented readings of it.
//
// Three parts:
//
//  1. The semantic map.  The paper's API (Section 5.1, "Hash table API") defines
//     Upsert(key, value, callback), Query(key, &value) and Erase(key) on a map
//     from keys to values; Section 4.1 requires concurrent operations to be
//     serialisable.  The oracle is that definition written out: a standard
//     library hash map, with a batch applied one operation at a time in input
//     order.  Insert is Upsert with the "insert if unique" callback (Section
//     5.1).  Sentinel keys are rejected (reading: the paper never names its
//     empty/tombstone/reservation patterns; the GPU tables reserve the top three
//     64-bit values, or the top two 32-bit values).
//
//  2. The layout checker.  Given a raw image of a GPU table (slots, tags, lock
//     bits) it re-derives every key's candidate buckets from the documented hash
//     rule (MurmurHash3's 64-bit finaliser of key XOR a fixed salt) and checks the
//     design invariants: no duplicate key, no reservation marker left, every key
//     in one of its candidate buckets, for double hashing every key before the
//     first bucket on its sequence that holds an empty slot, every tag equal to the
//     tag of its key (Section 4.3), every lock bit clear.  It also counts probes
//     (Section 5.1: unique 128-byte lines an operation touches).
//
//  3. A sequential layout simulator: the placement rule of each design applied
//     one key at a time (double hashing: first bucket on the sequence with a free
//     slot, Section 2.2; power-of-two-choice: less loaded of two buckets, with the
//     75% shortcut, Section 2.2).  Its probe counts are pinned to the paper's
//     Table 1 by the tests, which is what ties the checker's model to the paper.
//
// Every function is a plain C ABI for ctypes.
//
// ORC_MUTANT (0 = none) plants one known mistake, so the test suite can show
// that its pins catch it; the shipped build never sets it.
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

extern "C" {

// ---------------------------------------------------------------------------
// 1. Semantic map
// ---------------------------------------------------------------------------

// Operation codes of a batch (Section 5.1).
enum { ORC_QUERY = 0, ORC_INSERT = 1, ORC_UPSERT = 2, ORC_ERASE = 3 };
// Upsert callbacks offered as an enum (Section 5.1 gives "insert if unique" and
// atomic accumulation as examples; replace/min/max are the same kind of callback).
enum { ORC_SUM = 0, ORC_KEEP = 1, ORC_REPLACE = 2, ORC_MIN = 3, ORC_MAX = 4 };
// Per-operation status codes.
enum { ORC_MISS = 0, ORC_DONE = 1, ORC_EXISTED = 2, ORC_FULL = 3, ORC_INVALID = 4 };

struct orc_map {
  int key_bits;
  uint64_t capacity;  // 0 = unbounded; else inserting past it gives ORC_FULL
  std::unordered_map<uint64_t, uint64_t> m;
};

static uint64_t width_mask(int bits) { return bits == 64 ? ~0ull : ((1ull << bits) - 1); }

static bool is_sentinel(const orc_map* h, uint64_t k) {
  uint64_t top = width_mask(h->key_bits);
  int n_reserved = h->key_bits == 64 ? (ORC_MUTANT == 2 ? 2 : 3) : 2;
  return k > top - (uint64_t)n_reserved;
}

orc_map* orc_map_new(int key_bits, uint64_t capacity) {
  if (key_bits != 64 && key_bits != 32) return nullptr;
  orc_map* h = new orc_map;
  h->key_bits = key_bits;
  h->capacity = capacity;
  return h;
}

void orc_map_free(orc_map* h) { delete h; }

uint64_t orc_map_size(const orc_map* h) { return (uint64_t)h->m.size(); }

static uint64_t combine(int op, uint64_t old, uint64_t v, uint64_t mask) {
  switch (op) {
    case ORC_SUM: return ORC_MUTANT == 1 ? (old + v) : (old + v) & mask;
    case ORC_KEEP: return ORC_MUTANT == 5 ? v : old;
    case ORC_REPLACE: return v & mask;
    case ORC_MIN: return std::min(old, v & mask);
    case ORC_MAX: return std::max(old, v & mask);
  }
  return old;
}

// Applies n operations in input order.  `ops` may be NULL (then every op is
// `default_op`).  `vals` may be NULL for queries/erases.  Outputs: status[i] and,
// for queries, vals_out[i] = stored value if found else 0 (0 for other ops).
// Either output may be NULL.  Returns 0, or -1 on a bad argument.
int orc_map_apply(orc_map* h, uint64_t n, const uint8_t* ops, int default_op,
                  const uint64_t* keys, const uint64_t* vals, int combine_op,
                  uint8_t* status, uint64_t* vals_out) {
  if (!h || (n && !keys)) return -1;
  const uint64_t mask = width_mask(h->key_bits);
  for (uint64_t i = 0; i < n; i++) {
    int op = ops ? ops[i] : default_op;
    uint64_t k = keys[i];
    uint64_t v = vals ? (vals[i] & mask) : 0;
    uint8_t st = ORC_MISS;
    uint64_t out = 0;
    if (k > mask || is_sentinel(h, k)) {
      st = ORC_INVALID;
    } else if (op == ORC_QUERY) {
      auto it = h->m.find(k);
      if (it != h->m.end()) { st = ORC_DONE; out = ORC_MUTANT == 12 ? it->first : it->second; }
    } else if (op == ORC_INSERT || op == ORC_UPSERT) {
      int c = op == ORC_INSERT ? ORC_KEEP : combine_op;
      auto it = h->m.find(k);
      if (it != h->m.end()) {
        it->second = combine(c, it->second, v, mask);
        st = ORC_EXISTED;
      } else if (h->capacity && (ORC_MUTANT == 4 ? h->m.size() > h->capacity : h->m.size() >= h->capacity)) {
        st = ORC_FULL;
      } else {
        h->m.emplace(k, v);
        st = ORC_DONE;
      }
    } else if (op == ORC_ERASE) {
      st = (ORC_MUTANT == 3 ? h->m.count(k) : h->m.erase(k)) ? ORC_DONE : ORC_MISS;
    } else {
      return -1;
    }
    if (status) status[i] = st;
    if (vals_out) vals_out[i] = out;
  }
  return 0;
}

// Writes all (key, value) pairs sorted by key.  Arrays must hold orc_map_size().
void orc_map_dump(const orc_map* h, uint64_t* keys, uint64_t* vals) {
  std::vector<std::pair<uint64_t, uint64_t>> v(h->m.begin(), h->m.end());
  std::sort(v.begin(), v.end());
  for (size_t i = 0; i < v.size(); i++) {
    keys[i] = v[i].first;
    if (vals) vals[i] = v[i].second;
  }
}

// Order-independent digest of the map contents (sum and xor of a per-pair mix),
// used to compare two maps cheaply.
void orc_map_digest(const orc_map* h, uint64_t* sum_out, uint64_t* xor_out) {
  uint64_t s = 0, x = 0;
  for (auto& kv : h->m) {
    uint64_t z = kv.first * 0x9E3779B97F4A7C15ull ^ (kv.second + 0x632BE59BD9B4E019ull);
    z ^= z >> 29;
    s += z;
    x ^= z;
  }
  *sum_out = s;
  *xor_out = x;
}

// ---------------------------------------------------------------------------
// 2. Hash rule, probe model and layout checker (independent re-statement)
// ---------------------------------------------------------------------------
//
// Reading of the paper's silent hash functions (Section 2.2 names two hash
// functions for double hashing and two choices for power-of-two-choice, nothing
// more):  h = fmix64(key XOR 0x6a09e667f3bcc909), fmix64 being the 64-bit
// finaliser of Appleby's MurmurHash3.  Primary bucket = low 32 bits of h mod nb;
// second hash = high 32 bits of h.  Double hashing visits (b1 + i*step) mod nb
// with step = (second mod nb) | 1 (odd, so the sequence covers all nb buckets, nb
// a power of two).  Power-of-two-choice's alternate bucket = second mod nb.
// Tag (Section 5.1: the low 16 bits of the key) with the two top patterns
// reserved for empty (0xFFFF) and tombstone (0xFFFE): such keys take low16 - 2.
//
// Iceberg hashing (Section 2.2; the split is the evaluated one of Section 5, 83%
// front yard and 17% backyard, not the 90/10 of the design overview): of nb
// buckets the first nf = floor(83 nb / 100) (kept within 1 .. nb-1) form the front
// yard and the other nb - nf the backyard.  Reading of the silent hashes: front
// bucket = floor(lo32(h) * nf / 2^32); the two backyard choices are
// nf + floor(hi32(h) * (nb-nf) / 2^32) and nf + floor(lo32(g) * (nb-nf) / 2^32),
// with g = fmix64(key XOR 0xbb67ae8584caa73b).

enum { ORC_DOUBLE = 0, ORC_DOUBLE_M = 1, ORC_P2 = 2, ORC_P2_M = 3, ORC_ICEBERG = 4, ORC_ICEBERG_M = 5,
       ORC_CHAINING = 6, ORC_CUCKOO = 7 };

static uint64_t orc_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

static const uint64_t ORC_SALT = 0x6a09e667f3bcc909ull;

struct orc_hash {
  uint64_t b1, second;
};

static orc_hash orc_hash_key(uint64_t key, uint64_t nb) {
  uint64_t h = orc_fmix64(key ^ ORC_SALT);
  orc_hash r;
  r.b1 = (uint64_t)(uint32_t)h % nb;
  r.second = (uint64_t)(uint32_t)(h >> 32);
  return r;
}

static uint64_t orc_double_bucket(const orc_hash& h, uint64_t nb, uint64_t i) {
  uint64_t step = ORC_MUTANT == 6 ? (h.second % nb) : (h.second % nb) | 1;
  return (h.b1 + i * step) % nb;
}

static uint64_t orc_p2_alt(const orc_hash& h, uint64_t nb) { return h.second % nb; }

static const uint64_t ORC_SALT_B = 0xbb67ae8584caa73bull;

uint64_t orc_iceberg_front_buckets(uint64_t nb) {
  uint64_t nf = nb * (ORC_MUTANT == 13 ? 90 : 83) / 100;
  if (nf < 1) nf = 1;
  if (nf > nb - 1) nf = nb - 1;
  return nf;
}

struct orc_iceberg {
  uint64_t front, back1, back2;
};

// floor(x * n / 2^32) for a 32-bit x: a uniform x gives a near-uniform index below n.
static uint64_t orc_scale32(uint64_t x32, uint64_t n) { return (x32 * n) >> 32; }

static orc_iceberg orc_iceberg_of(uint64_t key, uint64_t nb) {
  const uint64_t nf = orc_iceberg_front_buckets(nb), nback = nb - nf;
  const uint64_t h = orc_fmix64(key ^ ORC_SALT);
  const uint64_t g = orc_fmix64(key ^ ORC_SALT_B);
  orc_iceberg r;
  r.front = orc_scale32(h & 0xFFFFFFFFull, nf);
  r.back1 = nf + orc_scale32(h >> 32, nback);
  r.back2 = nf + orc_scale32(g & 0xFFFFFFFFull, nback);
  return r;
}

uint16_t orc_tag(uint64_t key) {
  uint16_t t = (uint16_t)(key & 0xFFFF);
  return t >= 0xFFFE ? (uint16_t)(t - (ORC_MUTANT == 9 ? 1 : 2)) : t;
}

// Candidate-bucket helpers exported for tests.
uint64_t orc_primary_bucket(uint64_t key, uint64_t nb) { return orc_hash_key(key, nb).b1; }
uint64_t orc_double_probe(uint64_t key, uint64_t nb, uint64_t i) {
  return orc_double_bucket(orc_hash_key(key, nb), nb, i);
}
uint64_t orc_p2_alternate(uint64_t key, uint64_t nb) { return orc_p2_alt(orc_hash_key(key, nb), nb); }
void orc_iceberg_buckets(uint64_t key, uint64_t nb, uint64_t* out3) {
  orc_iceberg r = orc_iceberg_of(key, nb);
  out3[0] = r.front;
  out3[1] = r.back1;
  out3[2] = r.back2;
}

static bool design_has_tags(int d) { return d == ORC_DOUBLE_M || d == ORC_P2_M || d == ORC_ICEBERG_M; }
static bool design_is_double(int d) { return d == ORC_DOUBLE || d == ORC_DOUBLE_M; }
static bool design_is_iceberg(int d) { return d == ORC_ICEBERG || d == ORC_ICEBERG_M; }
static bool design_is_cuckoo(int d) { return d == ORC_CUCKOO; }

// Three-way cuckoo hashing (Section 2.2, configuration of Section 5): a key may
// live in any of three buckets.  Reading of the silent hashes: lo32(h) mod nb,
// hi32(h) mod nb and lo32(g) mod nb, with h of part 2 and g the salted hash of
// the iceberg backyard.
struct orc_cuckoo {
  uint64_t c[3];
  int n;  // distinct candidates, in that order
};

static orc_cuckoo orc_cuckoo_of(uint64_t key, uint64_t nb) {
  const uint64_t h = orc_fmix64(key ^ ORC_SALT);
  const uint64_t g = orc_fmix64(key ^ ORC_SALT_B);
  const uint64_t raw[3] = {(h & 0xFFFFFFFFull) % nb, (h >> 32) % nb, (g & 0xFFFFFFFFull) % nb};
  orc_cuckoo r;
  r.n = 0;
  for (int i = 0; i < 3; i++) {
    bool dup = false;
    for (int j = 0; j < r.n; j++) dup |= r.c[j] == raw[i];
    if (!dup) r.c[r.n++] = raw[i];
  }
  return r;
}

void orc_cuckoo_buckets(uint64_t key, uint64_t nb, uint64_t* out3) {
  const uint64_t h = orc_fmix64(key ^ ORC_SALT);
  const uint64_t g = orc_fmix64(key ^ ORC_SALT_B);
  out3[0] = (h & 0xFFFFFFFFull) % nb;
  out3[1] = (h >> 32) % nb;
  out3[2] = (g & 0xFFFFFFFFull) % nb;
}

// A table image in host memory.  Slots are (key, value) pairs of key_bits each,
// bucket-major: slot s = bucket * bucket_slots + j.
struct orc_image {
  int design, key_bits;
  uint64_t nb, bucket_slots;
  const uint8_t* slots;
  const uint16_t* tags;
  uint64_t key(uint64_t s) const {
    if (key_bits == 64) { uint64_t k; memcpy(&k, slots + 16 * s, 8); return k; }
    uint32_t k; memcpy(&k, slots + 8 * s, 4); return k;
  }
  uint64_t value(uint64_t s) const {
    if (key_bits == 64) { uint64_t v; memcpy(&v, slots + 16 * s + 8, 8); return v; }
    uint32_t v; memcpy(&v, slots + 8 * s + 4, 4); return v;
  }
  uint64_t empty_key() const { return key_bits == 64 ? ~0ull : 0xFFFFFFFFull; }
  uint64_t tomb_key() const { return empty_key() - 1; }
  uint64_t reserved_key() const { return empty_key() - 2; }  // 64-bit only
  uint64_t slot_bytes() const { return key_bits == 64 ? 16 : 8; }
};

static bool bucket_has_empty(const orc_image& im, uint64_t b) {
  for (uint64_t j = 0; j < im.bucket_slots; j++) {
    uint64_t s = b * im.bucket_slots + j;
    if (design_has_tags(im.design)) {
      if (im.tags[s] == 0xFFFF) return true;
    } else if (im.key(s) == im.empty_key()) {
      return true;
    }
  }
  return false;
}

// 128-byte lines spanned by a bucket's slots, and by its tags.
static uint64_t lines_of(uint64_t bytes) { return (bytes + 127) / 128; }

struct orc_layout_report {
  uint64_t live, tombs, empties, reserved;
  uint64_t duplicate_keys;   // extra copies beyond the first
  uint64_t misplaced;        // key outside its candidate buckets / past an empty-holding bucket
  uint64_t tag_mismatch;     // tag disagrees with its slot (tag designs)
  uint64_t locks_held;       // lock bits still set
  uint64_t in_alternate;     // power-of-two-choice: keys in their alternate bucket;
                             // iceberg: keys in the backyard
  double pos_probe_sum;      // sum over live keys of the positive-query probe count
  double neg_probe_sum;      // sum over `neg_keys` of the negative-query probe count
  uint64_t neg_count;
  uint64_t max_seq_index;    // double hashing: largest sequence index of a live key
  uint64_t front_room;       // iceberg: backyard keys whose front bucket has an empty
                             // slot (none in a table that has never erased)
};

// Positive-query probe count of a key found at sequence position `pos_bucket`
// (0 = primary / first bucket) in slot j of that bucket, in the paper's unit (unique
// 128-byte lines touched, Section 5.1).  Model:
//   double hashing, no tags: each visited bucket's lines are read one tile-width at a
//     time; a tile reads `tile_bytes` per step; the found bucket is read up to j.
//   tag designs: one tag-bucket read per visited bucket (lines of 2*bucket bytes) plus
//     one line for the key/value slot.
//   power-of-two-choice, no tags: primary read fully when the key is in the alternate.
static double probe_pos(const orc_image& im, uint64_t pos_bucket, uint64_t j, uint64_t tile_bytes) {
  const uint64_t sb = im.slot_bytes();
  if (design_has_tags(im.design)) {
    return (double)(pos_bucket + 1) * (double)lines_of(2 * im.bucket_slots) + 1.0;
  }
  uint64_t bucket_lines = lines_of(im.bucket_slots * sb);
  uint64_t step_lines = std::max<uint64_t>(1, tile_bytes / 128);
  uint64_t found_lines = std::min<uint64_t>(bucket_lines, ((j * sb) / 128) / step_lines * step_lines + step_lines);
  if (ORC_MUTANT == 10) found_lines = bucket_lines;
  return (double)(pos_bucket * bucket_lines + found_lines);
}

// Negative-query probe count for a key absent from the table.
static double probe_neg(const orc_image& im, uint64_t key) {
  const uint64_t sb = im.slot_bytes();
  orc_hash h = orc_hash_key(key, im.nb);
  uint64_t per_bucket = design_has_tags(im.design) ? lines_of(2 * im.bucket_slots)
                                                   : lines_of(im.bucket_slots * sb);
  if (design_is_double(im.design)) {
    for (uint64_t i = 0; i < im.nb; i++) {
      uint64_t b = orc_double_bucket(h, im.nb, i);
      if (bucket_has_empty(im, b)) return (double)((i + 1) * per_bucket);
    }
    return (double)(im.nb * per_bucket);
  }
  if (design_is_cuckoo(im.design)) return (double)(orc_cuckoo_of(key, im.nb).n * per_bucket);
  if (design_is_iceberg(im.design)) {
    // A table that has never erased keeps a key out of the backyard while its front
    // bucket has room, so a query stops at a front bucket with an empty slot.
    orc_iceberg ib = orc_iceberg_of(key, im.nb);
    if (bucket_has_empty(im, ib.front)) return (double)per_bucket;
    return (double)((ib.back1 == ib.back2 ? 2 : 3) * per_bucket);
  }
  uint64_t b2 = orc_p2_alt(h, im.nb);
  return (double)((b2 == h.b1 ? 1 : 2) * per_bucket);
}

// Checks a quiescent table image.  `tags` may be NULL for designs without tags;
// `locks` (nlock_words 64-bit words, bit b%64 of word b/64 = bucket b) may be NULL.
// `neg_keys` (may be NULL) are keys known absent, for negative probe counts.
// Returns the number of invariant violations found (0 = consistent).
uint64_t orc_layout_check(int design, int key_bits, uint64_t nb, uint64_t bucket_slots,
                          const void* slots, const uint16_t* tags, const uint64_t* locks,
                          uint64_t nlock_words, const uint64_t* neg_keys, uint64_t n_neg,
                          uint64_t tile_bytes, orc_layout_report* rep) {
  orc_image im{design, key_bits, nb, bucket_slots, (const uint8_t*)slots, tags};
  orc_layout_report r;
  memset(&r, 0, sizeof r);
  if (design_has_tags(design) && !tags) { r.tag_mismatch = 1; *rep = r; return 1; }
  const uint64_t nslots = nb * bucket_slots;
  std::unordered_set<uint64_t> seen;
  seen.reserve(nslots);
  for (uint64_t b = 0; b < nb; b++) {
    for (uint64_t j = 0; j < bucket_slots; j++) {
      uint64_t s = b * bucket_slots + j;
      uint64_t k = im.key(s);
      uint16_t t = tags ? tags[s] : 0;
      if (k == im.empty_key()) {
        r.empties++;
        if (tags && t != 0xFFFF) r.tag_mismatch++;
        continue;
      }
      if (k == im.tomb_key()) {
        r.tombs++;
        // Erase writes the tombstone tag in double hashing designs; tags of
        // power-of-two-choice and iceberg designs return to empty (no tombstones
        // are used).
        if (tags && t != 0xFFFE) r.tag_mismatch++;
        if (!design_is_double(design)) r.misplaced++;
        continue;
      }
      if (key_bits == 64 && k == im.reserved_key()) { r.reserved++; continue; }
      r.live++;
      if (!seen.insert(k).second && ORC_MUTANT != 11) r.duplicate_keys++;
      if (tags && t != orc_tag(k)) r.tag_mismatch++;
      orc_hash h = orc_hash_key(k, nb);
      if (design_is_double(design)) {
        // Key must sit on its sequence, with no empty-holding bucket before it.
        uint64_t i = 0;
        bool ok = false;
        for (; i < nb; i++) {
          uint64_t bi = orc_double_bucket(h, nb, i);
          if (bi == b) { ok = true; break; }
          if (bucket_has_empty(im, bi)) break;
        }
        if (!ok) { r.misplaced++; continue; }
        r.max_seq_index = std::max(r.max_seq_index, i);
        r.pos_probe_sum += probe_pos(im, i, j, tile_bytes);
      } else if (design_is_cuckoo(design)) {
        // Any of the three candidates; a query reads them in order.
        orc_cuckoo cc = orc_cuckoo_of(k, nb);
        int at = -1;
        for (int c = 0; c < cc.n; c++)
          if (cc.c[c] == b) at = c;
        if (at < 0) { r.misplaced++; continue; }
        if (at > 0) r.in_alternate++;
        r.pos_probe_sum += probe_pos(im, (uint64_t)at, j, tile_bytes);
      } else if (design_is_iceberg(design)) {
        // Front bucket, then the backyard choices in order (a repeated choice once).
        orc_iceberg ib = orc_iceberg_of(k, nb);
        if (b == ib.front) {
          r.pos_probe_sum += probe_pos(im, 0, j, tile_bytes);
        } else if (b == ib.back1 || b == ib.back2) {
          r.in_alternate++;
          r.pos_probe_sum += probe_pos(im, b == ib.back1 ? 1 : 2, j, tile_bytes);
          if (bucket_has_empty(im, ib.front)) r.front_room++;
        } else {
          r.misplaced++;
        }
      } else {
        uint64_t b2 = orc_p2_alt(h, nb);
        if (b == h.b1) {
          r.pos_probe_sum += probe_pos(im, 0, j, tile_bytes);
        } else if (b == b2) {
          r.in_alternate++;
          r.pos_probe_sum += probe_pos(im, 1, j, tile_bytes);
        } else {
          r.misplaced++;
        }
      }
    }
  }
  if (locks) {
    for (uint64_t w = 0; w < nlock_words; w++) r.locks_held += (uint64_t)__builtin_popcountll(locks[w]);
  }
  for (uint64_t i = 0; i < n_neg; i++) {
    r.neg_probe_sum += probe_neg(im, neg_keys[i]);
    r.neg_count++;
  }
  *rep = r;
  return r.duplicate_keys + r.misplaced + r.tag_mismatch + r.locks_held + r.reserved;
}

// Live (key, value) pairs of an image, in slot order.  Returns the count.
uint64_t orc_image_pairs(int key_bits, uint64_t nslots, const void* slots, uint64_t* keys,
                         uint64_t* vals) {
  orc_image im{0, key_bits, 1, nslots, (const uint8_t*)slots, nullptr};
  uint64_t c = 0;
  for (uint64_t s = 0; s < nslots; s++) {
    uint64_t k = im.key(s);
    if (k == im.empty_key() || k == im.tomb_key()) continue;
    if (key_bits == 64 && k == im.reserved_key()) continue;
    keys[c] = k;
    vals[c] = im.value(s);
    c++;
  }
  return c;
}

// ---------------------------------------------------------------------------
// 3. Sequential layout simulator (placement rules of Section 2.2)
// ---------------------------------------------------------------------------
//
// Inserts `n` distinct keys one at a time into an empty image (slots and tags
// pre-filled with the empty pattern by this function).  Within a bucket the
// lowest-index free slot is taken.
//   double hashing: first bucket along the sequence with a free slot.
//   power-of-two-choice: if `shortcut` and the primary holds fewer than 3/4 of
//     bucket_slots keys, the primary; else the less loaded of primary and
//     alternate, ties to the primary; full when both are full.
//   iceberg: the front bucket while it has a free slot; else the less loaded of
//     the two backyard choices, ties to the first; full when both are full.
// `visits` (nullable, n entries): for each key, the buckets its insert looks at
// before placing it -- double hashing: every bucket up to the one it goes to;
// power-of-two-choice: the primary, plus the alternate when the shortcut does
// not apply and the two differ; iceberg: the front bucket, plus both backyard
// choices (one if they coincide) when the front is full.  In the tag designs a
// visit reads one tag bucket, a line of its own (reading 13, Table 1's insert
// column).
// Returns the number of keys that could not be placed.
uint64_t orc_sim_insert(int design, int key_bits, uint64_t nb, uint64_t bucket_slots,
                        void* slots, uint16_t* tags, const uint64_t* keys, const uint64_t* vals,
                        uint64_t n, int shortcut, int init, uint32_t* visits) {
  const uint64_t nslots = nb * bucket_slots;
  const uint64_t sb = key_bits == 64 ? 16 : 8;
  uint8_t* S = (uint8_t*)slots;
  if (init) {
    memset(S, 0xFF, nslots * sb);
    if (tags) memset(tags, 0xFF, nslots * 2);
  }
  std::vector<uint32_t> fill(nb, 0);
  if (!init) {
    orc_image im{design, key_bits, nb, bucket_slots, S, tags};
    for (uint64_t b = 0; b < nb; b++)
      for (uint64_t j = 0; j < bucket_slots; j++)
        if (im.key(b * bucket_slots + j) != im.empty_key()) fill[b]++;
  }
  const uint64_t empty = key_bits == 64 ? ~0ull : 0xFFFFFFFFull;
  auto slot_key = [&](uint64_t s) -> uint64_t {
    if (key_bits == 64) { uint64_t k; memcpy(&k, S + 16 * s, 8); return k; }
    uint32_t k; memcpy(&k, S + 8 * s, 4); return k;
  };
  auto put = [&](uint64_t b, uint64_t key, uint64_t val) {
    for (uint64_t j = 0; j < bucket_slots; j++) {
      uint64_t s = b * bucket_slots + j;
      if (slot_key(s) != empty) continue;
      if (key_bits == 64) { memcpy(S + 16 * s, &key, 8); memcpy(S + 16 * s + 8, &val, 8); }
      else { uint32_t k = (uint32_t)key, v = (uint32_t)val; memcpy(S + 8 * s, &k, 4); memcpy(S + 8 * s + 4, &v, 4); }
      if (tags) tags[s] = orc_tag(key);
      fill[b]++;
      return;
    }
  };
  uint64_t failed = 0;
  for (uint64_t i = 0; i < n; i++) {
    orc_hash h = orc_hash_key(keys[i], nb);
    uint64_t v = vals ? vals[i] : 0;
    if (design_is_double(design)) {
      bool placed = false;
      uint64_t p = 0;
      for (; p < nb; p++) {
        uint64_t b = orc_double_bucket(h, nb, p);
        if (fill[b] < bucket_slots) { put(b, keys[i], v); placed = true; break; }
      }
      if (visits) visits[i] = (uint32_t)(placed ? p + 1 : nb);
      if (!placed) failed++;
    } else if (design_is_iceberg(design)) {
      orc_iceberg ib = orc_iceberg_of(keys[i], nb);
      if (fill[ib.front] < bucket_slots) {
        if (visits) visits[i] = 1;
        put(ib.front, keys[i], v);
        continue;
      }
      if (visits) visits[i] = ib.back1 == ib.back2 ? 2 : 3;
      uint64_t b = ORC_MUTANT == 14 ? (fill[ib.back2] <= fill[ib.back1] ? ib.back2 : ib.back1)
                                    : (fill[ib.back2] < fill[ib.back1] ? ib.back2 : ib.back1);
      if (fill[b] >= bucket_slots) { failed++; continue; }
      put(b, keys[i], v);
    } else {
      uint64_t b1 = h.b1, b2 = orc_p2_alt(h, nb);
      if (shortcut && (ORC_MUTANT == 7 ? 2 * fill[b1] < bucket_slots : 4 * fill[b1] < 3 * bucket_slots)) {
        if (visits) visits[i] = ORC_MUTANT == 18 ? 2 : 1;
        put(b1, keys[i], v);
        continue;
      }
      if (visits) visits[i] = b1 == b2 ? 1 : 2;
      uint64_t b = ORC_MUTANT == 8 ? (fill[b2] <= fill[b1] ? b2 : b1) : (fill[b2] < fill[b1] ? b2 : b1);
      if (fill[b] >= bucket_slots) { failed++; continue; }
      put(b, keys[i], v);
    }
  }
  return failed;
}

// ---------------------------------------------------------------------------
// 4. Sequential aging simulator (Section 6.5 workload, Table 1 "aging probes")
// ---------------------------------------------------------------------------
//
// Fills an empty 64-bit image with keys[0, n0), then runs `iters` iterations:
// insert the next s keys, erase the oldest s keys, and count the probes of s
// positive queries (keys[pos_start[i], pos_start[i] + s)) and s negative ones
// (negs[i*s, (i+1)*s)).  Placement follows each design's rules once erases
// have happened:
//   double hashing: the first free (empty or tombstone) slot along the probe
//     sequence; erase leaves a tombstone (key and tag);
//   power-of-two-choice: no shortcut after an erase, so the less loaded of the
//     two buckets (ties to the primary); erase empties the slot;
//   iceberg: the front bucket if it has a free slot, else the less loaded
//     backyard choice (ties to the first); erase empties the slot.
// Probes use the model of probe_pos; a negative query reads buckets until the
// design lets it stop: double hashing at the first bucket holding an empty slot
// or after `probe_cap` buckets (0 = no cap), power-of-two-choice after both
// buckets, iceberg after all three (the front-yard exit is off once erased).
// Probes are counted from iteration `from_iter` on.  out[0] = mean positive
// probes, out[1] = mean negative probes, out[2] = inserts that found no slot.
// Returns 0, or -1 on a bad argument.

static bool slot_free(const orc_image& im, uint64_t s) {
  if (design_has_tags(im.design)) return im.tags[s] >= 0xFFFE;
  uint64_t k = im.key(s);
  return k == im.empty_key() || k == im.tomb_key();
}

static uint64_t bucket_fill(const orc_image& im, uint64_t b) {
  uint64_t f = 0;
  for (uint64_t j = 0; j < im.bucket_slots; j++) f += !slot_free(im, b * im.bucket_slots + j);
  return f;
}

static int64_t first_free(const orc_image& im, uint64_t b) {
  for (uint64_t j = 0; j < im.bucket_slots; j++)
    if (slot_free(im, b * im.bucket_slots + j)) return (int64_t)(b * im.bucket_slots + j);
  return -1;
}

int orc_sim_aging(int design, uint64_t nb, uint64_t bucket_slots, uint64_t tile_bytes, uint64_t probe_cap,
                  const uint64_t* keys, uint64_t n0, uint64_t s, uint64_t iters, const uint64_t* pos_start,
                  const uint64_t* negs, uint64_t from_iter, double* out) {
  if (!keys || !out || nb == 0 || bucket_slots == 0 || design < ORC_DOUBLE || design > ORC_ICEBERG_M) return -1;
  const uint64_t nslots = nb * bucket_slots;
  std::vector<uint64_t> S(2 * nslots, ~0ull);
  std::vector<uint16_t> T(design_has_tags(design) ? nslots : 0, 0xFFFF);
  orc_image im{design, 64, nb, bucket_slots, (const uint8_t*)S.data(), T.empty() ? nullptr : T.data()};
  const uint64_t cap = probe_cap ? std::min(probe_cap, nb) : nb;
  bool erased = false;
  uint64_t failed = 0;
  auto write = [&](int64_t slot, uint64_t key, uint16_t tag) {
    S[2 * slot] = key;
    S[2 * slot + 1] = key * 3 + 1;
    if (!T.empty()) T[slot] = tag;
  };
  auto insert = [&](uint64_t key) {
    int64_t slot = -1;
    if (design_is_double(design)) {
      orc_hash h = orc_hash_key(key, nb);
      for (uint64_t i = 0; i < cap && slot < 0; i++) slot = first_free(im, orc_double_bucket(h, nb, i));
    } else if (design_is_iceberg(design)) {
      orc_iceberg ib = orc_iceberg_of(key, nb);
      slot = first_free(im, ib.front);
      if (slot < 0) {
        uint64_t b = bucket_fill(im, ib.back2) < bucket_fill(im, ib.back1) ? ib.back2 : ib.back1;
        slot = first_free(im, b);
        if (slot < 0) slot = first_free(im, b == ib.back1 ? ib.back2 : ib.back1);
      }
    } else {
      orc_hash h = orc_hash_key(key, nb);
      uint64_t b1 = h.b1, b2 = orc_p2_alt(h, nb);
      uint64_t f1 = bucket_fill(im, b1);
      if (!erased && 4 * f1 < 3 * bucket_slots) {
        slot = first_free(im, b1);
      } else {
        uint64_t b = bucket_fill(im, b2) < f1 ? b2 : b1;
        slot = first_free(im, b);
        if (slot < 0) slot = first_free(im, b == b1 ? b2 : b1);
      }
    }
    if (slot < 0) { failed++; return; }
    write(slot, key, orc_tag(key));
  };
  // Locates a live key: (position in the design's visiting order, slot), or pos -1.
  auto locate = [&](uint64_t key, int64_t* slot_out) -> int64_t {
    auto in = [&](uint64_t b) -> int64_t {
      for (uint64_t j = 0; j < bucket_slots; j++)
        if (S[2 * (b * bucket_slots + j)] == key) return (int64_t)(b * bucket_slots + j);
      return -1;
    };
    if (design_is_double(design)) {
      orc_hash h = orc_hash_key(key, nb);
      for (uint64_t i = 0; i < cap; i++) {
        int64_t sl = in(orc_double_bucket(h, nb, i));
        if (sl >= 0) { *slot_out = sl; return (int64_t)i; }
      }
      return -1;
    }
    uint64_t cand[3];
    int nc;
    if (design_is_iceberg(design)) {
      orc_iceberg ib = orc_iceberg_of(key, nb);
      cand[0] = ib.front; cand[1] = ib.back1; cand[2] = ib.back2;
      nc = ib.back2 == ib.back1 ? 2 : 3;
    } else {
      orc_hash h = orc_hash_key(key, nb);
      cand[0] = h.b1; cand[1] = orc_p2_alt(h, nb);
      nc = cand[1] == cand[0] ? 1 : 2;
    }
    for (int c = 0; c < nc; c++) {
      int64_t sl = in(cand[c]);
      if (sl >= 0) { *slot_out = sl; return c; }
    }
    return -1;
  };
  auto erase = [&](uint64_t key) {
    int64_t sl = -1;
    if (locate(key, &sl) < 0) return;
    const bool dbl = design_is_double(design) && ORC_MUTANT != 15;
    S[2 * sl] = dbl ? im.tomb_key() : im.empty_key();
    if (!T.empty()) T[sl] = dbl ? 0xFFFE : 0xFFFF;
    erased = true;
  };
  const uint64_t per_bucket = design_has_tags(design) ? lines_of(2 * bucket_slots) : lines_of(bucket_slots * 16);
  auto neg_probes = [&](uint64_t key) -> double {
    if (design_is_double(design)) {
      orc_hash h = orc_hash_key(key, nb);
      for (uint64_t i = 0; i < cap; i++)
        if (bucket_has_empty(im, orc_double_bucket(h, nb, i))) return (double)((i + 1) * per_bucket);
      return (double)(cap * per_bucket);
    }
    if (design_is_iceberg(design)) {
      orc_iceberg ib = orc_iceberg_of(key, nb);
      if (!erased && bucket_has_empty(im, ib.front)) return (double)per_bucket;
      return (double)((ib.back1 == ib.back2 ? 2 : 3) * per_bucket);
    }
    orc_hash h = orc_hash_key(key, nb);
    return (double)((orc_p2_alt(h, nb) == h.b1 ? 1 : 2) * per_bucket);
  };
  for (uint64_t i = 0; i < n0; i++) insert(keys[i]);
  double pos_sum = 0, neg_sum = 0;
  uint64_t pos_n = 0, neg_n = 0;
  for (uint64_t it = 0; it < iters; it++) {
    for (uint64_t i = 0; i < s; i++) insert(keys[n0 + it * s + i]);
    for (uint64_t i = 0; i < s; i++) erase(keys[it * s + i]);
    if (it < from_iter) continue;
    for (uint64_t i = 0; i < s; i++) {
      int64_t sl = -1;
      int64_t pos = locate(keys[pos_start[it] + i], &sl);
      if (pos < 0) continue;
      pos_sum += probe_pos(im, (uint64_t)pos, (uint64_t)sl % bucket_slots, tile_bytes);
      pos_n++;
    }
    if (negs)
      for (uint64_t i = 0; i < s; i++) { neg_sum += neg_probes(negs[it * s + i]); neg_n++; }
  }
  out[0] = pos_n ? pos_sum / (double)pos_n : 0.0;
  out[1] = neg_n ? neg_sum / (double)neg_n : 0.0;
  out[2] = (double)failed;
  return 0;
}

// ---------------------------------------------------------------------------
// 5. Chaining (Section 5: each chain node is one 128-byte line holding 7
//    key-value pairs and the pointer to the next node)
// ---------------------------------------------------------------------------
//
// Reading of the node layout: 8 units of 16 bytes; units 0..6 are (key, value)
// pairs, unit 7 is the link: its key word holds the empty pattern, its value word
// the index of the next node (all-ones = none).  Nodes 0 .. nb-1 are the
// buckets' first nodes; later nodes form the overflow pool.  Bucket of a key =
// floor(lo32(h) * nb / 2^32), with h the hash of part 2.  Erase empties a slot
// (a chain has no probe sequence to keep intact); an insert takes the first
// empty slot along its chain, else appends a node.

static const uint64_t ORC_NIL = ~0ull;

uint64_t orc_chain_bucket(uint64_t key, uint64_t nb) {
  return orc_scale32(orc_fmix64(key ^ ORC_SALT) & 0xFFFFFFFFull, nb);
}

// Checks a quiescent chaining image of n_nodes nodes (nb buckets).  Violations:
// duplicate keys, keys in the wrong bucket's chain, reserved/tombstone patterns,
// a link unit whose key word is not empty, a cycle or a node on two chains, a
// live key in a node no chain reaches, held locks.  Probes (Section 5.1 unit):
// a positive query reads the nodes up to the key's, a negative one the whole chain.
uint64_t orc_chain_check(uint64_t nb, uint64_t n_nodes, const uint64_t* nodes, const uint64_t* locks,
                         uint64_t nlock_words, const uint64_t* neg_keys, uint64_t n_neg, orc_layout_report* rep) {
  orc_layout_report r;
  memset(&r, 0, sizeof r);
  std::vector<uint8_t> reached(n_nodes, 0);
  std::vector<uint64_t> chain_len(nb, 0);
  std::unordered_set<uint64_t> seen;
  for (uint64_t b = 0; b < nb; b++) {
    uint64_t node = b, pos = 0;
    while (node != ORC_NIL) {
      if (node >= n_nodes || reached[node]) { r.misplaced++; break; }
      reached[node] = 1;
      pos++;
      const uint64_t* u = nodes + 16 * node;
      for (int j = 0; j < 7; j++) {
        const uint64_t k = u[2 * j];
        if (k == ~0ull) { r.empties++; continue; }
        if (k == ~0ull - 1 || k == ~0ull - 2) { r.reserved++; continue; }
        r.live++;
        if (!seen.insert(k).second && ORC_MUTANT != 11) r.duplicate_keys++;
        if (orc_chain_bucket(k, nb) != b) r.misplaced++;
        r.pos_probe_sum += (double)pos;
        if (pos > 1) r.in_alternate++;
      }
      if (u[14] != ~0ull) r.misplaced++;  // link unit key word
      node = u[15];
    }
    chain_len[b] = pos;
    r.max_seq_index = std::max<uint64_t>(r.max_seq_index, pos);
  }
  for (uint64_t n = 0; n < n_nodes; n++) {
    if (reached[n]) continue;
    const uint64_t* u = nodes + 16 * n;
    for (int j = 0; j < 7; j++)
      if (u[2 * j] != ~0ull) r.misplaced++;
  }
  if (locks)
    for (uint64_t w = 0; w < nlock_words; w++) r.locks_held += (uint64_t)__builtin_popcountll(locks[w]);
  for (uint64_t i = 0; i < n_neg; i++) {
    r.neg_probe_sum += (double)chain_len[orc_chain_bucket(neg_keys[i], nb)];
    r.neg_count++;
  }
  *rep = r;
  return r.duplicate_keys + r.misplaced + r.reserved + r.locks_held;
}

// Sequential chaining inserts of distinct keys into an image of n_nodes nodes
// (initialised empty when `init`): the first empty slot along the chain, else a
// new node from the pool (the lowest unused index) linked at the tail.  Returns
// the number of keys that found no room (pool exhausted).
uint64_t orc_sim_chain_insert(uint64_t nb, uint64_t n_nodes, uint64_t* nodes, const uint64_t* keys,
                              uint64_t n, int init) {
  if (init) memset(nodes, 0xFF, n_nodes * 128);
  uint64_t next_free = nb;
  // pool nodes in use are those some chain reaches
  {
    std::vector<uint8_t> reached(n_nodes, 0);
    for (uint64_t b = 0; b < nb; b++)
      for (uint64_t node = b; node != ORC_NIL && node < n_nodes; node = nodes[16 * node + 15]) reached[node] = 1;
    while (next_free < n_nodes && reached[next_free]) next_free++;
  }
  uint64_t failed = 0;
  for (uint64_t i = 0; i < n; i++) {
    const uint64_t k = keys[i];
    uint64_t node = orc_chain_bucket(k, nb), last = node;
    bool placed = false;
    bool first = true;
    while (node != ORC_NIL && !placed) {
      uint64_t* u = nodes + 16 * node;
      if (first || ORC_MUTANT != 16)
        for (int j = 0; j < 7; j++)
          if (u[2 * j] == ~0ull) { u[2 * j] = k; u[2 * j + 1] = k * 3 + 1; placed = true; break; }
      first = false;
      last = node;
      node = u[15];
    }
    if (placed) continue;
    if (next_free >= n_nodes) { failed++; continue; }
    uint64_t* nu = nodes + 16 * next_free;
    nu[0] = k;
    nu[1] = k * 3 + 1;
    nodes[16 * last + 15] = next_free;
    next_free++;
  }
  return failed;
}

// ---------------------------------------------------------------------------
// 6. Sequential three-way bucketed cuckoo inserts
// ---------------------------------------------------------------------------
//
// Distinct keys into a 64-bit cuckoo image (initialised empty when `init`): the
// first candidate bucket (in hash order) with an empty slot, else a random walk
// (Section 2.2: "the new key replaces a key already in a bucket, and the
// insertion procedure is restarted for the evicted key"): the key displaces a
// random slot of a random candidate and the displaced key goes on to one of its
// other candidates, for at most max_kicks displacements.  The walk's random
// numbers come from a splitmix64 stream seeded with `seed`.  A walk that runs out
// leaves its last homeless key counted as failed (the table already lost it,
// which only a sequential model may do).  Returns the number of failed keys.

static uint64_t orc_splitmix_next(uint64_t* st) {
  uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_sim_cuckoo_insert(uint64_t nb, uint64_t bucket_slots, uint64_t* slots, const uint64_t* keys,
                               uint64_t n, uint64_t max_kicks, uint64_t seed, int init) {
  const uint64_t nslots = nb * bucket_slots;
  if (init) memset(slots, 0xFF, nslots * 16);
  uint64_t rng = seed, failed = 0;
  auto free_in = [&](uint64_t b) -> int64_t {
    for (uint64_t j = 0; j < bucket_slots; j++)
      if (slots[2 * (b * bucket_slots + j)] == ~0ull) return (int64_t)(b * bucket_slots + j);
    return -1;
  };
  for (uint64_t i = 0; i < n; i++) {
    uint64_t k = keys[i], v = k * 3 + 1;
    bool placed = false;
    for (uint64_t kick = 0; kick <= max_kicks && !placed; kick++) {
      orc_cuckoo cc = orc_cuckoo_of(k, nb);
      for (int c = 0; c < cc.n && !placed; c++) {
        int64_t s = free_in(cc.c[ORC_MUTANT == 17 ? 0 : c]);
        if (s >= 0) { slots[2 * s] = k; slots[2 * s + 1] = v; placed = true; }
      }
      if (placed || kick == max_kicks) break;
      const uint64_t b = cc.c[orc_splitmix_next(&rng) % (uint64_t)cc.n];
      const uint64_t s = b * bucket_slots + orc_splitmix_next(&rng) % bucket_slots;
      const uint64_t ek = slots[2 * s], ev = slots[2 * s + 1];
      slots[2 * s] = k;
      slots[2 * s + 1] = v;
      k = ek;
      v = ev;
    }
    if (!placed) failed++;
  }
  return failed;
}

}  // extern "C"

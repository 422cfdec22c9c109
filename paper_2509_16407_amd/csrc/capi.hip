// C-ABI of HashWave (declared in include/hashwave.h): table creation and
// layout, argument checks, dispatch to the kernel instance of the table's
// (key width, design, bucket, tile), and the design-independent kernels
// (initialisation, counting, export, primary-bucket lookup).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "hashwave.h"
#include "hw_launch.hpp"
#include "hw_multi.hpp"

using namespace hw;

static void drop_groups_of(hwave_table* t);

struct hwave_table {
  int device;
  hwave_design design;
  hwave_config cfg;
  uint64_t nb, capacity, bytes;
  uint64_t units;  // (key, value) units in the slot region (chaining: link units too)
  uint64_t n_lock_words;
  void* base;
  bool owns;
  const KernelSet* ks;
  LaunchArgs la;
  bool has_merge;  // HWAVE_F_MERGE_MIXED: workspace for merging mixed calls' upserts
  MergeWs ws;
};

namespace {

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return HWAVE_EDEVICE;
}

constexpr uint64_t ALIGN = 256;
// A waiter's limit for its bucket lock (hwave_config.lock_timeout_us), converted
// to ticks of the 100 MHz wall clock, which must fit 32 bits.
constexpr uint32_t DEFAULT_LOCK_TIMEOUT_US = 10000000;
constexpr uint32_t MAX_LOCK_TIMEOUT_US = 40000000;
uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Layout {
  uint64_t nb, capacity, units, pool;
  uint64_t off_tags, off_locks, off_lockq, off_ctrl, off_pool_ctr, off_hot, off_merge, total;
  uint64_t n_lock_words;  // 32-bit words of the lock array (one byte per bucket, at a stride)
  uint32_t lock_shift;    // log2 of the lock stride in bytes
  uint64_t n_lockq;       // lock queues (hw_device.hpp): a power of two
};

// Lock bytes at a stride of 1 << lock_shift bytes (hw_device.hpp, LockArray:
// clamp(2^23 / nb, 1, 8) bytes), then the lock queues: the largest power of
// two <= nb, at most LOCK_QUEUES_MAX.  Returns the offset after them.
uint64_t place_locks(uint64_t nb, uint64_t off, Layout* L) {
  L->lock_shift = 0;
  while (L->lock_shift < 3 && (nb << (L->lock_shift + 1)) <= (1ull << 23)) ++L->lock_shift;
  L->off_locks = off;
  L->n_lock_words = ((nb << L->lock_shift) + 3) / 4;
  off += round_up(L->n_lock_words * 4, ALIGN);
  uint64_t nq = 1;
  while (nq * 2 <= nb && nq * 2 <= LOCK_QUEUES_MAX) nq *= 2;
  L->off_lockq = off;
  L->n_lockq = nq;
  return off + round_up(nq * 8, ALIGN);
}

// Hot-key accumulators (hw_ops.hpp, HOT_ROWS): tables that merge duplicates and
// never erase, except cuckoo (it moves keys) and the phased variant.
bool has_hot(hwave_design design, const hwave_config& c) {
  const uint32_t f = c.flags;
  return (f & HWAVE_F_AGGREGATE) && (f & HWAVE_F_NO_ERASE) && !(f & HWAVE_F_BSP) && design != HWAVE_CUCKOO;
}

// Appends the hot-key accumulators (tags, then accumulators) at `off` if the
// table has them; they lie in the zero-filled part of the table.  Then the
// merge workspace of HWAVE_F_MERGE_MIXED tables (hw_merge.hpp: 2 * MERGE_CHUNK
// entries of a key word and 16 bytes, and a word per operation of a chunk), also
// all zero when empty.
constexpr uint64_t MERGE_ENTRIES = 2ull * MERGE_CHUNK;
uint64_t merge_bytes() { return MERGE_ENTRIES * (8 + sizeof(MergeEntry)) + (uint64_t)MERGE_CHUNK * 4; }

uint64_t place_hot(hwave_design design, const hwave_config& c, uint64_t off, Layout* L) {
  L->off_hot = 0;
  L->off_merge = 0;
  if (has_hot(design, c)) {
    L->off_hot = off;
    off += round_up((uint64_t)HOT_N * 16, ALIGN);
  }
  if (c.flags & HWAVE_F_MERGE_MIXED) {
    L->off_merge = off;
    off += round_up(merge_bytes(), ALIGN);
  }
  return off;
}

bool design_tags(int d) { return d == HWAVE_DOUBLE_M || d == HWAVE_P2_M || d == HWAVE_ICEBERG_M; }
bool design_iceberg(int d) { return d == HWAVE_ICEBERG || d == HWAVE_ICEBERG_M; }
bool design_chain(int d) { return d == HWAVE_CHAINING; }

// Iceberg front yard: 83% of the buckets (Section 5), at least one bucket in
// each yard.
uint64_t iceberg_front(uint64_t nb) {
  uint64_t nf = nb * 83 / 100;
  if (nf < 1) nf = 1;
  if (nf > nb - 1) nf = nb - 1;
  return nf;
}

const std::vector<const KernelSet*>& registry() {
  static std::vector<const KernelSet*> all;
  static std::once_flag once;
  std::call_once(once, [] {
    const KernelSet* (*fns[])(size_t*) = {sets_u64_double, sets_u64_p2, sets_u64_iceberg, sets_u64_chain, sets_u64_cuckoo,
                                          sets_u32_double, sets_u32_p2, sets_u32_iceberg, sets_u64_bsp};
    for (auto f : fns) {
      size_t n = 0;
      const KernelSet* s = f(&n);
      for (size_t i = 0; i < n; i++) all.push_back(s + i);
    }
  });
  return all;
}

const KernelSet* find_set(const hwave_config& c, int design) {
  const bool bsp = (c.flags & HWAVE_F_BSP) != 0;
  for (const KernelSet* s : registry())
    if (s->kv_bits == (int)c.kv_bits && s->design == design && s->bucket == (int)c.bucket_slots &&
        s->tile == (int)c.tile && s->bsp == bsp)
      return s;
  return nullptr;
}

// Paper configurations (Section 5) for 64-bit keys; 32-bit keys keep the same
// bucket byte span with 8-byte slots where a design's default bucket is small.
void defaults_for(hwave_design design, uint32_t kv_bits, hwave_config* c) {
  memset(c, 0, sizeof *c);
  c->kv_bits = kv_bits;
  c->bucket_slots = design == HWAVE_DOUBLE ? (kv_bits == 64 ? 8 : 16)
                    : design_chain(design)   ? 7
                    : design == HWAVE_CUCKOO ? 8
                                             : 32;
  c->tile = design_tags(design) || design == HWAVE_CUCKOO ? 4 : 8;
}

int resolve_config(hwave_design design, const hwave_config* in, hwave_config* out) {
  if ((int)design < HWAVE_DOUBLE || (int)design > HWAVE_CUCKOO) return HWAVE_EINVAL;
  const uint32_t kv = in && in->kv_bits ? in->kv_bits : 64;
  if (kv != 64 && kv != 32) return HWAVE_EINVAL;
  hwave_config c;
  defaults_for(design, kv, &c);
  if (in) {
    if (in->bucket_slots) c.bucket_slots = in->bucket_slots;
    if (in->tile) c.tile = in->tile;
    c.probe_cap = in->probe_cap;
    c.flags = in->flags;
    c.lock_timeout_us = in->lock_timeout_us;
  }
  if (c.lock_timeout_us > MAX_LOCK_TIMEOUT_US) return HWAVE_EINVAL;
  *out = c;
  return HWAVE_OK;
}

int layout_of(uint64_t capacity, hwave_design design, const hwave_config& c, Layout* L) {
  if (capacity == 0 || c.bucket_slots == 0) return HWAVE_EINVAL;
  if (design_chain(design)) {
    // Chaining (Section 5): ceil(capacity / 7) buckets, each a 128-byte first
    // node (7 pairs and a link), then an overflow pool of twice as many nodes.
    // A node stays on its chain once linked (lock-free readers may be walking
    // it), so under churn a chain keeps the nodes its longest past content
    // needed; two spare nodes per bucket cover that for long aging runs.  The
    // capacity reported counts every slot of buckets and pool.
    const uint64_t nb = (capacity + 6) / 7;
    if (nb > (1ull << 30)) return HWAVE_EINVAL;
    const uint64_t pool = 2 * nb;
    L->nb = nb;
    L->pool = pool;
    L->units = (nb + pool) * 8;
    L->capacity = (nb + pool) * 7;
    uint64_t off = round_up(L->units * 16, ALIGN);
    L->off_tags = off;
    off = place_locks(nb, off, L);
    L->off_ctrl = off;
    off += ALIGN;
    L->off_pool_ctr = off;  // POOL_PARTS allocation counters, one per 128-byte line
    off += round_up((uint64_t)POOL_PARTS * POOL_CTR_STRIDE * 4, ALIGN);
    L->total = place_hot(design, c, off, L);
    return HWAVE_OK;
  }
  const uint64_t B = c.bucket_slots;
  uint64_t want = (capacity + B - 1) / B;
  uint64_t nb = design_iceberg(design) ? 2 : 1;  // iceberg: a bucket in each yard
  while (nb < want) nb <<= 1;
  if (nb > (1ull << 32)) return HWAVE_EINVAL;
  const uint64_t slot_bytes = c.kv_bits / 4;  // two words
  L->nb = nb;
  L->capacity = nb * B;
  L->units = L->capacity;
  L->pool = 0;
  uint64_t off = round_up(L->capacity * slot_bytes, ALIGN);
  L->off_tags = off;
  if (design_tags(design)) off += round_up(L->capacity * 2, ALIGN);
  off = place_locks(nb, off, L);
  L->off_ctrl = off;
  off += ALIGN;
  L->total = place_hot(design, c, off, L);
  return HWAVE_OK;
}

__global__ void k_fill16(uint4* p, uint64_t n16, uint32_t word) {
  const uint4 v = make_uint4(word, word, word, word);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename K>
__global__ void k_count(const K* __restrict__ slots, uint64_t nslots, uint64_t* count) {
  uint64_t c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x)
    c += slots[2 * i] < Keys<K>::FIRST_INVALID;
  // wave reduction, one atomic per wave
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd((unsigned long long*)count, (unsigned long long)c);
}

template <typename K>
__global__ void k_export(const K* __restrict__ slots, uint64_t nslots, K* __restrict__ okeys,
                         K* __restrict__ ovals, uint64_t* count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const K k = slots[2 * i];
    if (k < Keys<K>::FIRST_INVALID) {
      const uint64_t at = atomicAdd((unsigned long long*)count, 1ull);
      okeys[at] = k;
      ovals[at] = slots[2 * i + 1];
    }
  }
}

__global__ void k_zero_u64(uint64_t* p) { *p = 0; }

// The bucket whose lock a key's writers take: primary bucket, or the front-yard
// bucket of iceberg tables (nf != 0).
template <typename K>
__global__ void k_primary(const K* __restrict__ keys, uint64_t n, uint32_t mask, uint32_t nf,
                          uint64_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = nf ? front_bucket((uint64_t)keys[i], nf) : hash_key((uint64_t)keys[i], mask).b1;
}

// Every bucket a key may occupy (hwave_candidate_buckets): three per key,
// unused entries all-ones.
template <typename K>
__global__ void k_candidates(const K* __restrict__ keys, uint64_t n, int design, uint32_t mask, uint32_t nf,
                             uint32_t nback, uint64_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = (uint64_t)keys[i];
    uint64_t c0 = ~0ull, c1 = ~0ull, c2 = ~0ull;
    if (design == HWAVE_CHAINING) {
      c0 = front_bucket(k, nf);
    } else if (design == HWAVE_ICEBERG || design == HWAVE_ICEBERG_M) {
      const Yard y = yard_of(k, nf, nback);
      c0 = y.front;
      c1 = y.back1;
      c2 = y.back2;
    } else {
      const Hashed h = hash_key(k, mask);
      c0 = h.b1;
      if (design == HWAVE_DOUBLE || design == HWAVE_DOUBLE_M) {
        c1 = (h.h2 & mask) | 1u;  // the probe step
      } else {
        c1 = h.h2 & mask;
        if (design == HWAVE_CUCKOO) c2 = (uint32_t)fmix64(k ^ HASH_SALT_B) & mask;
      }
    }
    out[3 * i] = c0;
    out[3 * i + 1] = c1;
    out[3 * i + 2] = c2;
  }
}

// Grid cap for grid-stride kernels, cached per device (tables may be created
// from several host threads, e.g. beside a serving loop's worker).
unsigned max_blocks_for(int device) {
  static std::atomic<unsigned> cache[64];
  const bool cached = device >= 0 && device < 64;
  if (cached) {
    const unsigned c = cache[device].load(std::memory_order_relaxed);
    if (c) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    cus = 256;
  const unsigned v = (unsigned)cus * 32;
  if (cached) cache[device].store(v, std::memory_order_relaxed);
  return v;
}

unsigned stream_grid(uint64_t n, int device) {
  uint64_t blocks = (n + 255) / 256;
  uint64_t cap = max_blocks_for(device);
  if (blocks > cap) blocks = cap;
  return (unsigned)(blocks ? blocks : 1);
}

int init_table(hwave_table* t, void* base, uint64_t bytes, const Layout& L, hwave_design design,
               const hwave_config& c, const KernelSet* ks, void* stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  t->device = dev;
  t->design = design;
  t->cfg = c;
  t->nb = L.nb;
  t->capacity = L.capacity;
  t->units = L.units;
  t->bytes = bytes;
  t->n_lock_words = L.n_lock_words;
  t->base = base;
  t->ks = ks;
  uint8_t* b = (uint8_t*)base;
  TableDev& tv = t->la.tv;
  tv.slots = b;
  tv.tagw = design_tags(design) ? (uint32_t*)(b + L.off_tags) : nullptr;
  tv.locks.words = (uint32_t*)(b + L.off_locks);
  tv.locks.shift = L.lock_shift;
  tv.lockq = (uint64_t*)(b + L.off_lockq);
  tv.lockq_mask = (uint32_t)(L.n_lockq - 1);
  tv.ctrl = (uint32_t*)(b + L.off_ctrl);
  tv.bucket_mask = (uint32_t)(L.nb - 1);
  tv.nb_front = design_iceberg(design) ? (uint32_t)iceberg_front(L.nb) : (uint32_t)L.nb;
  tv.nb_back = design_iceberg(design) ? (uint32_t)(L.nb - tv.nb_front) : 0u;
  tv.pool_nodes = (uint32_t)L.pool;
  tv.pool_ctr = design_chain(design) ? (uint32_t*)(b + L.off_pool_ctr) : nullptr;
  uint64_t cap = c.probe_cap ? c.probe_cap : L.nb;
  if (cap > L.nb) cap = L.nb;
  tv.probe_cap = (uint32_t)(cap > 0xFFFFFFFFull ? 0xFFFFFFFFull : cap);
  tv.shortcut = (c.flags & HWAVE_F_NO_SHORTCUT) ? 0u : 1u;
  tv.no_erase = (c.flags & HWAVE_F_NO_ERASE) ? 1u : 0u;
  tv.aggregate = (c.flags & HWAVE_F_AGGREGATE) ? 1u : 0u;
  tv.lock_limit = (uint32_t)((c.lock_timeout_us ? c.lock_timeout_us : DEFAULT_LOCK_TIMEOUT_US) * 100ull);
  tv.hot_tag = L.off_hot ? (uint64_t*)(b + L.off_hot) : nullptr;
  tv.hot_acc = L.off_hot ? tv.hot_tag + HOT_N : nullptr;
  t->has_merge = L.off_merge != 0;
  t->ws = MergeWs{};
  if (t->has_merge) {
    uint8_t* m = b + L.off_merge;
    t->ws.key = (uint64_t*)m;
    t->ws.ent = (MergeEntry*)(m + MERGE_ENTRIES * 8);
    t->ws.op_ent = (uint32_t*)(m + MERGE_ENTRIES * (8 + sizeof(MergeEntry)));
    t->ws.ne_mask = (uint32_t)(MERGE_ENTRIES - 1);
    t->ws.chunk = MERGE_CHUNK;
  }
  tv.probe_ctr = nullptr;
#ifdef HW_INSTRUMENT
  {
    const size_t pb = (size_t)PROBE_STRIPES * 16 * sizeof(unsigned long long);
    e = hipMalloc((void**)&tv.probe_ctr, pb);
    if (e != hipSuccess) {
      tv.probe_ctr = nullptr;
      return hip_fail(e);
    }
    hipLaunchKernelGGL(k_fill16, dim3(1), dim3(256), 0, (hipStream_t)stream, (uint4*)tv.probe_ctr, pb / 16, 0u);
  }
#endif
  t->la.max_blocks = max_blocks_for(dev);
  const int rc = hwave_clear(t, stream);
  if (rc && tv.probe_ctr) {
    (void)hipFree(tv.probe_ctr);
    tv.probe_ctr = nullptr;
  }
  return rc;
}

bool bad_ptr(const void* p) { return p == nullptr; }

}  // namespace

extern "C" {

int hwave_config_default(hwave_design design, hwave_config* out) {
  if (!out || (int)design < HWAVE_DOUBLE || (int)design > HWAVE_CUCKOO) return HWAVE_EINVAL;
  defaults_for(design, 64, out);
  return HWAVE_OK;
}

int hwave_table_bytes(uint64_t capacity, hwave_design design, const hwave_config* cfg, uint64_t* bytes) {
  if (!bytes) return HWAVE_EINVAL;
  hwave_config c;
  int rc = resolve_config(design, cfg, &c);
  if (rc) return rc;
  if (!find_set(c, design)) return HWAVE_EUNSUPPORTED;
  Layout L;
  rc = layout_of(capacity, design, c, &L);
  if (rc) return rc;
  *bytes = L.total;
  return HWAVE_OK;
}

int hwave_create(hwave_table** out, uint64_t capacity, hwave_design design, const hwave_config* cfg,
                 void* stream) {
  if (!out) return HWAVE_EINVAL;
  *out = nullptr;
  hwave_config c;
  int rc = resolve_config(design, cfg, &c);
  if (rc) return rc;
  const KernelSet* ks = find_set(c, design);
  if (!ks) return HWAVE_EUNSUPPORTED;
  Layout L;
  rc = layout_of(capacity, design, c, &L);
  if (rc) return rc;
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, L.total);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    (void)hipGetLastError();
    return HWAVE_ENOMEM;
  }
  hwave_table* t = new hwave_table;
  t->owns = true;
  rc = init_table(t, base, L.total, L, design, c, ks, stream);
  if (rc) {
    (void)hipFree(base);
    delete t;
    return rc;
  }
  *out = t;
  return HWAVE_OK;
}

int hwave_create_in(hwave_table** out, void* d_buffer, uint64_t buffer_bytes, uint64_t capacity,
                    hwave_design design, const hwave_config* cfg, void* stream) {
  if (!out || !d_buffer || ((uintptr_t)d_buffer % ALIGN)) return HWAVE_EINVAL;
  *out = nullptr;
  hwave_config c;
  int rc = resolve_config(design, cfg, &c);
  if (rc) return rc;
  const KernelSet* ks = find_set(c, design);
  if (!ks) return HWAVE_EUNSUPPORTED;
  Layout L;
  rc = layout_of(capacity, design, c, &L);
  if (rc) return rc;
  if (buffer_bytes < L.total) return HWAVE_ENOMEM;
  hwave_table* t = new hwave_table;
  t->owns = false;
  rc = init_table(t, d_buffer, L.total, L, design, c, ks, stream);
  if (rc) {
    delete t;
    return rc;
  }
  *out = t;
  return HWAVE_OK;
}

int hwave_destroy(hwave_table* t) {
  if (!t) return HWAVE_EINVAL;
  drop_groups_of(t);
  hipError_t e = hipDeviceSynchronize();
  int rc = e == hipSuccess ? HWAVE_OK : hip_fail(e);
  if (t->la.tv.probe_ctr) (void)hipFree(t->la.tv.probe_ctr);
  if (t->owns) {
    e = hipFree(t->base);
    if (e != hipSuccess && rc == HWAVE_OK) rc = hip_fail(e);
  }
  delete t;
  return rc;
}

int hwave_clear(hwave_table* t, void* stream) {
  if (!t) return HWAVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // Every region size is a multiple of 256 bytes.  Slots and tags: all-ones
  // (empty); locks and control word: zero.
  const uint64_t fill_end = (uint64_t)((uint8_t*)t->la.tv.locks.words - (uint8_t*)t->base);
  hipLaunchKernelGGL(k_fill16, dim3(stream_grid(fill_end / 16, t->device)), dim3(256), 0, s,
                     (uint4*)t->base, fill_end / 16, 0xFFFFFFFFu);
  const uint64_t zero_bytes = t->bytes - fill_end;
  hipLaunchKernelGGL(k_fill16, dim3(stream_grid(zero_bytes / 16, t->device)), dim3(256), 0, s,
                     (uint4*)t->la.tv.locks.words, zero_bytes / 16, 0u);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_insert(hwave_table* t, const void* d_keys, const void* d_vals, uint64_t n, uint8_t* d_status,
                 void* stream) {
  return hwave_upsert(t, d_keys, d_vals, n, HWAVE_KEEP, d_status, stream);
}

int hwave_upsert(hwave_table* t, const void* d_keys, const void* d_vals, uint64_t n, hwave_combine combine,
                 uint8_t* d_status, void* stream) {
  if (!t || (int)combine < HWAVE_SUM || (int)combine > HWAVE_MAX) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  if (bad_ptr(d_keys) || bad_ptr(d_vals)) return HWAVE_EINVAL;
  hipError_t e = t->ks->upsert(t->la, d_keys, d_vals, n, (int)combine, d_status, (hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_query(hwave_table* t, const void* d_keys, uint64_t n, void* d_vals_out, uint8_t* d_found,
                void* stream) {
  if (!t) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  if (bad_ptr(d_keys)) return HWAVE_EINVAL;
  hipError_t e = t->ks->query(t->la, d_keys, n, d_vals_out, d_found, (hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_erase(hwave_table* t, const void* d_keys, uint64_t n, uint8_t* d_found, void* stream) {
  if (!t || t->la.tv.no_erase) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  if (bad_ptr(d_keys)) return HWAVE_EINVAL;
  hipError_t e = t->ks->erase(t->la, d_keys, n, d_found, (hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_mixed(hwave_table* t, const uint8_t* d_ops, const void* d_keys, const void* d_vals, uint64_t n,
                hwave_combine combine, void* d_vals_out, uint8_t* d_status, void* stream) {
  if (!t || (int)combine < HWAVE_SUM || (int)combine > HWAVE_MAX) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  if (bad_ptr(d_ops) || bad_ptr(d_keys)) return HWAVE_EINVAL;
  // Values are read only for inserts/upserts; a batch without them may pass NULL,
  // in which case the keys array stands in (never dereferenced for other ops).
  const void* vals = d_vals ? d_vals : d_keys;
  hipError_t e = t->ks->mixed(t->la, d_ops, d_keys, vals, n, (int)combine, d_vals_out, d_status,
                              t->has_merge ? &t->ws : nullptr, (hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

}  // extern "C"

namespace {

// The workspace of hwave_mixed_noalloc: one merge workspace (hw_merge.hpp) for
// chunks of NOALLOC_OPS operations, in a fixed device array that each device
// holds for the life of the process.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address comes from
// hipGetSymbolAddress, once per device (noalloc_ws), and only that address is
// ever given to kernels.
constexpr uint32_t NOALLOC_OPS = 1u << 18;
constexpr uint64_t NOALLOC_ENTRIES = 2ull * NOALLOC_OPS;
constexpr uint64_t NOALLOC_ZERO_BYTES = NOALLOC_ENTRIES * (8 + sizeof(MergeEntry));  // key words + entries
constexpr uint64_t NOALLOC_BYTES = NOALLOC_ZERO_BYTES + (uint64_t)NOALLOC_OPS * 4;  // + per-op words
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];

// Device address of this device's `scratch`, looked up on the first call per
// device (with that device current).  NULL on failure (*err set).
uint8_t* noalloc_base(int device, hipError_t* err) {
  if (device < 0 || device >= 64) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    g_noalloc_ptr[device] = ptr;
  }
  return (uint8_t*)g_noalloc_ptr[device];
}

}  // namespace

extern "C" {

int hwave_mixed_noalloc(hwave_table* t, const uint8_t* d_ops, const void* d_keys, const void* d_vals, uint64_t n,
                        hwave_combine combine, void* d_vals_out, uint8_t* d_status, void* stream) {
  if (!t || (int)combine < HWAVE_SUM || (int)combine > HWAVE_MAX) return HWAVE_EINVAL;
  if (n > NOALLOC_OPS) return HWAVE_ETOOBIG;
  if (n == 0) return HWAVE_OK;
  if (bad_ptr(d_ops) || bad_ptr(d_keys)) return HWAVE_EINVAL;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e);
  if (cur != t->device) return HWAVE_EINVAL;  // the table's device must be current
  uint8_t* base = noalloc_base(cur, &e);
  if (!base) return hip_fail(e);
  MergeWs ws;
  ws.key = (uint64_t*)base;
  ws.ent = (MergeEntry*)(base + NOALLOC_ENTRIES * 8);
  ws.op_ent = (uint32_t*)(base + NOALLOC_ZERO_BYTES);
  ws.ne_mask = (uint32_t)(NOALLOC_ENTRIES - 1);
  ws.chunk = NOALLOC_OPS;
  hipStream_t s = (hipStream_t)stream;
  // the array keeps the last call's contents: the entries must start empty (all
  // zero); a fill kernel, not a memset, so the call can be captured in a graph
  hipLaunchKernelGGL(k_fill16, dim3(stream_grid(NOALLOC_ZERO_BYTES / 16, cur)), dim3(256), 0, s, (uint4*)base,
                     NOALLOC_ZERO_BYTES / 16, 0u);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  const void* vals = d_vals ? d_vals : d_keys;
  e = t->ks->mixed(t->la, d_ops, d_keys, vals, n, (int)combine, d_vals_out, d_status, &ws, s);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_size(hwave_table* t, uint64_t* d_count, void* stream) {
  if (!t || !d_count) return HWAVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_count);
  const unsigned g = stream_grid(t->units, t->device);
  if (t->cfg.kv_bits == 64)
    hipLaunchKernelGGL(k_count<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t*)t->base, t->units, d_count);
  else
    hipLaunchKernelGGL(k_count<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t*)t->base, t->units, d_count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_export(hwave_table* t, void* d_keys, void* d_vals, uint64_t* d_count, void* stream) {
  if (!t || !d_keys || !d_vals || !d_count) return HWAVE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_count);
  const unsigned g = stream_grid(t->units, t->device);
  if (t->cfg.kv_bits == 64)
    hipLaunchKernelGGL(k_export<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t*)t->base, t->units,
                       (uint64_t*)d_keys, (uint64_t*)d_vals, d_count);
  else
    hipLaunchKernelGGL(k_export<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t*)t->base, t->units,
                       (uint32_t*)d_keys, (uint32_t*)d_vals, d_count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

uint64_t hwave_num_buckets(const hwave_table* t) { return t ? t->nb : 0; }
uint64_t hwave_capacity(const hwave_table* t) { return t ? t->capacity : 0; }

int hwave_primary_bucket(hwave_table* t, const void* d_keys, uint64_t n, uint64_t* d_out, void* stream) {
  if (!t || (n && (!d_keys || !d_out))) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = stream_grid(n, t->device);
  const uint32_t nf = design_iceberg(t->design) || design_chain(t->design) ? t->la.tv.nb_front : 0u;
  if (t->cfg.kv_bits == 64)
    hipLaunchKernelGGL(k_primary<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t*)d_keys, n,
                       t->la.tv.bucket_mask, nf, d_out);
  else
    hipLaunchKernelGGL(k_primary<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t*)d_keys, n,
                       t->la.tv.bucket_mask, nf, d_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_candidate_buckets(hwave_table* t, const void* d_keys, uint64_t n, uint64_t* d_out, void* stream) {
  if (!t || (n && (!d_keys || !d_out))) return HWAVE_EINVAL;
  if (n == 0) return HWAVE_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = stream_grid(n, t->device);
  const TableDev& tv = t->la.tv;
  if (t->cfg.kv_bits == 64)
    hipLaunchKernelGGL(k_candidates<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t*)d_keys, n,
                       (int)t->design, tv.bucket_mask, tv.nb_front, tv.nb_back, d_out);
  else
    hipLaunchKernelGGL(k_candidates<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t*)d_keys, n,
                       (int)t->design, tv.bucket_mask, tv.nb_front, tv.nb_back, d_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_probe_counters(hwave_table* t, hwave_probe_stats* out, int reset, void* stream) {
  if (!t || !out) return HWAVE_EINVAL;
  memset(out, 0, sizeof *out);
  unsigned long long* d = t->la.tv.probe_ctr;
  if (!d) return HWAVE_EUNSUPPORTED;  // not an instrumented build
  hipStream_t s = (hipStream_t)stream;
  std::vector<unsigned long long> h((size_t)PROBE_STRIPES * 16);
  hipError_t e = hipMemcpyAsync(h.data(), d, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  for (uint32_t i = 0; i < PROBE_STRIPES; i++) {
    out->bucket_lines += h[i * 16 + PC_BUCKET];
    out->slot_lines += h[i * 16 + PC_SLOT];
    out->queries += h[i * 16 + PC_QUERY];
    out->writes += h[i * 16 + PC_WRITE];
    out->write_visits += h[i * 16 + PC_VISIT];
  }
  if (reset) {
    hipLaunchKernelGGL(k_fill16, dim3(1), dim3(256), 0, s, (uint4*)d, h.size() * sizeof(unsigned long long) / 16, 0u);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
  }
  return HWAVE_OK;
}

int hwave_raw(const hwave_table* t, hwave_raw_view* out) {
  if (!t || !out) return HWAVE_EINVAL;
  out->slots = t->la.tv.slots;
  out->tags = (uint16_t*)t->la.tv.tagw;
  out->locks = t->la.tv.locks.words;
  out->n_lock_words = t->n_lock_words;
  out->lock_stride = 1u << t->la.tv.locks.shift;
  out->lock_queues = t->la.tv.lockq;
  out->n_lock_queues = (uint64_t)t->la.tv.lockq_mask + 1;
  out->num_buckets = t->nb;
  out->bucket_slots = t->cfg.bucket_slots;
  out->tile = t->cfg.tile;
  out->kv_bits = t->cfg.kv_bits;
  out->design = (uint32_t)t->design;
  out->slot_bytes = t->units * (t->cfg.kv_bits / 4);
  return HWAVE_OK;
}

const char* hwave_strerror(int code) {
  switch (code) {
    case HWAVE_OK: return "ok";
    case HWAVE_EINVAL: return "invalid argument";
    case HWAVE_ENOMEM: return "out of device memory or buffer too small";
    case HWAVE_EDEVICE: return "HIP error (see hwave_last_hip_error)";
    case HWAVE_EUNSUPPORTED: return "no kernel instance for this configuration";
    case HWAVE_EIO: return "file could not be read or written, or is malformed";
    case HWAVE_ETOOBIG: return "batch larger than the allocation-free call's fixed workspace";
  }
  return "unknown error";
}

int hwave_last_hip_error(void) { return g_last_hip_error; }

// ---------------------------------------------------------------- multi-table

}  // extern "C"

struct hwave_multi {
  int device;
  int kv_bits;
  int menu;  // MENU_BASE, MENU_EXT or MENU_SOLO
  int solo;  // menu entry shared by every table (MENU_SOLO), else -1
  bool agg;  // some table merges duplicate keys (64-bit solo kernels: the merging path)
  uint32_t n_tables;
  std::vector<uint64_t> table_bytes;  // footprint per table (queue placement)
  MultiTable* d_tables = nullptr;
  uint32_t* d_heads = nullptr;
  uint32_t* d_hot = nullptr;  // indices of the tables with hot-key accumulators the kernel fills
  uint32_t n_hot = 0;
  MultiItem* d_items = nullptr;
  size_t items_cap = 0;
  MultiItem* h_stage = nullptr;  // pinned staging of the item list
  size_t stage_cap = 0;
  hipEvent_t staged = nullptr;   // recorded after the last item upload
  bool staged_pending = false;
  unsigned grid = 0;
  std::vector<MultiItem> build;  // host scratch
  std::vector<uint32_t> qcount;
};

namespace {

// Items are split into chunks of at most this many ops so the queues balance big
// tables; the chunk shrinks (down to MULTI_CHUNK_MIN) when a launch has too little
// work to give every wave of the persistent grid several chunks.
constexpr uint64_t MULTI_CHUNK = 16384;
constexpr uint64_t MULTI_CHUNK_MIN = 256;
// Tables whose footprint fits comfortably in one XCD's L2 keep all their items on
// one queue.
constexpr uint64_t L2_RESIDENT_BYTES = 2ull << 20;

int multi_reserve(hwave_multi* m, size_t n) {
  if (n <= m->items_cap && n <= m->stage_cap) return HWAVE_OK;
  size_t cap = 1024;
  while (cap < n) cap <<= 1;
  hipError_t e = hipDeviceSynchronize();  // the old buffers may still be read by a launch
  if (e != hipSuccess) return hip_fail(e);
  if (m->d_items) (void)hipFree(m->d_items);
  if (m->h_stage) (void)hipHostFree(m->h_stage);
  m->d_items = nullptr;
  m->h_stage = nullptr;
  m->items_cap = m->stage_cap = 0;
  e = hipMalloc(&m->d_items, cap * sizeof(MultiItem));
  if (e != hipSuccess) { g_last_hip_error = (int)e; return HWAVE_ENOMEM; }
  e = hipHostMalloc((void**)&m->h_stage, cap * sizeof(MultiItem), hipHostMallocDefault);
  if (e != hipSuccess) { g_last_hip_error = (int)e; return HWAVE_ENOMEM; }
  m->items_cap = m->stage_cap = cap;
  m->staged_pending = false;
  return HWAVE_OK;
}

}  // namespace

extern "C" {

int hwave_multi_supported(uint32_t kv_bits, hwave_design design, uint32_t bucket_slots, uint32_t tile) {
  for (int menu : {MENU_BASE, MENU_EXT})
    if (multi_menu_index((int)kv_bits, menu, (int)design, (int)bucket_slots, (int)tile) >= 0) return 1;
  return 0;
}

int hwave_multi_create(hwave_multi** out, hwave_table* const* tables, uint32_t n_tables, void* stream) {
  if (!out || !tables || n_tables == 0) return HWAVE_EINVAL;
  *out = nullptr;
  const int kv = (int)tables[0]->cfg.kv_bits;
  const int dev = tables[0]->device;
  // the base menu when it holds every table's configuration, else the extended one
  int menu = MENU_BASE;
  for (uint32_t i = 0; i < n_tables; i++) {
    const hwave_table* t = tables[i];
    if (!t || (int)t->cfg.kv_bits != kv || t->device != dev) return HWAVE_EINVAL;
    if (t->cfg.flags & HWAVE_F_BSP) return HWAVE_EUNSUPPORTED;
    if (multi_menu_index(kv, MENU_BASE, (int)t->design, (int)t->cfg.bucket_slots, (int)t->cfg.tile) < 0)
      menu = MENU_EXT;
  }
  std::vector<MultiTable> h(n_tables);
  for (uint32_t i = 0; i < n_tables; i++) {
    const hwave_table* t = tables[i];
    int cls = multi_menu_index(kv, menu, (int)t->design, (int)t->cfg.bucket_slots, (int)t->cfg.tile);
    if (cls < 0) return HWAVE_EUNSUPPORTED;
    h[i].tv = t->la.tv;
    h[i].cls = (uint32_t)cls;
    h[i].pad = 0;
    const uint64_t locks_off = (uint64_t)((uint8_t*)t->la.tv.locks.words - (uint8_t*)t->base);
    h[i].fill_words = locks_off / 16;
    h[i].zero_words = (t->bytes - locks_off) / 16;
  }
  // every table on one configuration: that configuration's own kernel (its
  // entry in the 32-bit menu or in the 64-bit extended menu)
  int solo = (int)h[0].cls;
  for (uint32_t i = 1; i < n_tables && solo >= 0; i++)
    if ((int)h[i].cls != solo) solo = -1;
  if (solo >= 0) {
    const hwave_table* t = tables[0];
    solo = multi_menu_index(kv, MENU_SOLO, (int)t->design, (int)t->cfg.bucket_slots, (int)t->cfg.tile);
    if (solo < 0) return HWAVE_EUNSUPPORTED;
    menu = MENU_SOLO;
    for (uint32_t i = 0; i < n_tables; i++) h[i].cls = 0;
  }
  hwave_multi* m = new hwave_multi;
  m->device = dev;
  m->kv_bits = kv;
  m->menu = menu;
  m->solo = solo;
  m->agg = false;
  for (uint32_t i = 0; i < n_tables; i++) m->agg = m->agg || tables[i]->la.tv.aggregate;
  m->n_tables = n_tables;
  for (uint32_t i = 0; i < n_tables; i++) m->table_bytes.push_back(tables[i]->bytes);
  // only the 64-bit menu carries the merging path that fills the accumulators
  std::vector<uint32_t> hot;
  for (uint32_t i = 0; i < n_tables; i++)
    if (kv == 64 && tables[i]->la.tv.hot_tag) hot.push_back(i);
  m->n_hot = (uint32_t)hot.size();
  hipError_t e = hipMalloc(&m->d_tables, n_tables * sizeof(MultiTable));
  if (e == hipSuccess && m->n_hot) e = hipMalloc(&m->d_hot, m->n_hot * sizeof(uint32_t));
  if (e == hipSuccess && m->n_hot)
    e = hipMemcpyAsync(m->d_hot, hot.data(), m->n_hot * sizeof(uint32_t), hipMemcpyHostToDevice,
                       (hipStream_t)stream);
  if (e == hipSuccess) e = hipMalloc(&m->d_heads, NQ * HEAD_STRIDE * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_tables, h.data(), n_tables * sizeof(MultiTable),
                                          hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    hwave_multi_destroy(m);
    return hip_fail(e);
  }
  // Persistent grid: full occupancy of the multi-table kernel.
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  m->grid = (unsigned)cus * (4 * multi_waves(kv, menu, solo, m->agg) * 64 / BLOCK);
  *out = m;
  return HWAVE_OK;
}

int hwave_multi_kernel(const hwave_multi* m, uint32_t* kernel, uint32_t* waves) {
  if (!m) return HWAVE_EINVAL;
  static_assert(HWAVE_MULTI_MENU == MENU_BASE && HWAVE_MULTI_EXTENDED == MENU_EXT && HWAVE_MULTI_SOLO == MENU_SOLO,
                "kernel codes");
  if (kernel) *kernel = (uint32_t)m->menu;
  if (waves) *waves = (uint32_t)multi_waves(m->kv_bits, m->menu, m->solo, m->agg);
  return HWAVE_OK;
}

int hwave_multi_destroy(hwave_multi* m) {
  if (!m) return HWAVE_EINVAL;
  (void)hipDeviceSynchronize();
  if (m->d_tables) (void)hipFree(m->d_tables);
  if (m->d_heads) (void)hipFree(m->d_heads);
  if (m->d_hot) (void)hipFree(m->d_hot);
  if (m->d_items) (void)hipFree(m->d_items);
  if (m->h_stage) (void)hipHostFree(m->h_stage);
  if (m->staged) (void)hipEventDestroy(m->staged);
  delete m;
  return HWAVE_OK;
}

int hwave_multi_run(hwave_multi* m, const hwave_item* h_items, uint32_t n_items, const void* d_keys,
                    const void* d_vals, void* d_vals_out, uint8_t* d_status, void* stream) {
  if (!m || (n_items && (!h_items || !d_keys))) return HWAVE_EINVAL;
  if (n_items == 0) return HWAVE_OK;
  // Split items into chunks and deal them to queues: small tables to queue
  // table % NQ, big tables' chunks round-robin over all queues.
  m->build.clear();
  std::vector<std::vector<MultiItem>> per_q(NQ);
  uint32_t rr = 0;
  uint64_t total_ops = 0;
  bool merging = false;  // an upsert whose combine merges (it may fill hot-key accumulators)
  for (uint32_t i = 0; i < n_items; i++)
    if (h_items[i].end > h_items[i].begin) total_ops += h_items[i].end - h_items[i].begin;
  const uint64_t waves = (uint64_t)m->grid * (BLOCK / 64);
  uint64_t chunk = total_ops / (4 * waves);
  if (chunk > MULTI_CHUNK) chunk = MULTI_CHUNK;
  if (chunk < MULTI_CHUNK_MIN) chunk = MULTI_CHUNK_MIN;
  for (uint32_t i = 0; i < n_items; i++) {
    const hwave_item& it = h_items[i];
    if (it.table >= m->n_tables || it.end < it.begin) return HWAVE_EINVAL;
    const int op = (int)(it.op & 0xFF);
    if (op > HWAVE_OP_ERASE || ((it.op >> 8) & 0xFF) > HWAVE_MAX) return HWAVE_EINVAL;
    if ((op == HWAVE_OP_INSERT || op == HWAVE_OP_UPSERT) && !d_vals) return HWAVE_EINVAL;
    const int comb = (int)((it.op >> 8) & 0xFF);
    if (op == HWAVE_OP_UPSERT && (comb == HWAVE_SUM || comb == HWAVE_MIN || comb == HWAVE_MAX)) merging = true;
    const bool small = m->table_bytes[it.table] <= L2_RESIDENT_BYTES;
    for (uint64_t b = it.begin; b < it.end; b += chunk) {
      MultiItem c;
      c.table = it.table;
      c.op = it.op;
      c.begin = b;
      c.end = b + chunk < it.end ? b + chunk : it.end;
      const uint32_t q = small ? it.table % NQ : (rr++ % NQ);
      per_q[q].push_back(c);
    }
  }
  size_t total = 0;
  for (auto& v : per_q) total += v.size();
  if (total == 0) return HWAVE_OK;
  if (total > 0xFFFFFFFFull) return HWAVE_EINVAL;
  int rc = multi_reserve(m, total);
  if (rc) return rc;
  // the staging buffer may still be in flight from the previous call
  if (m->staged_pending) {
    hipError_t e = hipEventSynchronize(m->staged);
    if (e != hipSuccess) return hip_fail(e);
  }
  MultiQueues qs;
  size_t at = 0;
  for (int q = 0; q < NQ; q++) {
    qs.start[q] = (uint32_t)at;
    memcpy(m->h_stage + at, per_q[q].data(), per_q[q].size() * sizeof(MultiItem));
    at += per_q[q].size();
    qs.end[q] = (uint32_t)at;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(m->d_items, m->h_stage, total * sizeof(MultiItem), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(m->staged, s);
  if (e != hipSuccess) return hip_fail(e);
  m->staged_pending = true;
  e = launch_multi(m->kv_bits, m->menu, m->solo, m->agg, m->grid, m->d_tables, m->d_items, qs, m->d_heads, d_keys,
                   d_vals ? d_vals : d_keys, d_vals_out, d_status, s);
  if (e == hipSuccess && merging) e = launch_multi_hot_flush(m->kv_bits, m->d_tables, m->d_hot, m->n_hot, s);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_multi_clear(hwave_multi* m, void* stream) {
  if (!m) return HWAVE_EINVAL;
  const unsigned grid = m->n_tables < 4096 ? m->n_tables : 4096;
  hipError_t e = launch_multi_clear(grid, m->d_tables, m->n_tables, (hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

int hwave_multi_upsert(hwave_multi* m, const uint64_t* h_offsets, const void* d_keys, const void* d_vals,
                       hwave_combine combine, uint8_t* d_status, void* stream) {
  if (!m || !h_offsets || (int)combine < HWAVE_SUM || (int)combine > HWAVE_MAX) return HWAVE_EINVAL;
  std::vector<hwave_item> items;
  items.reserve(m->n_tables);
  for (uint32_t i = 0; i < m->n_tables; i++) {
    if (h_offsets[i + 1] < h_offsets[i]) return HWAVE_EINVAL;
    if (h_offsets[i + 1] == h_offsets[i]) continue;
    items.push_back(hwave_item{i, (uint32_t)HWAVE_OP_UPSERT | ((uint32_t)combine << 8), h_offsets[i],
                               h_offsets[i + 1]});
  }
  return hwave_multi_run(m, items.data(), (uint32_t)items.size(), d_keys, d_vals, nullptr, d_status, stream);
}

}  // extern "C"

namespace {

// Groups made by hwave_multi_upsert_tables, one per distinct table list, kept
// until one of their tables is destroyed.
std::mutex g_groups_mu;
std::vector<std::pair<std::vector<hwave_table*>, hwave_multi*>> g_groups;

}  // namespace

// Called by hwave_destroy: groups that hold `t` go with it.
static void drop_groups_of(hwave_table* t) {
  std::lock_guard<std::mutex> g(g_groups_mu);
  for (size_t i = 0; i < g_groups.size();) {
    const auto& v = g_groups[i].first;
    if (std::find(v.begin(), v.end(), t) != v.end()) {
      hwave_multi_destroy(g_groups[i].second);
      g_groups.erase(g_groups.begin() + (long)i);
    } else {
      ++i;
    }
  }
}

extern "C" {

int hwave_multi_upsert_tables(hwave_table* const* tables, uint32_t n_tables, const uint64_t* d_offsets,
                              const void* d_keys, const void* d_vals, hwave_combine combine, uint8_t* d_status,
                              void* stream) {
  if (!tables || n_tables == 0 || !d_offsets || (int)combine < HWAVE_SUM || (int)combine > HWAVE_MAX)
    return HWAVE_EINVAL;
  std::vector<hwave_table*> key(tables, tables + n_tables);
  hwave_multi* m = nullptr;
  {
    std::lock_guard<std::mutex> g(g_groups_mu);
    for (auto& e : g_groups)
      if (e.first == key) m = e.second;
    if (!m) {
      const int rc = hwave_multi_create(&m, tables, n_tables, stream);
      if (rc) return rc;
      g_groups.emplace_back(key, m);
    }
  }
  std::vector<uint64_t> h(n_tables + 1);
  hipError_t e = hipMemcpyAsync(h.data(), d_offsets, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  if (h[0] != 0) return HWAVE_EINVAL;
  return hwave_multi_upsert(m, h.data(), d_keys, d_vals, combine, d_status, stream);
}

int hwave_stream_sync(void* stream) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  return e == hipSuccess ? HWAVE_OK : hip_fail(e);
}

}  // extern "C"

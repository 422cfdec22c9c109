// Autotuner: picks a table configuration (design, bucket size, tile width) for a
// capacity class by timing every candidate of the multi-table menu on the work
// it will run -- a group-by SUM upsert batch that fills tables of that class to
// the requested load, spread over enough tables of the class to fill the GPU,
// through the persistent multi-table kernel.  The paper tunes bucket and tile
// size by exhaustive search per design (Section 5); this does the same per
// capacity class, at run time.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include <cstring>
#include <vector>

#include "hashwave.h"
#include "hw_multi.hpp"

using namespace hw;

namespace {

// Bijective 64-bit and 32-bit mixers (the splitmix64 output function, and
// Wellons' "lowbias32"): distinct indices give distinct synthetic keys.
__device__ __forceinline__ uint64_t bij64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint32_t bij32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Group-by batch for n_tab tables: table t gets ops [t*2D, (t+1)*2D): its D
// distinct keys interleaved with D repeats drawn from them; values pseudo-random.
template <typename K>
__global__ void k_gen_groupby(K* keys, K* vals, uint32_t n_tab, uint64_t D, uint64_t seed) {
  const uint64_t total = (uint64_t)n_tab * 2 * D;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t t = i / (2 * D), j = i % (2 * D);
    const uint64_t idx = (j & 1) ? bij64(seed ^ (i * 0x9E3779B97F4A7C15ull)) % D : (j >> 1);
    K k;
    if constexpr (sizeof(K) == 8) {
      k = bij64(idx + t * 0x100000000ull + seed);
      if (k >= Keys<uint64_t>::FIRST_INVALID) k >>= 1;
    } else {
      k = bij32((uint32_t)(idx + (uint32_t)seed));
      if (k >= Keys<uint32_t>::FIRST_INVALID) k >>= 1;
    }
    keys[i] = k;
    vals[i] = (K)bij64(i + seed * 3);
  }
}

__global__ void k_zero_count(unsigned long long* c) { *c = 0; }

// Adds the number of status bytes equal to `code` to *count.
__global__ void k_count_status(const uint8_t* __restrict__ st, uint64_t n, uint8_t code,
                               unsigned long long* __restrict__ count) {
  unsigned long long c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    c += st[i] == code;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

}  // namespace

extern "C" {

int hwave_autotune(uint32_t kv_bits, uint64_t capacity, uint32_t design_mask, double load, uint32_t reps,
                   uint32_t flags, hwave_tune_result* results, uint32_t results_cap, uint32_t* n_results,
                   hwave_tune_result* best, void* stream) {
  if ((kv_bits != 32 && kv_bits != 64) || capacity == 0 || !(load > 0.0 && load <= 1.0) || !best)
    return HWAVE_EINVAL;
  if (n_results) *n_results = 0;
  hipStream_t s = (hipStream_t)stream;
  int n_menu = 0;
  // 64-bit keys: every configuration of the extended menu (a group of one
  // configuration runs on the base menu whenever that holds it)
  const MenuEntry* menu = kv_bits == 64 ? menu_entries(MenuU64X{}, &n_menu) : menu_entries(MenuU32{}, &n_menu);
  if (reps == 0) reps = 3;
  // enough tables of this class to give each timed launch ~32M slots of work
  // (tens of milliseconds), so that launch and tail effects do not decide
  uint64_t n_tab64 = (32ull << 20) / capacity;
  if (n_tab64 < 1) n_tab64 = 1;
  if (n_tab64 > 8192) n_tab64 = 8192;
  const uint32_t n_tab = (uint32_t)n_tab64;
  memset(best, 0, sizeof *best);
  best->gops = -1.0;
  best->load = load;
  best->flags = flags;
  uint32_t nres = 0;
  const size_t kb = kv_bits / 8;
  for (int c = 0; c < n_menu; c++) {
    const hwave_design d = (hwave_design)menu[c].design;
    if (!(design_mask & (1u << d))) continue;
    hwave_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.kv_bits = kv_bits;
    cfg.bucket_slots = (uint32_t)menu[c].bucket;
    cfg.tile = (uint32_t)menu[c].tile;
    cfg.flags = flags;
    uint64_t tb = 0;
    int rc = hwave_table_bytes(capacity, d, &cfg, &tb);
    if (rc == HWAVE_EUNSUPPORTED) continue;
    if (rc) return rc;
    const uint64_t real_cap = [&] {
      const uint64_t want = (capacity + cfg.bucket_slots - 1) / cfg.bucket_slots;
      if (d == HWAVE_CHAINING) return want * cfg.bucket_slots;  // bucket nodes; the pool is spare
      uint64_t nb = 1;
      while (nb < want) nb <<= 1;
      return nb * cfg.bucket_slots;
    }();
    const uint64_t D = (uint64_t)(load * (double)real_cap);
    if (D == 0) continue;
    const uint64_t n_ops = (uint64_t)n_tab * 2 * D;
    uint8_t* region = nullptr;
    void *keys = nullptr, *vals = nullptr;
    uint8_t* status = nullptr;
    unsigned long long* n_full = nullptr;
    hipError_t e = hipMalloc(&region, tb * n_tab);
    if (e == hipSuccess) e = hipMalloc(&keys, n_ops * kb);
    if (e == hipSuccess) e = hipMalloc(&vals, n_ops * kb);
    if (e == hipSuccess) e = hipMalloc(&status, n_ops);
    if (e == hipSuccess) e = hipMalloc(&n_full, sizeof(unsigned long long));
    if (e != hipSuccess) {
      if (region) (void)hipFree(region);
      if (keys) (void)hipFree(keys);
      if (vals) (void)hipFree(vals);
      if (status) (void)hipFree(status);
      if (n_full) (void)hipFree(n_full);
      return HWAVE_ENOMEM;
    }
    std::vector<hwave_table*> tabs(n_tab, nullptr);
    for (uint32_t t = 0; t < n_tab && rc == HWAVE_OK; t++)
      rc = hwave_create_in(&tabs[t], region + tb * t, tb, capacity, d, &cfg, stream);
    hwave_multi* m = nullptr;
    if (rc == HWAVE_OK) rc = hwave_multi_create(&m, tabs.data(), n_tab, stream);
    std::vector<uint64_t> offs(n_tab + 1);
    for (uint32_t t = 0; t <= n_tab; t++) offs[t] = (uint64_t)t * 2 * D;
    float total_ms = 0.f;
    if (rc == HWAVE_OK) {
      if (kv_bits == 64)
        hipLaunchKernelGGL(k_gen_groupby<uint64_t>, dim3(2048), dim3(256), 0, s, (uint64_t*)keys, (uint64_t*)vals,
                           n_tab, D, 0x5eedull + c);
      else
        hipLaunchKernelGGL(k_gen_groupby<uint32_t>, dim3(2048), dim3(256), 0, s, (uint32_t*)keys, (uint32_t*)vals,
                           n_tab, D, 0x5eedull + c);
      hipEvent_t a, b;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      for (uint32_t r = 0; r <= reps && rc == HWAVE_OK; r++) {  // r == 0: warmup
        rc = hwave_multi_clear(m, stream);
        if (rc) break;
        (void)hipEventRecord(a, s);
        rc = hwave_multi_upsert(m, offs.data(), keys, vals, HWAVE_SUM, status, stream);
        (void)hipEventRecord(b, s);
        if (hipEventSynchronize(b) != hipSuccess) rc = HWAVE_EDEVICE;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (r > 0) total_ms += ms;
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
    unsigned long long full = 0;
    if (rc == HWAVE_OK) {  // FULL statuses of the last run
      hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, n_full);
      hipLaunchKernelGGL(k_count_status, dim3(1024), dim3(256), 0, s, (const uint8_t*)status, n_ops,
                         (uint8_t)HWAVE_ST_FULL, n_full);
      if (hipMemcpyAsync(&full, n_full, sizeof full, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        rc = HWAVE_EDEVICE;
    }
    if (m) hwave_multi_destroy(m);
    for (auto* t : tabs)
      if (t) hwave_destroy(t);
    (void)hipFree(region);
    (void)hipFree(keys);
    (void)hipFree(vals);
    (void)hipFree(status);
    (void)hipFree(n_full);
    if (rc) return rc;
    hwave_tune_result res;
    res.design = (uint32_t)d;
    res.bucket_slots = cfg.bucket_slots;
    res.tile = cfg.tile;
    res.kv_bits = kv_bits;
    res.gops = (double)n_ops * reps / ((double)total_ms * 1e6);
    res.full_ops = full;
    res.load = load;
    res.flags = flags;
    res.reserved = 0;
    if (results && nres < results_cap) results[nres] = res;
    nres++;
    if (full == 0 && res.gops > best->gops) *best = res;
  }
  if (n_results) *n_results = nres;
  return best->gops > 0 ? HWAVE_OK : HWAVE_EUNSUPPORTED;
}

int hwave_tune_save(const char* path, const uint32_t* log2_capacity, const hwave_tune_result* best, uint32_t n) {
  if (!path || (n && (!log2_capacity || !best))) return HWAVE_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return HWAVE_EIO;
  bool ok = fprintf(f, "hwave-tune 2\n") > 0;
  for (uint32_t i = 0; ok && i < n; i++) {
    const hwave_tune_result& r = best[i];
    ok = fprintf(f, "%u %.17g %u %u %u %u %u %.17g %llu\n", log2_capacity[i], r.load, r.flags, r.kv_bits, r.design,
                 r.bucket_slots, r.tile, r.gops, (unsigned long long)r.full_ops) > 0;
  }
  ok = (fclose(f) == 0) && ok;
  return ok ? HWAVE_OK : HWAVE_EIO;
}

int hwave_tune_load(const char* path, uint32_t* log2_capacity, hwave_tune_result* best, uint32_t cap,
                    uint32_t* n) {
  if (!path || !n || (cap && (!log2_capacity || !best))) return HWAVE_EINVAL;
  *n = 0;
  FILE* f = fopen(path, "r");
  if (!f) return HWAVE_EIO;
  char line[256];
  int rc = HWAVE_OK;
  if (!fgets(line, sizeof line, f) || strcmp(line, "hwave-tune 2\n") != 0) rc = HWAVE_EIO;
  uint32_t count = 0;
  const unsigned known_flags = HWAVE_F_NO_SHORTCUT | HWAVE_F_NO_ERASE | HWAVE_F_BSP | HWAVE_F_AGGREGATE;
  while (rc == HWAVE_OK && fgets(line, sizeof line, f)) {
    unsigned e, fl, kv, d, b, t;
    double ld, g;
    unsigned long long full;
    char tail;
    if (sscanf(line, "%u %lg %u %u %u %u %u %lg %llu %c", &e, &ld, &fl, &kv, &d, &b, &t, &g, &full, &tail) != 9 ||
        e > 40 || !(ld > 0.0 && ld <= 1.0) || (fl & ~known_flags) || (kv != 32 && kv != 64) ||
        d > (unsigned)HWAVE_CUCKOO || b == 0 || b > 1024 || t == 0 || t > 64 || count == cap) {
      rc = HWAVE_EIO;
      break;
    }
    log2_capacity[count] = e;
    hwave_tune_result& r = best[count];
    r.design = d;
    r.bucket_slots = b;
    r.tile = t;
    r.kv_bits = kv;
    r.gops = g;
    r.full_ops = full;
    r.load = ld;
    r.flags = fl;
    r.reserved = 0;
    count++;
  }
  fclose(f);
  if (rc == HWAVE_OK) *n = count;
  return rc;
}

}  // extern "C"

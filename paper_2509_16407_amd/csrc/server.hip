// Serving loop: continuous batching of table requests onto one GPU.
//
// Requests (one table, one operation kind, n keys in pinned host memory) are
// queued by hwave_server_submit.  A worker thread admits pending requests into a
// batch while the batch's request data fits one device staging slot (admission
// by memory) and no admitted request conflicts, packs them into one persistent
// multi-table launch, and overlaps batches: host-to-device copies, kernels and
// device-to-host copies run on three streams, with up to `slots` batches in
// flight, so requests arriving while others are on the GPU join the next batch.
//
// Determinism: a request that writes a table never shares a launch with another
// request on that table, requests on one table are admitted in submission order,
// and kernels run in admission order on one stream.  Every request therefore sees
// the table exactly as a one-request-at-a-time replay in submission order would
// (plain mode below), and within a request the usual batch semantics apply.
//
// Copies: a batch moves every request's arrays with ONE gather kernel (host to
// device) and ONE scatter kernel (device to host) that read and write the
// requests' pinned host memory directly, driven by a list of (destination,
// source, bytes) chunks the worker writes into coherent pinned memory.  One
// runtime copy per array would cost a dispatch each, and a batch of ~30
// requests has ~90 arrays.  Requests whose arrays are not device-mapped pinned
// memory fall back to runtime copies.
//
// Plain mode serves one request at a time with the single-table kernels and waits
// for each to finish: the baseline the batched mode is compared against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "hashwave.h"

namespace {

using clk = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(clk::now().time_since_epoch()).count(); }

struct Req {
  hwave_request r;
  bool mapped = false;  // every array is device-mapped pinned memory
  const void* g_keys = nullptr;  // device addresses of the host arrays (mapped)
  const void* g_vals = nullptr;
  void* g_vals_out = nullptr;
  uint8_t* g_status = nullptr;
  uint64_t ticket;
  double t_arrive;
  std::atomic<int> done{0};
  double t_done = 0;
};

// One piece of a copy: `bytes` from src to dst (device addresses; either may be
// mapped host memory).
struct CopyChunk {
  uint64_t dst, src, bytes;
};
constexpr uint64_t CHUNK_BYTES = 64 << 10;

struct Slot {
  CopyChunk* h_in = nullptr;   // gather list (coherent pinned host memory)
  CopyChunk* h_out = nullptr;  // scatter list
  const CopyChunk* g_in = nullptr;  // their device addresses
  const CopyChunk* g_out = nullptr;
  uint64_t chunk_cap = 0;
  void* d_keys = nullptr;
  void* d_vals = nullptr;
  void* d_out = nullptr;
  uint8_t* d_status = nullptr;
  uint64_t cap_ops = 0;
  hipEvent_t h2d = nullptr, kern = nullptr, d2h = nullptr;
  bool busy = false;
  std::vector<Req*> reqs;
};

bool writes(uint32_t op) {
  const uint32_t k = op & 0xFF;
  return k == HWAVE_OP_INSERT || k == HWAVE_OP_UPSERT || k == HWAVE_OP_ERASE;
}

// Blocks walk the chunk list (block b takes chunks b, b + grid, ...).  Loads and
// stores are system-scope (they bypass the GPU caches), so a pinned buffer the
// host has refilled is never read stale and results reach host memory; 8-byte
// words when both ends allow, bytes otherwise.  The grid is kept small
// (COPY_BLOCKS): PCIe bandwidth needs only ~100 KiB in flight, and the copies
// run beside another batch's multi-table kernel, whose persistent grid needs
// the wave slots.
constexpr unsigned COPY_BLOCKS = 128;

__global__ void __launch_bounds__(256) k_copy_chunks(const CopyChunk* __restrict__ list, uint32_t n) {
  for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
    const CopyChunk c = list[k];
    const uint64_t n8 = ((c.dst | c.src) & 7) == 0 ? c.bytes / 8 : 0;
    uint64_t* d8 = (uint64_t*)c.dst;
    const uint64_t* s8 = (const uint64_t*)c.src;
#pragma unroll 4
    for (uint64_t i = threadIdx.x; i < n8; i += 256)
      __hip_atomic_store(d8 + i, __hip_atomic_load(s8 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    uint8_t* d1 = (uint8_t*)c.dst;
    const uint8_t* s1 = (const uint8_t*)c.src;
    for (uint64_t i = n8 * 8 + threadIdx.x; i < c.bytes; i += 256)
      __hip_atomic_store(d1 + i, __hip_atomic_load(s1 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Device address of pinned host memory at p (null stays null); false if p is
// not device-mapped host memory.
bool map_host(const void* p, const void** g) {
  *g = nullptr;
  if (!p) return true;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: not an error for the caller
    return false;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return false;
  *g = a.devicePointer;
  return true;
}

// Appends [src, src + bytes) -> dst to a chunk list, CHUNK_BYTES at a time.
void add_chunks(CopyChunk* list, uint64_t* n, const void* dst, const void* src, uint64_t bytes) {
  for (uint64_t o = 0; o < bytes; o += CHUNK_BYTES)
    list[(*n)++] = CopyChunk{(uint64_t)dst + o, (uint64_t)src + o, bytes - o < CHUNK_BYTES ? bytes - o : CHUNK_BYTES};
}

// Chunks an array of `bytes` may need.
uint64_t chunks_for(uint64_t bytes) { return (bytes + CHUNK_BYTES - 1) / CHUNK_BYTES; }

}  // namespace

struct hwave_server {
  hwave_server_config cfg;
  std::vector<hwave_table*> tables;
  hwave_multi* multi = nullptr;
  uint32_t kb = 8;  // key / value bytes
  hipStream_t s_in = nullptr, s_kern = nullptr, s_out = nullptr;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> incoming;   // submitted, not yet seen by the worker
  std::deque<Req*> pending;    // seen, not yet admitted
  std::unordered_map<uint64_t, Req*> by_ticket;
  std::vector<double> latencies;
  uint64_t next_ticket = 1;
  uint64_t n_done = 0, ops_done = 0;
  // written by the worker outside `mu`, read by hwave_server_stats
  std::atomic<uint64_t> batches{0}, batch_reqs{0}, runtime_copied{0};
  double t_first = 0, t_last = 0;
  bool stop = false;
  std::atomic<int> error{0};  // first error; set by the worker, read by callers
  std::thread worker;
};

namespace {

// Records the first error and wakes callers waiting in hwave_server_drain.
int fail(hwave_server* s, int code) {
  int none = 0;
  s->error.compare_exchange_strong(none, code);
  {
    std::lock_guard<std::mutex> g(s->mu);  // a waiter checks `error` under mu
  }
  s->cv.notify_all();
  return code;
}

// Device bytes a request needs in a staging slot.
uint64_t req_ops(const Req* q) { return q->r.n; }

void retire(hwave_server* s, Slot& sl) {
  const double t = now_s();
  std::lock_guard<std::mutex> g(s->mu);
  for (Req* q : sl.reqs) {
    q->t_done = t;
    s->latencies.push_back(t - q->t_arrive);
    s->n_done++;
    s->ops_done += q->r.n;
    s->t_last = t;
    q->done.store(1, std::memory_order_release);
  }
  sl.reqs.clear();
  sl.busy = false;
  s->cv.notify_all();
}

// Batched mode: admit from `pending` into slot `sl` and launch.  Returns true if
// something was launched.
bool launch_batch(hwave_server* s, Slot& sl) {
  std::unordered_set<uint32_t> writers, readers, blocked;
  std::vector<hwave_item> items;
  uint64_t at = 0;
  uint64_t n_in = 0, n_out = 0;  // chunk-list entries the admitted requests need
  size_t scanned = 0;
  const uint32_t kb = s->kb;
  for (auto it = s->pending.begin(); it != s->pending.end() && scanned < 4096; ++scanned) {
    Req* q = *it;
    const uint32_t t = q->r.table;
    const bool w = writes(q->r.op);
    // each request starts 16 operations aligned, so its arrays in the slot are
    // 16-byte aligned and the copy kernels move whole words
    const uint64_t start = (at + 15) / 16 * 16;
    const uint64_t need_in = q->mapped ? 2 * chunks_for(q->r.n * kb) : 0;
    const uint64_t need_out = q->mapped ? chunks_for(q->r.n * kb) + chunks_for(q->r.n) : 0;
    bool ok = !blocked.count(t) && start + req_ops(q) <= sl.cap_ops && items.size() < s->cfg.max_requests &&
              n_in + need_in <= sl.chunk_cap && n_out + need_out <= sl.chunk_cap;
    if (ok && w) ok = !writers.count(t) && !readers.count(t);
    if (ok && !w) ok = !writers.count(t);
    if (!ok) {
      blocked.insert(t);  // later requests on this table keep their order
      ++it;
      continue;
    }
    (w ? writers : readers).insert(t);
    items.push_back(hwave_item{t, q->r.op, start, start + q->r.n});
    sl.reqs.push_back(q);
    at = start + q->r.n;
    n_in += need_in;
    n_out += need_out;
    it = s->pending.erase(it);
  }
  if (items.empty()) return false;
  // host -> device: each request's keys (and values for writers) into the slot,
  // one gather kernel for the mapped requests
  uint64_t n = 0;
  for (size_t i = 0; i < items.size(); i++) {
    const Req* q = sl.reqs[i];
    uint8_t* dk = (uint8_t*)sl.d_keys + items[i].begin * kb;
    uint8_t* dv = (uint8_t*)sl.d_vals + items[i].begin * kb;
    const bool wv = writes(q->r.op) && q->r.h_vals;
    if (q->mapped) {
      add_chunks(sl.h_in, &n, dk, q->g_keys, q->r.n * kb);
      if (wv) add_chunks(sl.h_in, &n, dv, q->g_vals, q->r.n * kb);
    } else {
      s->runtime_copied++;
      (void)hipMemcpyAsync(dk, q->r.h_keys, q->r.n * kb, hipMemcpyHostToDevice, s->s_in);
      if (wv) (void)hipMemcpyAsync(dv, q->r.h_vals, q->r.n * kb, hipMemcpyHostToDevice, s->s_in);
    }
  }
  if (n) {
    hipLaunchKernelGGL(k_copy_chunks, dim3(n < COPY_BLOCKS ? (unsigned)n : COPY_BLOCKS), dim3(256), 0, s->s_in,
                       sl.g_in, (uint32_t)n);
    if (hipGetLastError() != hipSuccess) fail(s, HWAVE_EDEVICE);
  }
  (void)hipEventRecord(sl.h2d, s->s_in);
  (void)hipStreamWaitEvent(s->s_kern, sl.h2d, 0);
  int rc = hwave_multi_run(s->multi, items.data(), (uint32_t)items.size(), sl.d_keys, sl.d_vals, sl.d_out,
                           sl.d_status, s->s_kern);
  if (rc) fail(s, rc);
  (void)hipEventRecord(sl.kern, s->s_kern);
  (void)hipStreamWaitEvent(s->s_out, sl.kern, 0);
  n = 0;
  for (size_t i = 0; i < items.size(); i++) {
    const Req* q = sl.reqs[i];
    const uint8_t* ds = sl.d_status + items[i].begin;
    const uint8_t* dout = (const uint8_t*)sl.d_out + items[i].begin * kb;
    const bool wo = (q->r.op & 0xFF) == HWAVE_OP_QUERY && q->r.h_vals_out;
    if (q->mapped) {
      if (q->r.h_status) add_chunks(sl.h_out, &n, q->g_status, ds, q->r.n);
      if (wo) add_chunks(sl.h_out, &n, q->g_vals_out, dout, q->r.n * kb);
    } else {
      if (q->r.h_status) (void)hipMemcpyAsync(q->r.h_status, ds, q->r.n, hipMemcpyDeviceToHost, s->s_out);
      if (wo) (void)hipMemcpyAsync(q->r.h_vals_out, dout, q->r.n * kb, hipMemcpyDeviceToHost, s->s_out);
    }
  }
  if (n) {
    hipLaunchKernelGGL(k_copy_chunks, dim3(n < COPY_BLOCKS ? (unsigned)n : COPY_BLOCKS), dim3(256), 0, s->s_out,
                       sl.g_out, (uint32_t)n);
    if (hipGetLastError() != hipSuccess) fail(s, HWAVE_EDEVICE);
  }
  (void)hipEventRecord(sl.d2h, s->s_out);
  sl.busy = true;
  s->batches++;
  s->batch_reqs += items.size();
  return true;
}

// Plain mode: the oldest pending request alone, single-table kernels, then wait.
bool launch_plain(hwave_server* s, Slot& sl) {
  if (s->pending.empty()) return false;
  Req* q = s->pending.front();
  s->pending.pop_front();
  const uint32_t kb = s->kb;
  hwave_table* t = s->tables[q->r.table];
  (void)hipMemcpyAsync(sl.d_keys, q->r.h_keys, q->r.n * kb, hipMemcpyHostToDevice, s->s_kern);
  const uint32_t op = q->r.op & 0xFF, comb = (q->r.op >> 8) & 0xFF;
  if (writes(op) && q->r.h_vals)
    (void)hipMemcpyAsync(sl.d_vals, q->r.h_vals, q->r.n * kb, hipMemcpyHostToDevice, s->s_kern);
  int rc = HWAVE_OK;
  if (op == HWAVE_OP_QUERY)
    rc = hwave_query(t, sl.d_keys, q->r.n, sl.d_out, sl.d_status, s->s_kern);
  else if (op == HWAVE_OP_INSERT)
    rc = hwave_insert(t, sl.d_keys, sl.d_vals, q->r.n, sl.d_status, s->s_kern);
  else if (op == HWAVE_OP_UPSERT)
    rc = hwave_upsert(t, sl.d_keys, sl.d_vals, q->r.n, (hwave_combine)comb, sl.d_status, s->s_kern);
  else
    rc = hwave_erase(t, sl.d_keys, q->r.n, sl.d_status, s->s_kern);
  if (rc) fail(s, rc);
  if (q->r.h_status)
    (void)hipMemcpyAsync(q->r.h_status, sl.d_status, q->r.n, hipMemcpyDeviceToHost, s->s_kern);
  if (op == HWAVE_OP_QUERY && q->r.h_vals_out)
    (void)hipMemcpyAsync(q->r.h_vals_out, sl.d_out, q->r.n * kb, hipMemcpyDeviceToHost, s->s_kern);
  (void)hipEventRecord(sl.d2h, s->s_kern);
  (void)hipEventSynchronize(sl.d2h);
  sl.reqs.push_back(q);
  sl.busy = true;
  s->batches++;
  s->batch_reqs++;
  return true;
}

void worker_main(hwave_server* s) {
  (void)hipSetDevice(s->cfg.device);
  const bool plain = s->cfg.mode == HWAVE_SERVE_PLAIN;
  while (true) {
    {
      std::unique_lock<std::mutex> g(s->mu);
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
      bool inflight = false;
      for (auto& sl : s->slots) inflight |= sl.busy;
      if (s->stop && s->pending.empty() && !inflight) break;
      if (s->pending.empty() && !inflight) {
        s->cv.wait_for(g, std::chrono::microseconds(200));
        continue;
      }
    }
    bool progressed = false;
    for (auto& sl : s->slots) {  // retire finished batches
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.d2h);
      if (e == hipErrorNotReady) continue;
      // a device error retires the batch too (its requests report the error),
      // so drain and destroy never wait on an event that cannot complete
      if (e != hipSuccess) fail(s, HWAVE_EDEVICE);
      retire(s, sl);
      progressed = true;
    }
    for (auto& sl : s->slots) {  // fill free slots
      if (sl.busy) continue;
      bool launched;
      {
        std::lock_guard<std::mutex> g(s->mu);
        while (!s->incoming.empty()) {
          s->pending.push_back(s->incoming.front());
          s->incoming.pop_front();
        }
      }
      launched = plain ? launch_plain(s, sl) : launch_batch(s, sl);
      progressed |= launched;
      if (plain && launched) retire(s, sl);
      if (!launched) break;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(10));
  }
}

}  // namespace

extern "C" {

int hwave_server_create(hwave_server** out, hwave_table* const* tables, uint32_t n_tables,
                        const hwave_server_config* cfg) {
  if (!out || !tables || !n_tables || !cfg || cfg->slot_ops == 0 || cfg->slots == 0) return HWAVE_EINVAL;
  *out = nullptr;
  hwave_server* s = new hwave_server;
  s->cfg = *cfg;
  if (s->cfg.max_requests == 0) s->cfg.max_requests = 1u << 16;
  s->tables.assign(tables, tables + n_tables);
  hwave_raw_view rv;
  int rc = hwave_raw(tables[0], &rv);
  if (rc) { delete s; return rc; }
  s->kb = rv.kv_bits / 8;
  (void)hipSetDevice(cfg->device);
  hipError_t e = hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_kern, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking);
  if (e != hipSuccess) { delete s; return HWAVE_EDEVICE; }
  if (cfg->mode != HWAVE_SERVE_PLAIN) {
    rc = hwave_multi_create(&s->multi, tables, n_tables, s->s_kern);
    if (rc) { hwave_server_destroy(s); return rc; }
  }
  const uint32_t nslots = cfg->mode == HWAVE_SERVE_PLAIN ? 1 : cfg->slots;
  s->slots.resize(nslots);
  for (auto& sl : s->slots) {
    sl.cap_ops = cfg->slot_ops;
    // two arrays per direction, each split into CHUNK_BYTES pieces, plus one
    // partial piece per array and request
    sl.chunk_cap = 2 * (chunks_for(sl.cap_ops * s->kb) + s->cfg.max_requests) + 16;
    const size_t lb = sl.chunk_cap * sizeof(CopyChunk);
    e = hipHostMalloc((void**)&sl.h_in, lb, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_out, lb, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&sl.g_in, sl.h_in, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&sl.g_out, sl.h_out, 0);
    if (e == hipSuccess) e = hipMalloc(&sl.d_keys, sl.cap_ops * s->kb);
    if (e == hipSuccess) e = hipMalloc(&sl.d_vals, sl.cap_ops * s->kb);
    if (e == hipSuccess) e = hipMalloc(&sl.d_out, sl.cap_ops * s->kb);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_status, sl.cap_ops);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.h2d, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.kern, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.d2h, hipEventDisableTiming);
    if (e != hipSuccess) { hwave_server_destroy(s); return HWAVE_ENOMEM; }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return HWAVE_OK;
}

int hwave_server_submit(hwave_server* s, const hwave_request* r, double arrival_s, uint64_t* ticket) {
  if (!s || !r || r->table >= s->tables.size() || r->n == 0 || !r->h_keys) return HWAVE_EINVAL;
  if ((r->op & 0xFF) > HWAVE_OP_ERASE || r->n > s->cfg.slot_ops) return HWAVE_EINVAL;
  if (writes(r->op) && (r->op & 0xFF) != HWAVE_OP_ERASE && !r->h_vals) return HWAVE_EINVAL;
  Req* q = new Req;
  q->r = *r;
  const void* gv_out = nullptr;
  const void* g_status = nullptr;
  q->mapped = map_host(r->h_keys, &q->g_keys) && map_host(r->h_vals, &q->g_vals) &&
              map_host(r->h_vals_out, &gv_out) && map_host(r->h_status, &g_status);
  q->g_vals_out = (void*)gv_out;
  q->g_status = (uint8_t*)g_status;
  q->t_arrive = arrival_s > 0 ? arrival_s : now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    q->ticket = s->next_ticket++;
    s->by_ticket[q->ticket] = q;
    if (s->t_first == 0) s->t_first = q->t_arrive;
    s->incoming.push_back(q);
  }
  s->cv.notify_all();
  if (ticket) *ticket = q->ticket;
  return HWAVE_OK;
}

int hwave_server_poll(hwave_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return HWAVE_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return HWAVE_EINVAL;
  *done = it->second->done.load(std::memory_order_acquire);
  return s->error;
}

int hwave_server_drain(hwave_server* s) {
  if (!s) return HWAVE_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  s->cv.wait(g, [&] {
    uint64_t submitted = s->next_ticket - 1;
    return s->n_done == submitted || s->error;
  });
  return s->error;
}

double hwave_now(void) { return now_s(); }

int hwave_server_replay(hwave_server* s, const hwave_request* reqs, const double* offsets_s, uint64_t n,
                        double* t0_out) {
  if (!s || (n && (!reqs || !offsets_s))) return HWAVE_EINVAL;
  const double t0 = now_s() + 1e-3;
  if (t0_out) *t0_out = t0;
  for (uint64_t i = 0; i < n; i++) {
    const double due = t0 + offsets_s[i];
    double t;
    while ((t = now_s()) < due) {
      if (due - t > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    int rc = hwave_server_submit(s, reqs + i, due, nullptr);
    if (rc) return rc;
  }
  return HWAVE_OK;
}

int hwave_server_stats(hwave_server* s, hwave_serve_stats* out) {
  if (!s || !out) return HWAVE_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->requests = s->n_done;
  out->ops = s->ops_done;
  const uint64_t nb = s->batches.load(), nr = s->batch_reqs.load();
  out->batches = nb;
  out->mean_requests_per_batch = nb ? (double)nr / (double)nb : 0.0;
  out->wall_s = s->t_last > s->t_first ? s->t_last - s->t_first : 0.0;
  out->runtime_copied = s->runtime_copied.load();
  if (!s->latencies.empty()) {
    std::vector<double> v = s->latencies;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
    out->p50_ms = pct(0.50) * 1e3;
    out->p99_ms = pct(0.99) * 1e3;
    out->max_ms = v.back() * 1e3;
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / (double)v.size() * 1e3;
  }
  return s->error;
}

int hwave_server_destroy(hwave_server* s) {
  if (!s) return HWAVE_EINVAL;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
  }
  (void)hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    if (sl.h_in) (void)hipHostFree(sl.h_in);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.d_keys) (void)hipFree(sl.d_keys);
    if (sl.d_vals) (void)hipFree(sl.d_vals);
    if (sl.d_out) (void)hipFree(sl.d_out);
    if (sl.d_status) (void)hipFree(sl.d_status);
    if (sl.h2d) (void)hipEventDestroy(sl.h2d);
    if (sl.kern) (void)hipEventDestroy(sl.kern);
    if (sl.d2h) (void)hipEventDestroy(sl.d2h);
  }
  if (s->multi) hwave_multi_destroy(s->multi);
  if (s->s_in) (void)hipStreamDestroy(s->s_in);
  if (s->s_kern) (void)hipStreamDestroy(s->s_kern);
  if (s->s_out) (void)hipStreamDestroy(s->s_out);
  for (auto& kv : s->by_ticket) delete kv.second;
  delete s;
  return HWAVE_OK;
}

}  // extern "C"

/*
 * hashwave.h -- C-ABI of HashWave, concurrent open-addressing hash tables for
 * AMD MI355X (gfx950).
 *
 * The operations follow the paper's hash-table API (Section 5.1, "Hash table
 * API"): Upsert(key, value, callback), Query(key, &value) and Erase(key), here
 * in bulk form over device arrays, enqueued on a HIP stream.  The callback of
 * Upsert is offered as a fixed set of combine operations (hwave_combine),
 * because a C-ABI cannot carry a device function pointer.  Insert is Upsert with
 * the "insert if unique" callback (Section 5.1).
 *
 * Designs (Section 2.2 and Section 5): bucketed double hashing,
 * power-of-two-choice hashing and iceberg hashing, each with an optional 16-bit fingerprint
 * ("metadata", Section 4.3) array.  Every write operation takes the lock of the
 * key's primary bucket (Section 4.1); queries take no lock (Section 4.2).
 *
 * Conventions for every call below:
 *  - Pointers named d_* are device pointers (hipMalloc or torch CUDA tensors) on
 *    the table's device; the caller owns them and keeps them alive until the
 *    enqueued work completes.  Element width of keys and values is the table's
 *    kv_bits (uint64_t or uint32_t elements); status/found arrays are uint8_t.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous; nothing blocks except hwave_destroy and the
 *    *_sync helpers.
 *  - Return value: HWAVE_OK (0) once the work is enqueued, or a negative
 *    HWAVE_E* code; on an error nothing was enqueued.  n == 0 is a no-op.
 *  - The table is concurrent: calls on different streams may overlap and the
 *    result equals some serialisation of all their operations.  Calls within
 *    one batch are concurrent with each other (any serialisation).
 */
#ifndef HASHWAVE_H
#define HASHWAVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hwave_table hwave_table;

/* Table designs (Section 2.2, configurations of Section 5).  The lock a key's
 * writers take is that of its primary bucket, for iceberg its front-yard
 * bucket (hwave_primary_bucket reports it). */
typedef enum {
  HWAVE_DOUBLE = 0,   /* bucketed double hashing; default bucket 8, tile 8     */
  HWAVE_DOUBLE_M = 1, /* double hashing with 16-bit tags; bucket 32, tile 4    */
  HWAVE_P2 = 2,       /* power-of-two-choice; bucket 32, tile 8                */
  HWAVE_P2_M = 3,     /* power-of-two-choice with 16-bit tags; bucket 32, tile 4 */
  HWAVE_ICEBERG = 4,  /* iceberg: 83% single-hash front yard, 17% power-of-two-
                         choice backyard (Section 2.2, Section 5); bucket 32,
                         tile 8; at least two buckets                          */
  HWAVE_ICEBERG_M = 5, /* iceberg with 16-bit tags; bucket 32, tile 4          */
  HWAVE_CHAINING = 6  /* chaining: per bucket a chain of 128-byte nodes of 7
                         pairs and a link (Section 5); ceil(capacity/7)
                         buckets plus an overflow pool of twice as many nodes
                         (hwave_capacity counts both); 64-bit keys, tile 8;
                         insert/upsert return FULL once the pool is spent     */,
  HWAVE_CUCKOO = 7    /* three-way bucketed cuckoo hashing (Section 5): bucket
                         8, tile 4, 64-bit keys; keys move between their three
                         buckets, so every operation, queries included, locks
                         all three (the phased variant's queries excepted);
                         FULL when no room can be made                        */
} hwave_design;

/* Upsert callbacks (Section 5.1): SUM accumulates with wrap-around modulo
 * 2^kv_bits, KEEP is "insert if unique", REPLACE overwrites, MIN/MAX keep the
 * unsigned minimum/maximum. */
typedef enum { HWAVE_SUM = 0, HWAVE_KEEP = 1, HWAVE_REPLACE = 2, HWAVE_MIN = 3, HWAVE_MAX = 4 } hwave_combine;

/* Opcodes of hwave_mixed. */
typedef enum { HWAVE_OP_QUERY = 0, HWAVE_OP_INSERT = 1, HWAVE_OP_UPSERT = 2, HWAVE_OP_ERASE = 3 } hwave_op;

/* Per-operation status codes written to d_status / d_found. */
enum {
  HWAVE_ST_MISS = 0,     /* query/erase: key absent                               */
  HWAVE_ST_DONE = 1,     /* insert/upsert: inserted; query: found; erase: erased   */
  HWAVE_ST_EXISTED = 2,  /* insert/upsert: key present, combine applied           */
  HWAVE_ST_FULL = 3,     /* insert/upsert: no free slot among the key's buckets   */
  HWAVE_ST_INVALID = 4,  /* key equals a reserved pattern; the op had no effect   */
  HWAVE_ST_TIMEOUT = 5   /* insert/upsert/erase: waited longer than the table's
                            lock_timeout_us for the key's bucket lock, or saw
                            that another operation of the table had; the op
                            had no effect.  A failure report, not a result: the
                            abandoned ticket blocks its lock queue, so later
                            writers that find a bucket of that queue busy time
                            out as well, until hwave_clear empties the table  */
};

/* Return codes. */
enum {
  HWAVE_OK = 0,
  HWAVE_EINVAL = -1,      /* bad argument (null pointer, size, unsupported value)  */
  HWAVE_ENOMEM = -2,      /* device allocation failed or buffer too small          */
  HWAVE_EDEVICE = -3,     /* a HIP call failed; see hwave_last_hip_error()         */
  HWAVE_EUNSUPPORTED = -4, /* no kernel instance for this design/width/bucket/tile */
  HWAVE_EIO = -5,          /* a file could not be opened, read or written, or is malformed */
  HWAVE_ETOOBIG = -6       /* batch larger than hwave_mixed_noalloc's fixed workspace  */
};

/* Flags of hwave_config.flags. */
enum {
  HWAVE_F_NO_SHORTCUT = 1, /* power-of-two-choice: never take the 75% shortcut    */
  HWAVE_F_NO_ERASE = 2     /* the table never erases: hwave_erase returns
                              HWAVE_EINVAL, erase ops of hwave_mixed and erase
                              items of hwave_multi_run get HWAVE_ST_INVALID,
                              and upserts of present keys are
                              combined in place without taking the bucket lock
                              (stable slots are never reused; Section 2.1)    */,
  HWAVE_F_BSP = 4          /* phased (bulk-synchronous) variant, to measure what
                              concurrency costs (Section 6.4): writes take no
                              lock (chaining and cuckoo keep their write locks),
                              queries take none and read with plain cacheable
                              loads.  Results are defined only for phased use: the
                              writes of one call are to distinct keys, and no
                              call overlaps another that writes the keys it
                              touches.  64-bit tables at the default bucket and
                              tile of each design; not accepted by
                              hwave_multi_create                               */,
  HWAVE_F_AGGREGATE = 8    /* merge duplicate keys of insert and upsert calls
                              (SUM, KEEP, MIN, MAX; not REPLACE) within windows
                              of 128 operations before they reach the table:
                              one table operation per distinct key, the first
                              of a window's duplicates reports the table's
                              status and the others EXISTED (or its FULL).
                              For skewed batches, whose hot keys would
                              otherwise serialise on one lock or value word.
                              With HWAVE_F_NO_ERASE too (not CUCKOO, not BSP)
                              the table also holds 64 KiB of hot-key
                              accumulators: a present key met more than once
                              in a window is combined into one of 32 striped
                              accumulators instead of its value word, and a
                              second kernel on the same stream folds them
                              into the table before the call's work is
                              complete.  Calls that write such a table must
                              then run one at a time (stream-ordered); queries
                              may overlap them as with any write            */,
  HWAVE_F_MERGE_MIXED = 16 /* hwave_mixed merges the upserts of each call by key
                              before they reach the table (SUM, KEEP, MIN,
                              MAX; not REPLACE, and not inserts): every key's
                              upserts become ONE table upsert of their combined
                              value, run by the one with the smallest index,
                              which reports the table's status; the others
                              report EXISTED (or its FULL / INVALID / TIMEOUT).
                              That is the serialisation "each key's upserts
                              back to back" (Section 4.1 serialises a key's
                              writers on one lock anyway), and it spares a
                              skewed batch's hot keys thousands of locked
                              operations in one lock queue.  Costs two more
                              launches per 2^20 operations and 52 MiB of
                              workspace in the table; calls that write the
                              table must then run one at a time
                              (stream-ordered)                              */
};

/* Table configuration.  Zero fields take the design's defaults (the
 * configurations of Section 5).  Supported (kv_bits, design, bucket/tile);
 * others return HWAVE_EUNSUPPORTED:
 *   64-bit keys/values:
 *     DOUBLE    b8/t4 b8/t8 b16/t4 b16/t8 b16/t16 b32/t8 b32/t16 b32/t32
 *     DOUBLE_M  b16/t4 b32/t2 b32/t4 b32/t8 b32/t16 b64/t8
 *     P2        b16/t8 b32/t4 b32/t8 b32/t16 b32/t32
 *     P2_M      b16/t4 b32/t2 b32/t4 b32/t8 b32/t16 b64/t8
 *     ICEBERG   b32/t4 b32/t8 b32/t16;  ICEBERG_M b32/t2 b32/t4 b32/t8 b64/t8
 *     CHAINING  7 pairs per node, tile 8 (the defaults)
 *     CUCKOO    b8/t4 b8/t8 b16/t8
 *     HWAVE_F_BSP: each design's default configuration only.
 *   32-bit keys/values:
 *     DOUBLE    b8/t4 b16/t4 b16/t8 b32/t8 b32/t16 b64/t32 b128/t64
 *     DOUBLE_M  b16/t4 b32/t4 b32/t8 b32/t16 b64/t8
 *     P2        b16/t4 b16/t8 b32/t4 b32/t8 b32/t16 b64/t32
 *     P2_M      b16/t4 b32/t4 b32/t8 b32/t16 b32/t32 b64/t8
 *     ICEBERG, ICEBERG_M  b32/t4 b32/t8  (no chaining or cuckoo)
 * Reserved key patterns (rejected with HWAVE_ST_INVALID): 64-bit keys
 * 0xFFFFFFFFFFFFFFFF (empty), ...FE (tombstone), ...FD (reservation marker);
 * 32-bit keys 0xFFFFFFFF and 0xFFFFFFFE. */
typedef struct {
  uint32_t kv_bits;      /* 64 or 32                                          */
  uint32_t bucket_slots; /* slots per bucket                                  */
  uint32_t tile;         /* lanes cooperating on one operation                */
  uint32_t probe_cap;    /* double hashing: max buckets visited (0 = all)      */
  uint32_t flags;        /* HWAVE_F_*                                         */
  uint32_t lock_timeout_us; /* longest wait of one operation for its bucket's
                           lock, in microseconds (0 = 10 s; at most 40 s, else
                           HWAVE_EINVAL).  Section 4.1 serialises a key's
                           writers on its primary bucket's lock; writers that
                           find it held wait in a FIFO ticket queue, so a wait
                           is bounded by the operations queued ahead times one
                           critical section; an operation still waiting at the
                           limit gives up with HWAVE_ST_TIMEOUT (see there)    */
} hwave_config;

/* Fills *out with the design's defaults: the bucket size and tile width of the
 * paper's configuration of that design (Section 5).  Returns HWAVE_OK or
 * HWAVE_EINVAL. */
int hwave_config_default(hwave_design design, hwave_config* out);

/* Device bytes a table needs (slots + tags + lock array and queues + control words) for a
 * capacity rounded up to bucket_slots * 2^k slots: the space accounting of
 * Section 6.1 plus the locks (Section 5.1).  Host-only arithmetic. */
int hwave_table_bytes(uint64_t capacity_slots, hwave_design design, const hwave_config* cfg,
                      uint64_t* bytes);

/* Creates an empty table of at least capacity_slots slots (rounded up to
 * bucket_slots * 2^k; hwave_capacity() reports the result).  Memory comes from
 * hipMalloc and is owned by the table.  The table is initialised on `stream`.
 * Capacity is fixed for the table's life (Section 3.2: no resizing). */
int hwave_create(hwave_table** out, uint64_t capacity_slots, hwave_design design,
                 const hwave_config* cfg, void* stream);

/* Same as hwave_create (fixed capacity, Section 3.2) but in caller-owned device
 * memory (e.g. a torch tensor) of buffer_bytes >= hwave_table_bytes(); d_buffer
 * must be 256-byte aligned and outlive the table; HWAVE_EINVAL otherwise. */
int hwave_create_in(hwave_table** out, void* d_buffer, uint64_t buffer_bytes,
                    uint64_t capacity_slots, hwave_design design, const hwave_config* cfg,
                    void* stream);

/* Synchronises the device, then frees the table (and its memory if owned).  Not
 * a paper operation: table lifetime. */
int hwave_destroy(hwave_table* t);

/* Empties the table (every slot empty, tags empty, locks and lock queues free,
 * the lock failure flag of HWAVE_ST_TIMEOUT cleared) on `stream`: the empty
 * table every benchmark run of Section 6 starts from. */
int hwave_clear(hwave_table* t, void* stream);

/* Insert = Upsert with KEEP (Section 5.1).  d_vals may not be NULL.  d_status
 * (nullable): DONE (inserted), EXISTED (left unchanged), FULL or INVALID. */
int hwave_insert(hwave_table* t, const void* d_keys, const void* d_vals, uint64_t n,
                 uint8_t* d_status, void* stream);

/* Upsert (Section 5.1): absent key -> inserted with its value (DONE); present
 * key -> value = combine(stored, value) atomically (EXISTED). */
int hwave_upsert(hwave_table* t, const void* d_keys, const void* d_vals, uint64_t n,
                 hwave_combine combine, uint8_t* d_status, void* stream);

/* Query (Section 5.1), lock-free (Section 4.2).  d_vals_out[i] = stored value
 * or 0 when absent; d_found[i] = DONE / MISS / INVALID.  Either output may be
 * NULL. */
int hwave_query(hwave_table* t, const void* d_keys, uint64_t n, void* d_vals_out,
                uint8_t* d_found, void* stream);

/* Erase (Section 5.1): d_found[i] = DONE (erased) / MISS (absent, table
 * unchanged) / INVALID.  d_found may be NULL.  HWAVE_EINVAL on a table created
 * with HWAVE_F_NO_ERASE. */
int hwave_erase(hwave_table* t, const void* d_keys, uint64_t n, uint8_t* d_found, void* stream);

/* One launch running a different operation per element (the paper runs all
 * operations of an aging iteration concurrently in one kernel, Section 6.5).
 * d_ops[i] is a hwave_op; upserts use `combine`; d_vals is read for inserts and
 * upserts (nullable when there are none); d_vals_out (nullable) receives query
 * results (0 for other ops); d_status (nullable) the per-op status.  The
 * operations of one call are concurrent: the kernel runs each group of 64 in
 * order of kind (queries, inserts/upserts, erases), not in array order. */
int hwave_mixed(hwave_table* t, const uint8_t* d_ops, const void* d_keys, const void* d_vals,
                uint64_t n, hwave_combine combine, void* d_vals_out, uint8_t* d_status,
                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): hwave_mixed with the
 * upserts merged by key as on a HWAVE_F_MERGE_MIXED table, whatever the table's
 * flags, using a workspace in a fixed device array instead of one the library
 * allocates.  Calls no allocating routine.  Limit: n <= 262,144 (2^18)
 * operations, else HWAVE_ETOOBIG and nothing is enqueued.  The array (14 MiB:
 * 2^19 merge entries of 24 bytes and a 4-byte word per operation) is held by
 * each device the library runs on until the process ends; the first call on a
 * device looks up its address.  Every call on a device shares that array and
 * clears it (with a kernel) before use: calls on one device that overlap in
 * time (other streams, other host threads) race and must not be issued.  The
 * table's device must be current.  Results equal those of hwave_mixed on a
 * table with HWAVE_F_MERGE_MIXED. */
int hwave_mixed_noalloc(hwave_table* t, const uint8_t* d_ops, const void* d_keys, const void* d_vals,
                        uint64_t n, hwave_combine combine, void* d_vals_out, uint8_t* d_status,
                        void* stream);

/* Writes the number of live keys to *d_count (one uint64_t on the device).  Not
 * a paper operation: the size check of the benchmarks' verification (live keys =
 * successful inserts - successful erases). */
int hwave_size(hwave_table* t, uint64_t* d_count, void* stream);

/* Copies every live (key, value) pair to d_keys/d_vals (capacity elements
 * each, in slot order) and their number to *d_count.  Meant for a quiescent
 * table (checkpoint dump, tests).  Not a paper operation: the dump that the
 * verification compares with the oracle's map. */
int hwave_export(hwave_table* t, void* d_keys, void* d_vals, uint64_t* d_count, void* stream);

/* Number of buckets (host call), and the primary bucket of each key (device
 * call): the two hooks of the paper's adversarial benchmark (Section 4.1). */
uint64_t hwave_num_buckets(const hwave_table* t);
int hwave_primary_bucket(hwave_table* t, const void* d_keys, uint64_t n, uint64_t* d_out,
                         void* stream);

/* The buckets each key may occupy, three entries per key in d_out (3n
 * uint64_t; unused entries all-ones): power-of-two-choice -- primary and
 * alternate bucket (Section 2.2); iceberg -- front-yard bucket and the two
 * backyard choices; cuckoo -- its three buckets; double hashing -- the primary
 * bucket and the probe step (the sequence is primary + i * step modulo the
 * bucket count); chaining -- the bucket.  With a raw image (hwave_raw) this
 * lets a caller check that a FULL status was legal: every candidate bucket
 * full (Section 2.2: a power-of-two-choice insert fails only when both of
 * its buckets are full). */
int hwave_candidate_buckets(hwave_table* t, const void* d_keys, uint64_t n, uint64_t* d_out,
                            void* stream);

/* Slot capacity after rounding (bucket_slots * 2^k, Section 3.2). */
uint64_t hwave_capacity(const hwave_table* t);

/* Device pointers and geometry of a table, for tests that inspect its raw image
 * against the layouts of Section 2.2 (the oracle's layout checker). */
typedef struct {
  void* slots;          /* slots of (key, value), bucket-major; chaining: nodes of
                           8 16-byte units, unit 7 the link (empty key word,
                           next node index or all-ones in the value word)     */
  uint16_t* tags;       /* capacity 16-bit tags, or NULL without tags             */
  uint32_t* locks;      /* bucket b's lock: byte b * lock_stride of this array
                           (Section 5.1), nonzero while held                   */
  uint64_t n_lock_words; /* 32-bit words of the lock array:
                           ceil(buckets * lock_stride / 4)                     */
  uint64_t* lock_queues; /* ticket queues of contended acquires: per word, next
                           ticket (high 32 bits) and ticket being served (low
                           32 bits); idle when equal.  Bucket b queues on word
                           b mod n_lock_queues                                 */
  uint64_t n_lock_queues; /* a power of two                                     */
  uint64_t num_buckets;
  uint32_t bucket_slots, tile, kv_bits, design;
  uint64_t slot_bytes;  /* bytes of the slot region (chaining: every node)     */
  uint32_t lock_stride; /* bytes per bucket lock: clamp(2^23 / buckets, 1, 8),
                           a power of two                                      */
} hwave_raw_view;
int hwave_raw(const hwave_table* t, hwave_raw_view* out);

/* ------------------------------------------------------------------------
 * Batched form: one persistent launch over many tables.  Not a paper operation:
 * the paper runs one table per launch; each item here is one of its bulk
 * operations (Section 5.1) on one table.
 *
 * A hwave_multi groups tables of one key width (any designs and sizes whose
 * configuration is in the multi-table menu: hwave_multi_supported).  Each call
 * takes a list of work items over shared device arrays; item i applies its
 * operation to ops [begin, end) of the arrays on table `table`.  All items run
 * in ONE kernel launch whose waves pull chunks of items from per-XCD queues.
 * Items on different tables are independent; items on the same table are
 * concurrent (any serialisation), like one batch.
 */
typedef struct hwave_multi hwave_multi;

typedef struct {
  uint32_t table; /* index into the tables given to hwave_multi_create          */
  uint32_t op;    /* hwave_op | (hwave_combine << 8) for HWAVE_OP_UPSERT         */
  uint64_t begin; /* first op of this item in the shared arrays                  */
  uint64_t end;   /* one past the last                                            */
} hwave_item;

/* 1 if a table with this (kv_bits, design, bucket, tile) can join a hwave_multi.
 * Menus: 32-bit keys -- DOUBLE b16 t4/t8, b32 t16, b64 t32, b128 t64; DOUBLE_M
 * b32 t4; P2 b32 t8; P2_M b16 t4, b32 t4/t8.  64-bit keys -- DOUBLE b8 t8, b16
 * t8; DOUBLE_M b32 t4/t8; P2 b32 t8; P2_M b32 t4/t8, b64 t8; and, on an
 * extended kernel that a group runs on when it holds one of them (more
 * registers, lower occupancy), ICEBERG b32 t8, ICEBERG_M b32 t4, CHAINING
 * (default), CUCKOO b8 t4. */
int hwave_multi_supported(uint32_t kv_bits, hwave_design design, uint32_t bucket_slots, uint32_t tile);

/* Creates a group over n_tables existing tables (same device and key width).
 * The tables must outlive the group.  Uploads their descriptors on `stream`.
 * When every table has the same configuration, the group runs on that
 * configuration's own kernel (fewer registers, no switch over the menu); 64-bit
 * groups with a HWAVE_F_AGGREGATE table take its variant with the merging path. */
int hwave_multi_create(hwave_multi** out, hwave_table* const* tables, uint32_t n_tables, void* stream);
int hwave_multi_destroy(hwave_multi* m);

/* Which kernel a group runs on (no paper operation: for callers that tune or
 * profile the batched form).  *kernel: HWAVE_MULTI_MENU (the key width's base
 * menu), HWAVE_MULTI_EXTENDED (64-bit extended menu) or HWAVE_MULTI_SOLO (one
 * configuration); *waves: its occupancy target, waves per SIMD, which sizes the
 * persistent grid.  Either pointer may be null.  HWAVE_EINVAL if m is null. */
enum { HWAVE_MULTI_MENU = 0, HWAVE_MULTI_EXTENDED = 1, HWAVE_MULTI_SOLO = 2 };
int hwave_multi_kernel(const hwave_multi* m, uint32_t* kernel, uint32_t* waves);

/* Runs n_items host-described items in one launch.  d_vals is read by insert
 * and upsert items (nullable if there are none); d_vals_out (nullable) receives
 * query values; d_status (nullable) one status byte per op.  Blocks only until
 * the host item list has been copied out of the group's staging buffer from
 * the previous call. */
int hwave_multi_run(hwave_multi* m, const hwave_item* h_items, uint32_t n_items, const void* d_keys,
                    const void* d_vals, void* d_vals_out, uint8_t* d_status, void* stream);

/* The batched group-by upsert over a table list, offsets on the device: tables[i]
 * receives ops [d_offsets[i], d_offsets[i+1]) of the shared arrays as one upsert
 * with `combine` (the accumulating upsert of Section 5.1; d_offsets: n_tables + 1
 * device words, d_offsets[0] = 0, non-decreasing, else HWAVE_EINVAL), all in one
 * persistent launch.  The library keeps a group (hwave_multi) per
 * distinct table list, made on the first call and dropped when one of its
 * tables is destroyed.  Blocks until the offsets have been copied to the host
 * (the stream's earlier work has completed), then enqueues like
 * hwave_multi_upsert. */
int hwave_multi_upsert_tables(hwave_table* const* tables, uint32_t n_tables, const uint64_t* d_offsets,
                              const void* d_keys, const void* d_vals, hwave_combine combine, uint8_t* d_status,
                              void* stream);

/* Empties every table of the group in one launch on `stream`. */
int hwave_multi_clear(hwave_multi* m, void* stream);

/* Convenience: table i receives ops [h_offsets[i], h_offsets[i+1]) as one upsert
 * with `combine` (h_offsets has n_tables + 1 entries). */
int hwave_multi_upsert(hwave_multi* m, const uint64_t* h_offsets, const void* d_keys, const void* d_vals,
                       hwave_combine combine, uint8_t* d_status, void* stream);

/* ------------------------------------------------------------------------
 * Autotuner (the paper picks bucket and tile size per design by exhaustive
 * search, Section 5): times every multi-table menu configuration whose design
 * bit is set in design_mask (1 << hwave_design) for tables of `capacity` slots,
 * on a synthetic group-by SUM-upsert batch that fills them to `load`, spread
 * over enough tables of that class to fill the GPU and run through the
 * persistent multi-table kernel.  `flags` are the tables' HWAVE_F_* flags.
 * Writes up to results_cap timings to `results` (their count to *n_results) and
 * the fastest to *best.  A configuration that cannot hold the load -- any
 * operation of its batch ended FULL -- is reported with its FULL count and is
 * never chosen.  Allocates and frees its own device memory; blocks.
 */
typedef struct {
  uint32_t design;       /* hwave_design                        */
  uint32_t bucket_slots;
  uint32_t tile;
  uint32_t kv_bits;
  double gops;           /* measured upserts per ns (G ops/s)   */
  uint64_t full_ops;     /* operations that ended FULL (0 = holds the load) */
  double load;           /* the load factor it was timed at      */
  uint32_t flags;        /* the tables' HWAVE_F_* flags it was timed with */
  uint32_t reserved;     /* zero                                 */
} hwave_tune_result;

int hwave_autotune(uint32_t kv_bits, uint64_t capacity, uint32_t design_mask, double load, uint32_t reps,
                   uint32_t flags, hwave_tune_result* results, uint32_t results_cap, uint32_t* n_results,
                   hwave_tune_result* best, void* stream);

/* Persisted tuning, one capacity class per entry: class i is log2_capacity[i]
 * with its chosen configuration best[i], which also records the load factor
 * and table flags it was tuned for (one file may hold classes tuned at several
 * loads or flags).  The file is text: a first line "hwave-tune 2", then one
 * line per class, "<log2_capacity> <load> <flags> <kv_bits> <design>
 * <bucket_slots> <tile> <gops> <full_ops>".  Save overwrites `path`.  Load
 * reads at most `cap` classes into the caller's arrays and their count into
 * *n; it rejects (HWAVE_EIO) a file with another first line, a line it cannot
 * parse, more than `cap` classes, or a load outside (0, 1], unknown flags, or a
 * design, key width, bucket or tile that is out of range.  Host-only; no device
 * work. */
int hwave_tune_save(const char* path, const uint32_t* log2_capacity, const hwave_tune_result* best, uint32_t n);
int hwave_tune_load(const char* path, uint32_t* log2_capacity, hwave_tune_result* best, uint32_t cap,
                    uint32_t* n);

/* ------------------------------------------------------------------------
 * Served form: a request loop over resident tables (continuous batching).  Not
 * a paper operation: each request is one of its bulk operations (Section 5.1).
 *
 * A request is one operation kind on n keys of one table, with its arrays in
 * host memory; they must stay valid until the request completes.  In batched
 * mode, arrays in device-mapped pinned memory (hipHostMalloc, torch
 * pin_memory) are read and written directly by one gather and one scatter
 * kernel per batch; a request with any other array is copied with runtime
 * copies instead (slower, same results).  A worker thread
 * admits pending requests into the next batch while their data fits a device
 * staging slot of `slot_ops` operations (admission by memory), packs them into
 * one persistent multi-table launch, and keeps up to `slots` batches in flight
 * with copies and kernels overlapped on separate streams.  A request that
 * writes a table never shares a launch with another request on that table and
 * requests on a table are admitted in submission order, so each request's
 * results equal those of a one-at-a-time replay in submission order.
 * HWAVE_SERVE_PLAIN serves one request at a time with the single-table kernels,
 * waiting for each: the baseline.
 */
typedef struct hwave_server hwave_server;

enum { HWAVE_SERVE_BATCHED = 0, HWAVE_SERVE_PLAIN = 1 };

typedef struct {
  uint32_t table;      /* index into the server's tables                      */
  uint32_t op;         /* hwave_op | (hwave_combine << 8)                      */
  uint64_t n;          /* operations (1 .. slot_ops)                           */
  const void* h_keys;  /* n keys                                               */
  const void* h_vals;  /* n values (insert / upsert)                           */
  void* h_vals_out;    /* n values out (query; nullable)                       */
  uint8_t* h_status;   /* n status bytes out (nullable)                        */
} hwave_request;

typedef struct {
  uint32_t mode;          /* HWAVE_SERVE_*                                     */
  uint32_t slots;         /* batches in flight (batched mode)                  */
  uint64_t slot_ops;      /* staging capacity per batch, in operations         */
  uint32_t max_requests;  /* per batch (0 = 65536)                             */
  int32_t device;
} hwave_server_config;

typedef struct {
  uint64_t requests, ops, batches;
  double mean_requests_per_batch;
  double wall_s;                      /* first arrival to last completion     */
  double p50_ms, p99_ms, max_ms, mean_ms; /* completion - arrival             */
  uint64_t runtime_copied;            /* batched requests moved by runtime
                                         copies (arrays not device-mapped)    */
} hwave_serve_stats;

/* The tables (same key width; in the multi-table menu for batched mode) must
 * outlive the server. */
int hwave_server_create(hwave_server** out, hwave_table* const* tables, uint32_t n_tables,
                        const hwave_server_config* cfg);
/* Queues a request; arrival_s (hwave_now() clock, 0 = now) is its arrival time
 * for latency accounting.  *ticket identifies it for hwave_server_poll. */
int hwave_server_submit(hwave_server* s, const hwave_request* r, double arrival_s, uint64_t* ticket);
int hwave_server_poll(hwave_server* s, uint64_t ticket, int* done);
/* Blocks until every submitted request has completed. */
int hwave_server_drain(hwave_server* s);
/* Load generator: submits reqs[i] at t0 + offsets_s[i] (t0 = now + 1 ms, written
 * to *t0_out), sleeping between arrivals; returns when all are submitted. */
int hwave_server_replay(hwave_server* s, const hwave_request* reqs, const double* offsets_s, uint64_t n,
                        double* t0_out);
int hwave_server_stats(hwave_server* s, hwave_serve_stats* out);
int hwave_server_destroy(hwave_server* s);
/* Seconds on the server's monotonic clock. */
double hwave_now(void);

/* Query probe counters (the paper's probe unit, Section 5.1: unique 128-byte
 * lines a query touches), kept by instrumented builds of the library
 * (libhashwave_instr.so, compiled with -DHW_INSTRUMENT; its queries pay an
 * atomic per counted line).  Since the table's creation or the last reset:
 * queries counted, lines of buckets / tag buckets / chain nodes they read
 * (each bucket's lines counted once; slot designs count the lines of the
 * tile-width steps read up to a hit), and key/value slots read after a tag
 * match.  Cuckoo queries are not counted.  Also the upserts and inserts that
 * searched under their bucket lock (double hashing, power-of-two-choice,
 * iceberg) and the buckets those searches looked at before deciding: in the tag
 * designs one tag line each, the search part of Table 1's insert column.
 * Synchronises `stream`; reset != 0 zeroes the counters afterwards (on
 * `stream`).  Other builds return HWAVE_EUNSUPPORTED with *out zeroed. */
typedef struct {
  uint64_t queries;
  uint64_t bucket_lines;
  uint64_t slot_lines;
  uint64_t writes;
  uint64_t write_visits;
} hwave_probe_stats;
int hwave_probe_counters(hwave_table* t, hwave_probe_stats* out, int reset, void* stream);

/* Text of a return code; HIP error code of the last failing HIP call. */
const char* hwave_strerror(int code);
int hwave_last_hip_error(void);

/* Blocks until all work on `stream` is done (HIP error -> HWAVE_EDEVICE). */
int hwave_stream_sync(void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HASHWAVE_H */

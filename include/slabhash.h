/*
 * slabhash.h -- C ABI of an MI355X (gfx950) slab hash: the dynamic GPU hash table of
 * Ashkiani, Farach-Colton and Owens, "A Dynamic Hash Table for the GPU" (IPDPS 2018).
 *
 * The table is a direct-address array of B base slabs ("Slab Hash" subsection), each the head
 * of a slab list ("Slab list" subsection). Slabs are 256 bytes: 31 key/value slots of 8 bytes
 * (key in the low 32 bits, value in the high 32 bits), then one 8-byte word holding an auxiliary
 * 32-bit field and the 32-bit index of the next slab. Extra slabs come from a pool managed by a
 * wavefront-synchronous bitmap allocator in blocks of 2048 slabs ("Dynamic memory allocation":
 * SlabAlloc; the table's own pool is one contiguous array, and further super blocks can be
 * registered, see sh_add_super_block). A wavefront of 64 lanes processes the
 * operations its lanes hold one at a time ("warp-cooperative work sharing").
 *
 * Conventions for every call:
 *   - Pointers prefixed d_ are device pointers, caller-owned; the library never allocates or
 *     frees device memory. h_ pointers are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream). Operation calls are asynchronous:
 *     the caller keeps buffers alive until the stream has passed the call.
 *   - Keys are uint32 in [0, 0xFFFFFFFE]; 0xFFFFFFFF is reserved (the empty marker). Values
 *     are any uint32.
 *   - Argument errors (NULL where not allowed, zero buckets, storage too small or not 256-byte
 *     aligned, n >= 2^32) return SH_EINVAL before anything is enqueued; n == 0 is a no-op.
 *   - Errors found on the device (a reserved key in the input, pool exhausted) do not stop the
 *     call: the affected op gets status 0 (found 0, value 0xFFFFFFFF for a search) and a bit is
 *     set in the table's sticky error word, read by sh_stats.
 *   - sh_search, sh_insert, sh_delete and sh_mixed may run concurrently on one table from
 *     different streams, and each operation is linearizable with respect to the calls' time
 *     spans: an operation sees every update of a call that finished before its own call began,
 *     updates of calls running at the same time may or may not be seen, and each result is a
 *     state its key held at some instant during the call. sh_insert, sh_delete and sh_mixed read
 *     slabs device-coherently and are linearizable at the level of single operations as well.
 *     sh_search reads through the caches (a search after an update on another stream sees it
 *     once the update's call has finished); use sh_mixed with search ops for searches that must
 *     see updates completing while they run.
 *     sh_create, sh_reset, sh_stats and sh_dump must not overlap any other call on
 *     the same table.
 *   - Per-op status: search 1 found / 0 not found; insert 1 new key / 2 replaced the value of
 *     an existing key / 0 failed; delete 1 deleted / 0 absent or failed.
 */
#ifndef SLABHASH_H
#define SLABHASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SH_OK = 0,
    SH_EINVAL = 1, /* bad argument; nothing enqueued */
    SH_ENOMEM = 2, /* host-side allocation of the table handle failed */
    SH_EHIP = 3,   /* a HIP runtime call failed */
    SH_EBUSY = 4   /* resource busy (server admission) */
} sh_status_t;

/* Op codes of sh_mixed. */
enum { SH_OP_SEARCH = 0, SH_OP_INSERT = 1, SH_OP_DELETE = 2 };

/* Bits of the sticky device error word. */
enum { SH_ERR_RESERVED_KEY = 1u, SH_ERR_POOL_EXHAUSTED = 2u };

#define SH_EMPTY_KEY 0xFFFFFFFFu
#define SH_HASH_PRIME 4294967291u /* p of the bucket hash, the largest prime below 2^32 */
#define SH_SLAB_BYTES 256u
#define SH_SLAB_PAIRS 31u
#define SH_BLOCK_SLABS 2048u /* pool slabs per allocator block (one 256-byte bitmap) */

/* Table geometry and hash ("Slab Hash" subsection): bucket(k) = ((a k + b) mod p) mod B. */
/* Table flags ("Supported Operations"): with SH_TABLE_DUPLICATES the table is a multiset: an
   insert adds its pair without looking for the key (INSERT, not REPLACE), and a delete turns the
   first matching slot into an empty slot that later inserts may fill (the paper's deletion when
   duplicates are allowed). Without it keys are unique (REPLACE) and deleted slots stay
   tombstones. Searches return the first match in list order in both modes.
   With SH_TABLE_KEYS_ONLY the table holds keys alone (the paper's 32-bit entries): a slab holds
   62 keys, then its auxiliary word and next index, each four bytes. Inserts ignore d_vals (it may
   be NULL); a search that finds its key reports the key itself as the value. 0xFFFFFFFE is then
   reserved too, as the deleted-entry marker (the paper reserves two key values, empty and
   deleted); an operation carrying it fails like one carrying 0xFFFFFFFF. The two flags combine. */
enum { SH_TABLE_DUPLICATES = 1u, SH_TABLE_KEYS_ONLY = 2u };

typedef struct {
    uint32_t num_buckets; /* B >= 1 */
    uint32_t pool_slabs;  /* slabs beyond the base slabs (super block 0): a multiple of
                             SH_BLOCK_SLABS, at most 2^27 - 2048, may be 0 */
    uint32_t hash_a;      /* 1 <= a < p */
    uint32_t hash_b;      /* 0 <= b < p */
    uint32_t flags;       /* SH_TABLE_DUPLICATES and/or SH_TABLE_KEYS_ONLY; other bits invalid */
} sh_params_t;

/* Launch shape of the operation kernels. Never changes results.
   waves_per_cu: persistent grid of waves_per_cu * (compute units) wavefronts, at most 64
                 (0 = the operation's default: 20 for inserts and deletes, 32 for
                 sh_search_all and sh_delete_all, 16 otherwise, lowered to the wavefronts of
                 the chosen kernel that fit on a compute unit at once; a value set here is used
                 as given).
   ops_per_wave: operations each wavefront holds at a time, one per lane: 8, 16, 32 or 64
                 (0 = chosen per call: the operation's largest chunk, 16 for inserts and
                 deletes, 32 for searches, 64 for mixed batches, whatever the table's
                 flags, halved while the batch's chunks would not fill the grid; 8 for
                 sh_search_all and sh_delete_all, which by default run up to 32 wavefronts
                 per CU).
   flags:        SH_LAUNCH_COUNTERS makes the operation kernels accumulate the counters that
                 sh_stats reports (off by default: it adds atomics at the end of each kernel). */
enum { SH_LAUNCH_COUNTERS = 1u };
typedef struct {
    uint32_t waves_per_cu;
    uint32_t ops_per_wave;
    uint32_t flags;
    uint32_t reserved;
} sh_launch_t;

typedef struct sh_table sh_table_t; /* opaque host handle */

typedef struct {
    uint64_t live;           /* live key/value pairs */
    uint64_t tombstones;     /* deleted slots still occupying space */
    uint64_t slabs_total;    /* base slabs + linked pool slabs */
    uint64_t pool_allocated; /* set bits in the allocator bitmaps */
    uint64_t pool_capacity;  /* pool_slabs */
    uint32_t error_word;     /* SH_ERR_* bits raised since create/reset */
    uint32_t violations;     /* structure-invariant violations seen by the walk (0 expected) */
    uint32_t num_buckets, hash_a, hash_b, hash_p;
    /* Operation counters since create/reset, summed over wavefronts, accumulated only while
       SH_LAUNCH_COUNTERS is set: decision rounds (one per chunk of ops and pass over it), swaps
       lost to another wavefront, slabs allocated, links lost (slab freed again), allocator
       moves to another block, allocator claims that found their bitmap bit already taken by
       another wavefront (sh_alloc_slabs counts its allocations, block moves and lost claims
       here too). */
    uint64_t rounds, cas_lost, allocs, link_lost, block_moves, alloc_lost;
} sh_stats_t;

/* Device bytes a table with these parameters needs (header + base slabs + pool + bitmaps).
   Returns 0 for invalid parameters (including num_buckets + pool_slabs >= 2^32 - 1). */
size_t sh_storage_bytes(const sh_params_t *p);

/* Bind a table to caller-owned device storage (256-byte aligned, at least sh_storage_bytes)
   and enqueue its initialisation on `stream`: every slot empty, every next pointer empty, all
   pool slabs free, error word cleared. On success *out receives a host handle. */
sh_status_t sh_create(const sh_params_t *p, void *d_storage, size_t bytes, void *stream,
                      sh_table_t **out);

/* Re-initialise the table in place: afterwards its storage is byte for byte what sh_create's
   initialisation writes. Only the header, the base slabs, the pool slabs in use and the bitmaps
   are written: a free pool slab is always empty (allocation hands slabs out untouched, an
   insert that loses the link of its new slab takes its pair out again before freeing it, FLUSH
   empties the slabs it frees, sh_free_slabs takes empty slabs only). Must not overlap any other
   call on the table. */
sh_status_t sh_reset(sh_table_t *t, void *stream);

/* FLUSH ("Flush" subsection) of buckets first_bucket .. first_bucket + num_buckets - 1. In each
   bucket the live elements move, in list order, to the front of its slab list; deleted elements
   are dropped; the list is cut to max(1, ceil(live / 31)) slabs, and the slabs cut off are reset
   to empty and returned to the pool. Later operations give the same results as without the
   flush; only the layout, the deleted count and the slab count change. Like sh_reset it must not
   overlap any other call on the table. (A server started on the table counts pool use from the
   allocations it sees, so slabs a flush frees become available to its admission only after it
   is restarted.) Requires first_bucket <= B and num_buckets <= B - first_bucket, else
   SH_EINVAL; num_buckets == 0 is a no-op. Asynchronous on `stream`. */
sh_status_t sh_flush(sh_table_t *t, uint32_t first_bucket, uint32_t num_buckets, void *stream);

/* SlabAlloc on its own ("Dynamic memory allocation"), for measuring and testing the allocator
   the way the paper does (one million slab allocations, one per thread). Request i of n is
   served by lane i % 64 of wavefront i / 64; the wavefront serves its lanes one at a time from
   its resident block, as when a list needs a new slab. d_out[i] (device, n entries) receives
   the pool index of a free slab, now marked allocated, or 0xFFFFFFFF once the pool is exhausted
   (SH_ERR_POOL_EXHAUSTED is then set in the error word). The slabs belong to no list: use a
   table set aside for this, or return them with sh_free_slabs before the table serves
   operations again (sh_stats counts them in pool_allocated). n < 2^32, else SH_EINVAL; n == 0 is
   a no-op. Asynchronous; must not overlap other calls on the table. */
sh_status_t sh_alloc_slabs(sh_table_t *t, uint64_t n, uint32_t *d_out, void *stream);

/* Return slabs to the pool: the bit of every entry of d_idx (device, n entries) below the pool
   size is cleared in its block's bitmap; other entries are skipped. The slabs must belong to no
   list and still be empty (all ones), as allocation hands them out: allocations do not clear
   slabs. n < 2^32, else SH_EINVAL. Asynchronous; must not overlap other calls on the table. */
sh_status_t sh_free_slabs(sh_table_t *t, const uint32_t *d_idx, uint64_t n, void *stream);

/* Super blocks ("Dynamic memory allocation": SlabAlloc's pool is a set of super blocks, each
   of memory blocks of memory units, addressed by one 32-bit word). A table's own pool is its
   super block 0. sh_add_super_block registers caller-owned device memory d_mem (256-byte
   aligned) as the table's next super block: the most slabs S (a multiple of SH_BLOCK_SLABS,
   at most 2^27 - 2048) whose S * 256 bytes of slabs plus S / 2048 bitmap rows of 256 bytes fit
   in `bytes` (sh_super_block_bytes(S) gives the bytes for S slabs), laid out as those slabs
   followed by their bitmap rows. It enqueues the memory's initialisation (every slab empty,
   every bitmap bit free) and the super block's entry in the table's directory on `stream`.
   A pool slab's address, the next index stored in a slab, is then its super block in the top
   5 bits and its slab within the super block in the low 27 (allocator block in bits 26..11,
   slab within the block in bits 10..0); super block 0's addresses are its plain slab indices.
   The allocator hands out slabs of the super blocks it is using and moves on to the next
   registered super block only once a full cycle of those finds no free slab, so memory
   registered ahead of need is used when the pool would otherwise run out (an insert fails
   with the pool-exhausted error only when every registered super block is full). At most
   SH_MAX_SUPER_BLOCKS super blocks per table, super block 0 included; sh_reset keeps them
   registered and empties them; sh_stats counts them in pool_capacity and pool_allocated.
   Must not overlap other calls on the table (a server started earlier does not see later
   super blocks). SH_EINVAL for a NULL or misaligned d_mem, fewer bytes than one block, or a
   table that already has SH_MAX_SUPER_BLOCKS. The memory stays the caller's and must outlive
   the table's use. */
#define SH_MAX_SUPER_BLOCKS 32u
size_t sh_super_block_bytes(uint32_t slabs); /* 0 unless a positive multiple of 2048, <= 2^27 - 2048 */
sh_status_t sh_add_super_block(sh_table_t *t, void *d_mem, size_t bytes, void *stream);

/* Free the host handle only; the device storage stays the caller's. Handles that belong to a
   multi-table object (sh_multi_table) give SH_EINVAL. */
sh_status_t sh_destroy(sh_table_t *t);

/* Set the launch shape used by later calls on this table (NULL restores the default).
   Out-of-range fields give SH_EINVAL. */
sh_status_t sh_set_launch(sh_table_t *t, const sh_launch_t *shape);

/* The launch shape a call of n operations of one kind would use on this table now, after
   sh_set_launch and the defaults above: kind is SH_OP_SEARCH, SH_OP_INSERT (build and insert),
   SH_OP_DELETE, or SH_KIND_MIXED (sh_mixed). *waves_per_cu and *ops_per_wave receive the
   wavefronts per compute unit of the persistent grid and the ops each wavefront holds at a
   time; the grid is the smaller of that many wavefronts and the batch's chunks. Host-only.
   A NULL argument or an unknown kind gives SH_EINVAL. */
enum { SH_KIND_MIXED = 3 };
sh_status_t sh_launch_shape(const sh_table_t *t, int kind, uint64_t n, uint32_t *waves_per_cu,
                            uint32_t *ops_per_wave);

/* Bulk build: insert n pairs, each lane of a wavefront holding one ("Bulk benchmarks"; the
   paper notes a bulk build and an incremental batch insertion are the same operation). Uses
   REPLACE semantics ("Supported Operations": replace the value of an existing key, else insert
   at the first empty slot, else in slot 0 of a new slab linked when the tail is full); on a table with
   SH_TABLE_DUPLICATES, INSERT semantics (the first empty slot from the head, status always 1
   unless the pool is exhausted). d_status may be NULL. */
sh_status_t sh_build(sh_table_t *t, const uint32_t *d_keys, const uint32_t *d_vals, uint64_t n,
                     uint8_t *d_status, void *stream);

/* Incremental insertion of a batch ("Incremental insertion" experiment): same semantics and
   kernel as sh_build. */
sh_status_t sh_insert(sh_table_t *t, const uint32_t *d_keys, const uint32_t *d_vals,
                      uint64_t n, uint8_t *d_status, void *stream);

/* DELETE ("Deletion" subsection): the first matching slot in list order becomes a tombstone
   (never empty again, so not reused), or on a table with SH_TABLE_DUPLICATES an empty slot.
   Absent keys give status 0. d_status may be NULL. */
sh_status_t sh_delete(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint8_t *d_status,
                      void *stream);

/* SEARCH ("Search" subsection): d_vals_out[i] = value of d_keys[i], or 0xFFFFFFFF if absent.
   d_found (may be NULL) gets 1/0; it is authoritative since a stored value may be 0xFFFFFFFF. */
sh_status_t sh_search(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_vals_out,
                      uint8_t *d_found, void *stream);

/* Concurrent mixed batch ("Concurrent benchmarks"): d_ops[i] in {SH_OP_SEARCH, SH_OP_INSERT,
   SH_OP_DELETE} applies to d_keys[i] (and d_vals_in[i] for inserts); all ops of the batch run
   concurrently and the outcome is linearizable. d_vals_out[i] gets the search result
   (0xFFFFFFFF for non-search ops), d_status[i] the op's status. Unknown op codes give status 0. */
sh_status_t sh_mixed(sh_table_t *t, const uint8_t *d_ops, const uint32_t *d_keys,
                     const uint32_t *d_vals_in, uint64_t n, uint32_t *d_vals_out,
                     uint8_t *d_status, void *stream);

/* SEARCHALL ("Supported Operations"; "Search": the whole list is searched): for each key, every
   live element with that key, in list order. d_counts[i] receives how many there are. With
   d_offsets and d_vals_out (both or neither), query i's values also go to d_vals_out[d_offsets[i]],
   d_vals_out[d_offsets[i] + 1], ..., but never past d_offsets[i + 1] (d_vals_cap for the last
   query): a caller sizes the output from the counts of a first call without them (their
   exclusive prefix sum gives the offsets), and a table changed in between cannot make a query
   write outside its range. Reads through the caches, like sh_search. */
sh_status_t sh_search_all(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_counts,
                          const uint64_t *d_offsets, uint32_t *d_vals_out, uint64_t d_vals_cap,
                          void *stream);

/* DELETEALL ("Supported Operations"; "Deletion": the whole list is processed): every live
   element with the key is deleted as sh_delete deletes one (a tombstone, or an empty slot with
   SH_TABLE_DUPLICATES). d_counts[i] (may be NULL) receives how many this call deleted. */
sh_status_t sh_delete_all(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_counts,
                          void *stream);

/* Walk every bucket and return totals, allocator occupancy and the error word in *h_out.
   Synchronises `stream`. */
sh_status_t sh_stats(sh_table_t *t, sh_stats_t *h_out, void *stream);

/* Walk every bucket and emit each live pair as (bucket, key, value) into the device arrays
   (at most cap entries, in no particular order); *d_count (device uint64) receives the number
   of live pairs even if larger than cap. d_bucket_counts (may be NULL) receives, per bucket,
   three uint32: live, tombstones, slabs. d_violations (device uint32, may be NULL) receives the
   number of invariant violations found: on unique-key tables an empty slot before a full one
   or in a non-tail slab; on every table a malformed slot or auxiliary word, a next index out of
   range or not allocated, a chain that does not end. Every output is written by the call (no pre-zeroing needed). */
sh_status_t sh_dump(sh_table_t *t, uint32_t *d_bucket, uint32_t *d_key, uint32_t *d_val,
                    uint64_t cap, uint32_t *d_bucket_counts, uint64_t *d_count,
                    uint32_t *d_violations, void *stream);

/* ---- Batched form: many tables, one launch ------------------------------------------------
   A multi-table object holds T independent slab hashes (each with its own buckets, pool and
   hash) in one caller-owned device allocation, plus a device directory of them. One call runs
   the ops of many per-table batches in a single persistent kernel launch; that launch can be
   captured once into a HIP graph and replayed. */

#define SH_MAX_BATCHES 4096u /* descriptors per batched launch */

/* Ops [offset, offset + length) of the shared op arrays go to table `table`. */
typedef struct {
    uint64_t offset;
    uint32_t length;
    uint32_t table;
} sh_batch_desc_t;

typedef struct sh_multi sh_multi_t;
typedef struct sh_graph sh_graph_t;

/* Device bytes for T tables with these parameters (directory + each table's storage, each
   256-byte aligned). Returns 0 if T == 0 or any parameter set is invalid. */
size_t sh_multi_storage_bytes(uint32_t T, const sh_params_t *h_params);

/* Bind T tables to caller-owned storage (256-byte aligned, at least sh_multi_storage_bytes) and
   enqueue their initialisation and the directory upload on `stream`. The batched kernel runs
   the unique-key operations on key-value pairs: tables with any flag give SH_EINVAL. */
sh_status_t sh_multi_create(uint32_t T, const sh_params_t *h_params, void *d_storage,
                            size_t bytes, void *stream, sh_multi_t **out);

/* Handle of table t for the single-table calls (build, search, stats, dump, ...). It stays
   owned by the multi-table object: sh_destroy rejects it with SH_EINVAL. */
sh_status_t sh_multi_table(sh_multi_t *m, uint32_t t, sh_table_t **out);

/* Launch shape for sh_multi_mixed (same fields as sh_set_launch). */
sh_status_t sh_multi_set_launch(sh_multi_t *m, const sh_launch_t *shape);

/* Run nb batches (d_desc, device memory, nb <= SH_MAX_BATCHES) in one launch. The op arrays
   (d_ops, d_keys, d_vals_in, d_vals_out, d_status) hold n_ops entries. Each batch is a
   concurrent mixed batch on its table with the semantics of sh_mixed; batches on different
   tables are independent, and several batches on one table run concurrently with each other.
   Descriptor contents are read on the device at run time, so a captured launch can be replayed
   with new descriptors and ops written into the same buffers. On the device, a descriptor
   naming a table >= T is skipped and ranges are clipped to [0, n_ops); overlapping ranges give
   unspecified results for the overlapping ops. nb == 0 or n_ops == 0 is a no-op. */
sh_status_t sh_multi_mixed(sh_multi_t *m, const sh_batch_desc_t *d_desc, uint32_t nb,
                           const uint8_t *d_ops, const uint32_t *d_keys,
                           const uint32_t *d_vals_in, uint32_t *d_vals_out, uint8_t *d_status,
                           uint64_t n_ops, void *stream);

/* The same batches as sh_multi_mixed, but the plain way: one sh_mixed launch per descriptor,
   issued in order on `stream` from host-side descriptors h_desc (nb of them, any number).
   Descriptors naming a table >= T or a range outside [0, n_ops) give SH_EINVAL before anything
   is enqueued. */
sh_status_t sh_multi_mixed_each(sh_multi_t *m, const sh_batch_desc_t *h_desc, uint32_t nb,
                                const uint8_t *d_ops, const uint32_t *d_keys,
                                const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                uint8_t *d_status, uint64_t n_ops, void *stream);

/* Capture one sh_multi_mixed launch with these arguments into an executable HIP graph. The
   graph reads the same buffers on every replay. */
sh_status_t sh_multi_graph(sh_multi_t *m, const sh_batch_desc_t *d_desc, uint32_t nb,
                           const uint8_t *d_ops, const uint32_t *d_keys,
                           const uint32_t *d_vals_in, uint32_t *d_vals_out, uint8_t *d_status,
                           uint64_t n_ops, sh_graph_t **out);

/* Capture instead of run: the work that the calls made from this host thread enqueue on
   `stream` between sh_capture_begin and sh_capture_end is recorded into one HIP graph, which
   sh_graph_launch replays as a single submission (a sequence of many short launches, such as a
   round of batched launches or a whole build-search-mixed pass, then pays one launch cost).
   Every call that only enqueues kernels may be captured: sh_reset, sh_build, sh_insert,
   sh_delete, sh_search, sh_mixed, sh_flush, sh_search_all, sh_delete_all, sh_alloc_slabs,
   sh_free_slabs, sh_multi_mixed and sh_multi_mixed_each. A replay runs them with the
   arguments given at capture (the same pointers, sizes and launch shapes) on whatever the
   buffers hold when it runs. Calls that synchronise or read results on the host (sh_stats,
   sh_dump, the server) must not be made on a capturing stream. The NULL stream cannot be
   captured (SH_EINVAL), nor one already capturing. sh_capture_end returns SH_EHIP if the
   capture failed (a call above made an uncapturable request); the stream is then no longer
   capturing either way. */
sh_status_t sh_capture_begin(void *stream);
sh_status_t sh_capture_end(void *stream, sh_graph_t **out);

/* Replay a captured graph on `stream`. */
sh_status_t sh_graph_launch(sh_graph_t *g, void *stream);

/* Free the graph and its handle; SH_EHIP if HIP reported an error while destroying it. */
sh_status_t sh_graph_destroy(sh_graph_t *g);

/* Free the host objects only; the device storage stays the caller's. */
sh_status_t sh_multi_destroy(sh_multi_t *m);

/* ---- Served form: continuous batching -----------------------------------------------------
   A server owns one table and a native request loop. Requests are ranges of ops already in the
   server's device op arrays (n_ops entries; results go to the same positions of d_vals_out and
   d_status). A request is admitted when fewer than max_requests are unfinished and the pool's
   free slabs, minus those promised to unfinished requests and reserve_slabs, cover its worst
   case (one new slab per insert). The loop gathers every admitted request not yet on the
   device, up to max_batch_ops ops (and SH_MAX_BATCHES requests), into one launch of the
   batched kernel, one descriptor per request; up to max_launches launches run at once on their
   own streams, so work admitted while others run overlaps with them on the device. Requests
   of one launch, and of launches in flight together, run concurrently: results are
   linearizable, with requests that finished before another was admitted ordered before it. */

typedef struct {
    uint32_t max_launches;  /* launches in flight at once, 1..8 (0 = 4) */
    uint32_t max_batch_ops; /* ops one launch takes at most (0 = 2^20); a larger request runs alone */
    uint32_t max_requests;  /* admitted, unfinished requests at most (0 = 4096) */
    uint32_t reserved0;
    uint64_t reserve_slabs; /* pool slabs never promised to requests */
} sh_server_cfg_t;

typedef struct {
    uint64_t offset;  /* ops [offset, offset + length) of the server's op arrays */
    uint32_t length;
    uint32_t inserts; /* insert ops among them: bounds the new slabs the request can need */
} sh_request_t;

typedef struct sh_server sh_server_t;

/* Device scratch the server needs (directory + one descriptor buffer per launch slot). */
size_t sh_server_scratch_bytes(const sh_server_cfg_t *cfg);

/* Start serving table t. d_scratch: caller-owned device memory (256-byte aligned, at least
   sh_server_scratch_bytes). Synchronises `stream` once to read the pool occupancy. No other call
   may use the table while the server runs. A table with any flag gives SH_EINVAL (requests run
   through the batched kernel); SH_EHIP if a HIP call fails, SH_ENOMEM if host memory or the
   server thread cannot be had (nothing is left running in either case). */
sh_status_t sh_server_start(sh_table_t *t, const sh_server_cfg_t *cfg, const uint8_t *d_ops,
                            const uint32_t *d_keys, const uint32_t *d_vals_in,
                            uint32_t *d_vals_out, uint8_t *d_status, uint64_t n_ops,
                            void *d_scratch, size_t scratch_bytes, void *stream,
                            sh_server_t **out);

/* Admit a request. SH_OK gives a ticket; SH_EBUSY means not admissible now (retry later);
   SH_ENOMEM means it can never be admitted (its worst case exceeds the pool) or the server's
   host records could not grow (nothing was admitted); SH_EINVAL for a range outside the op
   arrays, an empty request or a stopping server. */
sh_status_t sh_server_submit(sh_server_t *s, const sh_request_t *req, uint64_t *ticket);

/* *done = 1 once the request's results are in device memory; times on sh_clock_ns's clock.
   A server remembers the last 2^20 tickets; an older ticket whose finish has been reported (by a
   poll that returned *done = 1, or by sh_server_replay) expires and gives SH_EINVAL, as does any
   finished ticket 2^22 or more behind the newest. */
sh_status_t sh_server_poll(sh_server_t *s, uint64_t ticket, int *done, uint64_t *t_admit_ns,
                           uint64_t *t_done_ns);

/* Load driver: submit request i at time t0 + arrival_ns[i] (t0 = the call's start; arrival_ns
   non-decreasing), keeping requests that are not yet admissible in arrival order, until all
   have finished. admit_ns[i] and done_ns[i] (relative to t0) receive the admission and
   completion times; a request that can never be admitted gets UINT64_MAX in both. SH_EHIP if
   the server reports a HIP error; SH_ENOMEM if the driver's host bookkeeping cannot be
   allocated (requests already submitted still run on the server). */
sh_status_t sh_server_replay(sh_server_t *s, const sh_request_t *h_reqs,
                             const uint64_t *h_arrival_ns, uint64_t n, uint64_t *h_admit_ns,
                             uint64_t *h_done_ns);

/* Finish all admitted work, stop the loop and free the server's host resources. */
sh_status_t sh_server_stop(sh_server_t *s);

/* The server's monotonic clock, in nanoseconds. */
uint64_t sh_clock_ns(void);

/* Short description of a status code. */
const char *sh_strerror(sh_status_t s);

#ifdef __cplusplus
}
#endif

#endif /* SLABHASH_H */

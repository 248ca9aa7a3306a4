/*
 * slabhash_roofs.h -- microbenchmarks of the memory access patterns the slab hash is made of,
 * used to measure the ceilings its kernels run against on one GPU. Nothing here touches a table.
 *
 * The patterns, each over a buffer of whole 256-byte slabs with slab s of operation i chosen by
 * a fixed 32-bit mix of (seed + i) scaled into [0, slabs):
 *   SH_ROOF_SLAB_LOAD  one operation = one 256-byte slab read by half a wavefront, 8 bytes per
 *                      lane with device-coherent loads; a wavefront reads two slabs per load
 *                      instruction, as the operation kernels do ("Search": one slab read per
 *                      operation when the key is in its base slab).
 *   SH_ROOF_CAS        one operation = one 64-bit compare-and-swap with return, device scope, on
 *                      a random word of a random slab, expecting all ones (an empty slot); one
 *                      operation per lane.
 *   SH_ROOF_LOAD_CAS   one operation = one slab read as in SH_ROOF_SLAB_LOAD, then one 64-bit
 *                      compare-and-swap on the slab's first all-ones word (slot 0 if none) by
 *                      the half-wavefront's first lane: the memory pattern of an insert that
 *                      finds its key absent and an empty slot in its base slab ("Insertion").
 *
 * The compare-and-swap patterns overwrite the words they win; fill the buffer with 0xFF bytes
 * before each timed run so every run starts from empty slots.
 *
 * sh_roof_search is the memory pattern of a search whose every list is one slab ("Search": one
 * slab read per operation), with the query and result streams: op i loads d_keys[i], reads
 * slab mix(d_keys[i]) scaled into [0, slabs) through the caches (half a wavefront, 8 bytes per
 * lane), and writes the high word of the first of slots 0..30 whose low word equals the key to
 * d_vals_out[i] (all ones if none) and 1/0 to d_found[i]. It reads the buffer only.
 *
 * sh_roof_insert is the memory pattern of an insert whose key is absent and whose base slab has
 * room ("Insertion"), with its input and status streams: op i loads d_keys[i] and d_vals[i],
 * reads slab mix(d_keys[i]) scaled into [0, slabs) with device-coherent loads (half a
 * wavefront, 8 bytes per lane), swaps the pair (value in the high word) into the first
 * all-ones slot of 0..30 (slot 0 if none), expecting all ones, and writes 1 to d_status[i] if
 * the swap won, else 0. Fill the buffer with 0xFF bytes before each timed run.
 */
#ifndef SLABHASH_ROOFS_H
#define SLABHASH_ROOFS_H

#include <stddef.h>
#include <stdint.h>

#include "slabhash.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { SH_ROOF_SLAB_LOAD = 0, SH_ROOF_CAS = 1, SH_ROOF_LOAD_CAS = 2 };

/* Enqueue n_ops operations of pattern `kind` over d_buf on `stream` (a hipStream_t, NULL = the
   default stream); asynchronous.
   d_buf:        device buffer, 256-byte aligned, caller-owned.
   bytes:        a multiple of 256, at least 256, at most (2^32 - 1) * 256.
   n_ops:        below 2^32 - 64; 0 is a no-op.
   waves_per_cu: persistent grid of waves_per_cu * (compute units) wavefronts, 1..64 (0 = 32).
   depth:        operations in flight per wavefront iteration: the slab patterns issue the loads
                 of `depth` op pairs before using any; the swap pattern issues `depth` swaps per
                 lane back to back. 1, 4, 8 or 16 (0 = 8).
   Returns SH_EINVAL for a bad kind or argument (nothing enqueued), SH_EHIP if the device query
   or the launch fails, else SH_OK. */
sh_status_t sh_roof_run(int kind, void *d_buf, size_t bytes, uint64_t n_ops,
                        uint32_t waves_per_cu, uint32_t depth, uint32_t seed, void *stream);

/* Enqueue n_ops one-slab searches (above) over d_buf on `stream`; asynchronous.
   d_buf, bytes, n_ops, waves_per_cu: as for sh_roof_run; the buffer is not written.
   d_keys:       n_ops keys (device, caller-owned); any 32-bit values.
   d_vals_out:   n_ops values out; d_found: n_ops flags out (device, caller-owned).
   depth:        op pairs whose slab loads are issued before any is used: 1, 4, 8 or 16 (0 = 8);
                 a wavefront takes 2 * depth ops per iteration.
   Returns SH_EINVAL for a bad argument or, with n_ops > 0, a NULL array (nothing enqueued),
   SH_EHIP if the device query or the launch fails, else SH_OK. */
sh_status_t sh_roof_search(const void *d_buf, size_t bytes, const uint32_t *d_keys,
                           uint64_t n_ops, uint32_t *d_vals_out, uint8_t *d_found,
                           uint32_t waves_per_cu, uint32_t depth, void *stream);

/* Enqueue n_ops one-slab inserts (above) over d_buf on `stream`; asynchronous.
   d_buf, bytes, n_ops, waves_per_cu, depth: as for sh_roof_search; the buffer is written.
   d_keys, d_vals: n_ops keys and values (device, caller-owned).
   d_status:     n_ops statuses out (device, caller-owned).
   Returns SH_EINVAL for a bad argument or, with n_ops > 0, a NULL array (nothing enqueued),
   SH_EHIP if the device query or the launch fails, else SH_OK. */
sh_status_t sh_roof_insert(void *d_buf, size_t bytes, const uint32_t *d_keys,
                           const uint32_t *d_vals, uint64_t n_ops, uint8_t *d_status,
                           uint32_t waves_per_cu, uint32_t depth, void *stream);

#ifdef __cplusplus
}
#endif

#endif

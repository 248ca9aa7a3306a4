// Slab hash for MI355X (gfx950, wave64): kernels and the C ABI declared in include/slabhash.h.
//
// Paper: Ashkiani, Farach-Colton, Owens, "A Dynamic Hash Table for the GPU".
//
// Memory layout of one table (one caller-owned device allocation, 256-byte aligned):
//   [header 4 KB][B base slabs][P pool slabs][P/2048 bitmap rows of 256 B]
// A slab is 256 B = 32 eight-byte words. Words 0..30 are key/value slots (key in the low half,
// value in the high half); word 31 holds an auxiliary half (always 0xFFFFFFFF) and the index
// of the next pool slab (0xFFFFFFFF = none) in its high half. Slot encodings:
//   empty     = key 0xFFFFFFFF, value 0xFFFFFFFF
//   tombstone = key 0xFFFFFFFF, value 0          (a deleted element, never empty again)
//   live      = key != 0xFFFFFFFF
// A wavefront reads a slab with one 8-byte load per lane: lanes 0..31 cover slots 0..31 and
// lanes 32..63 either mirror them or hold a second slab. Each slot is therefore read whole, so a
// reader never sees a key from one write and a value from another.
//
// Work sharing ("Our warp-cooperative work sharing strategy"): every lane holds one operation
// and the whole wavefront decides the queued operations one at a time in lane order, with
// ballots and lane reads; the slab loads for all of a chunk's operations are issued ahead of the
// decisions and the resulting swaps are committed together (see ops_kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "slabhash.h"

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kEmptyPair = ~0ull;
constexpr uint64_t kTombPair = 0x00000000FFFFFFFFull; // key half all ones, value half 0
constexpr uint32_t kTombKey = 0xFFFFFFFEu;            // a deleted entry of a key-only slab
constexpr uint32_t kKeyEntries = 62;                  // keys per key-only slab
constexpr uint64_t kSlotMask = 0x7FFFFFFFull;         // slots 0..30 of a half wavefront
constexpr uint32_t kPrime = SH_HASH_PRIME;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr size_t kHeaderBytes = 4096;   // Header, counter slots, super-block directory
constexpr uint32_t kCounterSlots = 32;   // 64-byte slots of 8 counters, one per wavefront % 32
constexpr uint32_t kFlagCounters = SH_LAUNCH_COUNTERS;
constexpr uint32_t kMaxBatches = SH_MAX_BATCHES;
constexpr uint32_t kDefaultWavesPerCU = 16;

enum Kind { kSearch = 0, kInsert = 1, kDelete = 2, kMixed = 3 };
static_assert(kSearch == SH_OP_SEARCH && kInsert == SH_OP_INSERT && kDelete == SH_OP_DELETE &&
                  kMixed == SH_KIND_MIXED,
              "kernel kinds are the public operation codes");

struct Header {
    uint32_t err;
    uint32_t violations;
    unsigned long long live, tomb, slabs, pool_alloc, dump_count;
};

// Super blocks ("Dynamic memory allocation"): super block 0 is the table's own pool, which
// directly follows the base slabs; super blocks 1 .. nsuper-1 are further caller-owned regions
// of slabs and bitmap rows, registered with sh_add_super_block. A pool slab's 32-bit address
// (the next index of a slab, an op's cursor) is its super block in the top 5 bits and its slab
// within the super block below (allocator block in bits 26..11, slab within the block in bits
// 10..0), so super block 0's addresses are plain pool indices. The allocator numbers the blocks
// of all super blocks in order of registration and moves on to the next super block only when
// a full cycle over the ones in use found no free slab.
constexpr uint32_t kSuperShift = 27;
constexpr uint32_t kSlabInSuper = (1u << kSuperShift) - 1u;
constexpr uint32_t kMaxSupers = SH_MAX_SUPER_BLOCKS;
constexpr uint32_t kMaxSuperSlabs = (1u << kSuperShift) - SH_BLOCK_SLABS;

struct SuperDesc {
    uint64_t *pool;   // its slab 0
    uint32_t *bitmap; // its bitmap rows
    uint32_t slabs;   // a multiple of SH_BLOCK_SLABS
    uint32_t first;   // allocator number of its first block
};
// Header bytes: [0, 256) Header, [256, 2304) counter slots, then the super-block directory, then
// the number of super blocks beyond super block 0 the allocator has moved on to.
constexpr size_t kDirOffset = 2304;
constexpr size_t kGrownOffset = kDirOffset + kMaxSupers * sizeof(SuperDesc);
static_assert(kGrownOffset + 16 <= 4096, "the directory fits in the header");

struct View {
    uint64_t *base;   // B slabs of 32 words
    uint64_t *pool;   // super block 0: P slabs of 32 words
    uint32_t *bitmap; // super block 0: P/2048 rows of 64 words
    Header *hdr;
    unsigned long long *counters; // kCounterSlots x 8
    const SuperDesc *dir;         // entries 1 .. nsuper-1 in use (entry 0 is pool/bitmap above)
    uint32_t *grown;              // super blocks beyond 0 the allocator has moved on to
    uint32_t B, a, b, pool_slabs, nblk;
    uint32_t nsuper, total_blocks; // super blocks registered, allocator blocks in all of them
    uint32_t mode; // SH_TABLE_DUPLICATES | SH_TABLE_KEYS_ONLY bits of the table's flags
};

// ---------------------------------------------------------------------------------------------
// Device primitives

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rl(uint32_t v, uint32_t lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t ffs0(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// This lane's bit of a wave-uniform lane mask (no instruction: the mask is used as the lane
// condition directly).
__device__ __forceinline__ bool inverse_ballot(uint64_t m)
{
    return __builtin_amdgcn_inverse_ballot_w64(m);
}

// Lanes holding a slot of a slab: every lane but slot 31 of each half (the next index).
constexpr uint64_t kSlotLanes = ~((1ull << 31) | (1ull << 63));

// A wave-uniform 64-bit value kept in scalar registers. (The builtin returns int: each half is
// taken back to uint32_t before widening, or the low half would be sign-extended.)
__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
    return ((uint64_t)hi << 32) | lo;
}

// v_writelane_b32: lane `j` of x takes the wave-uniform value v (bound to the LLVM intrinsic so
// the compiler still schedules and checks hazards around it).
extern "C" __device__ uint32_t sh_llvm_writelane(uint32_t v, uint32_t j, uint32_t x)
    __asm("llvm.amdgcn.writelane.i32");

__device__ __forceinline__ uint32_t wl(uint32_t x, uint32_t j, uint32_t v)
{
    return sh_llvm_writelane(v, j, x);
}

// s_waitcnt vmcnt(0): wait for every outstanding vector memory access of this wavefront
// (gfx9 encoding: vmcnt 0, expcnt 7, lgkmcnt 15 left unconstrained).
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Universal hash of the "Slab Hash" subsection: ((a k + b) mod p) mod B with p = 2^32 - 5.
// a k + b < 2^64; since 2^32 = 5 (mod p) two folds of the high half bring it below 2^32 + 30,
// and one conditional subtraction finishes the reduction mod p.
__device__ __forceinline__ uint32_t bucket_of(uint32_t k, uint32_t a, uint32_t b, uint32_t B)
{
    uint64_t x = (uint64_t)a * k + b;
    uint64_t t = (x >> 32) * 5u + (x & 0xFFFFFFFFull);
    t = (t >> 32) * 5u + (t & 0xFFFFFFFFull);
    uint32_t r = (t >= kPrime) ? (uint32_t)(t - kPrime) : (uint32_t)t;
    return r % B;
}

// Every table access goes through a global-address-space pointer: slab and bitmap addresses
// are often read back from LDS or from the super-block directory, where the compiler can no
// longer tell that they point to device memory, and would otherwise emit FLAT instructions.
// A FLAT access also counts against the LDS counter, so each LDS read between the loads of a
// straight run would wait for the loads issued before it.
template <typename X>
__device__ __forceinline__ __attribute__((address_space(1))) X *gmem(X *p)
{
    return (__attribute__((address_space(1))) X *)p;
}

// One 8-byte slab word. Coherent: an agent-scope relaxed atomic load, which sees the swaps of
// other XCDs and of kernels running at the same time on other streams (the update kernels
// re-read slabs after lost swaps, so they need it). Otherwise a plain load through the caches,
// which sees everything written before the kernel started: searches keep slabs that many lists
// share (the pool slabs of long lists) in L2.
template <bool Coherent>
__device__ __forceinline__ uint64_t load_slot(const uint64_t *p)
{
    if constexpr (Coherent)
        return __hip_atomic_load(gmem(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *gmem(p);
}

__device__ __forceinline__ uint32_t load_word_coherent(const uint32_t *p)
{
    return __hip_atomic_load(gmem(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t cas64(uint64_t *p, uint64_t expected, uint64_t desired)
{
    __hip_atomic_compare_exchange_strong(gmem(p), &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected; // the value found at p (equal to `expected` on success)
}

__device__ __forceinline__ uint32_t cas32(uint32_t *p, uint32_t expected, uint32_t desired)
{
    __hip_atomic_compare_exchange_strong(gmem(p), &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected;
}

__device__ __forceinline__ uint32_t or32(uint32_t *p, uint32_t m)
{
    return __hip_atomic_fetch_or(gmem(p), m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_error(const View &T, uint32_t bits, uint32_t lane,
                                            uint32_t who)
{
    if (lane == who)
        or32(&T.hdr->err, bits);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// ---------------------------------------------------------------------------------------------
// SlabAlloc for wave64 ("Dynamic memory allocation"). The pool is made of super blocks, each a
// contiguous array of blocks of 2048 slabs; a block's occupancy is one 256-byte bitmap row,
// which a wavefront holds in registers as one 32-bit word per lane (lane l covers slabs
// 32l .. 32l+31 of the block). The wavefront's "resident" block serves its allocations: lanes
// with a free bit vote, the first such lane in the wavefront's own priority order (lane order
// rotated by a per-wavefront offset) claims its lowest free bit with an atomic OR on the row in
// memory and, if the bit was still free, broadcasts the slab address. A lost race refreshes
// that lane's word. When the resident block is full the wavefront moves to the next block,
// reading its row with one coalesced load; after a full cycle of the blocks in use without
// success it moves on to the next registered super block, and with none left the pool counts
// as exhausted.

// Pool slab `idx` (a 32-bit pool address) and a cursor's slab (kEmpty = the bucket's base slab).
__device__ __forceinline__ uint64_t *pool_slab(const View &T, uint32_t idx)
{
    const uint32_t sb = idx >> kSuperShift;
    if (sb == 0)
        return T.pool + (size_t)idx * 32;
    return gmem(T.dir)[sb].pool + (size_t)(idx & kSlabInSuper) * 32;
}

__device__ __forceinline__ uint64_t *cursor_slab(const View &T, uint32_t loc, uint32_t bkt)
{
    return loc == kEmpty ? T.base + (size_t)bkt * 32 : pool_slab(T, loc);
}

// Whether `idx` addresses a slab of a registered super block.
__device__ __forceinline__ bool pool_in_range(const View &T, uint32_t idx)
{
    const uint32_t sb = idx >> kSuperShift;
    if (sb == 0)
        return idx < T.pool_slabs;
    return sb < T.nsuper && (idx & kSlabInSuper) < gmem(T.dir)[sb].slabs;
}

// The bitmap word holding pool slab idx's bit (bit idx mod 32).
__device__ __forceinline__ uint32_t *bitmap_word(const View &T, uint32_t idx)
{
    const uint32_t sb = idx >> kSuperShift, i = idx & kSlabInSuper;
    uint32_t *bm = sb ? gmem(T.dir)[sb].bitmap : T.bitmap;
    return bm + (size_t)(i >> 11) * 64 + ((i >> 5) & 63);
}

// Allocator block g (numbered over all registered super blocks): its bitmap row and the
// address of its first slab.
__device__ __forceinline__ void block_ref(const View &T, uint32_t g, uint32_t *&row,
                                          uint32_t &code)
{
    if (g < T.nblk) {
        row = T.bitmap + (size_t)g * 64;
        code = g * SH_BLOCK_SLABS;
        return;
    }
    uint32_t sb = 1;
    while (sb + 1 < T.nsuper && gmem(T.dir)[sb + 1].first <= g)
        ++sb;
    const uint32_t lb = g - gmem(T.dir)[sb].first;
    row = gmem(T.dir)[sb].bitmap + (size_t)lb * 64;
    code = (sb << kSuperShift) | (lb * SH_BLOCK_SLABS);
}

// Blocks of super block 0 and of the `grown` super blocks after it.
__device__ __forceinline__ uint32_t blocks_in_use(const View &T, uint32_t grown)
{
    return 1 + grown >= T.nsuper ? T.total_blocks : gmem(T.dir)[1 + grown].first;
}

struct Alloc {
    uint32_t blk;   // resident block (wave-uniform), kEmpty = none yet
    uint32_t word;  // this lane's bitmap word of the resident block
    uint32_t *row;  // the resident block's bitmap row
    uint32_t code;  // address of the resident block's first slab
    uint32_t nact;  // blocks in use (super blocks the allocator has reached)
    uint32_t moves; // block moves since the last successful allocation
    uint32_t total_moves;
    uint32_t start; // first block tried (taken modulo the blocks in use)
    uint32_t rot;   // this wavefront's rotation of the lane priority order
    uint32_t lost;  // claims that found their bit already taken by another wavefront
    bool full;      // this wavefront found the pool exhausted
};

__device__ __forceinline__ void alloc_goto(const View &T, Alloc &s, uint32_t g, uint32_t lane)
{
    s.blk = g;
    block_ref(T, g, s.row, s.code);
    s.word = load_word_coherent(&s.row[lane]);
}

// A full cycle over the blocks in use found no free slab: move on to the first block of the
// next registered super block (the first wavefront to get here records the move for all), or
// report that there is none.
__device__ bool alloc_grow(const View &T, Alloc &s, uint32_t lane)
{
    if (T.nsuper == 1)
        return false;
    uint32_t g = load_word_coherent(T.grown);
    if (blocks_in_use(T, g) <= s.nact && 1 + g < T.nsuper) {
        uint32_t old = 0;
        if (lane == 0)
            old = cas32(T.grown, g, g + 1);
        old = rl(old, 0);
        g = (old == g) ? g + 1 : old; // another wavefront may have moved on already
    }
    const uint32_t n = blocks_in_use(T, g);
    if (n <= s.nact)
        return false;
    const uint32_t first = s.nact;
    s.nact = n;
    s.moves = 0;
    alloc_goto(T, s, first, lane);
    return true;
}

// The wavefront's first block, its bitmap row read ahead of any need (kernels that may grow
// lists call this at their start, so the first allocation costs one atomic, not a row read and
// an atomic).
__device__ __forceinline__ void alloc_preload(const View &T, Alloc &s, uint32_t lane)
{
    if (T.total_blocks == 0 || s.blk != kEmpty)
        return;
    const uint32_t g = T.nsuper == 1 ? 0u : load_word_coherent(T.grown);
    s.nact = T.nsuper == 1 ? T.nblk : blocks_in_use(T, g);
    s.moves = 0;
    // start in the newest super block in use (the older ones had filled up when it was
    // reached); the cyclic moves still cover every block in use
    const uint32_t first = (g == 0 || g >= T.nsuper) ? 0u : gmem(T.dir)[g].first;
    if (s.nact <= first) {
        // nothing in use yet (the table's own pool is empty): the first registered super block
        if (!alloc_grow(T, s, lane))
            s.full = true;
        return;
    }
    alloc_goto(T, s, first + s.start % (s.nact - first), lane);
}

__device__ uint32_t wave_alloc(const View &T, Alloc &s, uint32_t lane)
{
    if (T.total_blocks == 0 || s.full)
        return kEmpty;
    if (s.blk == kEmpty) {
        alloc_preload(T, s, lane);
        if (s.full)
            return kEmpty;
    }
    for (;;) {
        const uint64_t free_lanes = ballot(s.word != kEmpty);
        if (free_lanes) {
            // the first lane with a free slab in this wavefront's priority order: lanes
            // rot, rot + 1, ..., 63, 0, ... (wavefronts sharing a block start at different
            // bitmap words instead of all claiming the same bit)
            const uint64_t r = (free_lanes >> s.rot) | (free_lanes << ((64u - s.rot) & 63u));
            const uint32_t l = (ffs0(r) + s.rot) & 63u;
            uint32_t got = kEmpty;
            if (lane == l) {
                const uint32_t bit = (uint32_t)__builtin_ctz(~s.word);
                const uint32_t m = 1u << bit;
                const uint32_t old = or32(&s.row[l], m);
                s.word = old | m;
                if (!(old & m))
                    got = s.code + l * 32 + bit;
            }
            const uint32_t idx = rl(got, l);
            if (idx != kEmpty) {
                s.moves = 0;
                return idx;
            }
            ++s.lost;
            continue;
        }
        if (++s.moves > s.nact) {
            if (alloc_grow(T, s, lane))
                continue;
            s.full = true;
            return kEmpty;
        }
        ++s.total_moves;
        alloc_goto(T, s, (s.blk + 1 >= s.nact) ? 0 : s.blk + 1, lane);
    }
}

// Exclusive prefix sum of x over the lanes in this wavefront's rotated order (lane rot first),
// and the total over all lanes.
__device__ __forceinline__ uint32_t rotated_scan(uint32_t x, uint32_t lane, uint32_t rot,
                                                 uint32_t *total)
{
    const uint32_t pos = (lane - rot) & 63u;
    uint32_t incl = x;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl((int)incl, (int)((lane - d) & 63u), 64);
        if (pos >= d)
            incl += t;
    }
    *total = (uint32_t)__shfl((int)incl, (int)((rot + 63u) & 63u), 64);
    return incl - x;
}

// Serve `need` (<= 64) allocations of this wavefront together from its resident block: the
// lanes whose bitmap words hold free bits claim, in the wavefront's rotated lane order, as many
// as are still needed, each with one atomic OR of several bits; bits another wavefront took in
// the meantime are left to the next pass. The j-th slab claimed (rotated lane order, then bit
// order) is written by its lane to out[j]. Moves on to the next block as wave_alloc does.
// Returns how many were served: `need`, unless the pool is exhausted.
__device__ uint32_t wave_alloc_many(const View &T, Alloc &s, uint32_t lane, uint32_t need,
                                    uint32_t *__restrict__ out)
{
    if (T.total_blocks == 0 || s.full)
        return 0;
    if (s.blk == kEmpty) {
        alloc_preload(T, s, lane);
        if (s.full)
            return 0;
    }
    uint32_t got = 0;
    while (got < need) {
        const uint32_t fw = ~s.word;
        uint32_t total;
        const uint32_t before = rotated_scan((uint32_t)__popc(fw), lane, s.rot, &total);
        if (total == 0) {
            if (++s.moves > s.nact) {
                if (alloc_grow(T, s, lane))
                    continue;
                s.full = true;
                break;
            }
            ++s.total_moves;
            alloc_goto(T, s, (s.blk + 1 >= s.nact) ? 0 : s.blk + 1, lane);
            continue;
        }
        // this lane's share: its lowest free bits, up to what the lanes before it leave over
        const uint32_t left = need - got;
        uint32_t take = before >= left ? 0u : left - before;
        uint32_t m = 0, f = fw;
        for (; take && f; --take) {
            m |= f & (0u - f);
            f &= f - 1u;
        }
        uint32_t mine = 0;
        if (m) {
            const uint32_t old = or32(&s.row[lane], m);
            mine = m & ~old;
            s.word = old | m;
        }
        s.lost += (uint32_t)__popcll(ballot((m & ~mine) != 0u));
        uint32_t served;
        uint32_t at = got + rotated_scan((uint32_t)__popc(mine), lane, s.rot, &served);
        for (uint32_t w = mine; w; w &= w - 1u)
            out[at++] = s.code + lane * 32 + (uint32_t)__builtin_ctz(w);
        got += served;
        if (served)
            s.moves = 0;
    }
    return got;
}

// The bits this lane claims so that the wavefront's lanes together claim `need` free slabs of
// the resident block (in the rotated lane order of wave_alloc_many, lowest free bits first); 0
// for every lane when there is no resident block yet. Fewer than `need` when the block holds
// fewer free slabs.
__device__ __forceinline__ uint32_t claim_plan(const Alloc &s, uint32_t lane, uint32_t need)
{
    if (s.blk == kEmpty || s.full)
        return 0u;
    const uint32_t fw = ~s.word;
    uint32_t total;
    const uint32_t before = rotated_scan((uint32_t)__popc(fw), lane, s.rot, &total);
    uint32_t take = before >= need ? 0u : need - before;
    uint32_t m = 0, f = fw;
    for (; take && f; --take) {
        m |= f & (0u - f);
        f &= f - 1u;
    }
    return m;
}

__device__ __forceinline__ void slab_free(const View &T, uint32_t idx)
{
    __hip_atomic_fetch_and(gmem(bitmap_word(T, idx)), ~(1u << (idx & 31)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------------------------
// Operation kernel. Persistent grid: wavefront w takes chunks w, w + W, w + 2W, ... of C ops
// (C = ops per wavefront, 8..64), lane l < C holding op l of its chunk. Each op keeps a cursor
// `loc` (kEmpty = its bucket's base slab, else a pool slab index). The pool directly follows the
// base slabs in memory, so slab (loc == kEmpty ? bucket : B + loc) of the base array addresses
// either. A chunk is processed in rounds until every op has finished:
//   1. load: the cursor slab of every unfinished op is read, two ops per load instruction
//      (lanes 0..31 read op 2q's slab, lanes 32..63 op 2q+1's), all loads issued up front in one
//      straight run (a pair with no unfinished op reads slab 0; searches, after their first
//      round, read only the slabs of pairs still running).
//   2. decide: the ops are taken in lane order, a pair per step. The wavefront votes on each
//      slab for the op's key (and, for inserts, for empty slots). The op's slot is the slot
//      holding the key, else (inserts) the first empty slot, else slot 31, which holds the
//      next-slab index. On key-value slabs each op receives its half of the votes in its own
//      lane and decides there, fetching the one word it needs (the value at its key, or the
//      next index) from the slab lane that holds it; on key-only slabs the target lane writes
//      the outcome to the op's cell in LDS. The outcome: found (with the value), a swap to
//      record (insert into the empty slot, replace the key's value, tombstone the key; with the
//      observed value), move on to the next slab (with its index), end of list, or a new slab
//      needed.
//   3. each op acts on its outcome: searches finish or move; updates record their swap; the swaps
//      are issued together as one vector atomic. An insert that loses its empty slot learns the
//      slot's new occupant from the swap: the same key turns it into a replace of that slot,
//      another key sends it to the following slot at once. Slots fill in order, so this walk
//      sees every slot filled since the slab was read. Any other lost swap keeps its op and
//      cursor, and the next round re-reads that slab;
//   4. allocate: ops at a full tail slab are served one at a time: SlabAlloc gives a slab, lane 0
//      links it with a swap on the tail's next index (a lost link frees the slab and follows
//      the winner's), and the op's cursor moves to the linked slab.
// With kFlagCounters, per-wavefront counts of rounds, lost swaps, allocations, lost links and
// allocator block moves are added at the end to one of kCounterSlots header slots.

struct Counters {
    uint32_t rounds, cas_lost, allocs, link_lost;
};

// Outcome codes written by a target lane (bits 8.. of the message's high word; bits 0..7 hold
// the target slot).
enum : uint32_t { kMsgFound = 1, kMsgEnd = 2, kMsgMove = 3, kMsgGrow = 4, kMsgSwapIns = 5,
                  kMsgSwapRep = 6, kMsgSwapDel = 7 };

// Per-wavefront LDS: cursor slab index, key and op kind of each op, and each op's outcome cell.
struct WaveLds {
    uint64_t p[64]; // each op's cursor slab (its address)
    uint64_t msg[64];
    uint32_t key[64];
    uint32_t op[64];
    uint32_t claimed[64]; // slabs the round's bitmap claims won, in rotated lane order
};

// The inputs of one chunk, one op per lane (lanes past the chunk's end hold no op).
struct ChunkIn {
    uint32_t key, val, op;
};

template <int K, bool KO>
__device__ __forceinline__ ChunkIn load_chunk(const uint8_t *__restrict__ ops,
                                              const uint32_t *__restrict__ keys,
                                              const uint32_t *__restrict__ vals, uint64_t base,
                                              uint32_t count)
{
    const uint32_t lane = lane_id();
    const bool in = lane < count;
    ChunkIn c;
    c.key = in ? keys[base + lane] : kEmpty;
    c.val = 0;
    if constexpr ((K == kInsert || K == kMixed) && !KO)
        c.val = in ? vals[base + lane] : 0u;
    c.op = (uint32_t)K;
    if constexpr (K == kMixed)
        c.op = in ? (uint32_t)ops[base + lane] : 0u;
    return c;
}

// The decide step on key-value slabs. The wavefront votes on each pair's two slabs (one ballot
// of `slot == key`, and for updates one of `slot == empty`) and hands each op its half of the
// votes, in the op's own lane. Each op then decides alone. Slot 31 holds the auxiliary half (all
// ones) and the next index: it never matches a key, and it votes empty exactly when the slab has
// no next slab. pre[q] holds this lane's word of the slab of op 2q (lanes 0..31) or op 2q + 1
// (lanes 32..63); bits of `todo` name the ops still running (pairs with neither are skipped);
// L.key holds each op's key and `op` this lane's op kind. Returns this lane's outcome: (code << 8
// | slot) in the high word, the payload in the low word.
template <int K, bool Dup, int NQ>
__device__ __forceinline__ uint64_t decide_kv(const uint64_t (&pre)[NQ], uint64_t todo,
                                              const WaveLds &L, uint32_t op)
{
    constexpr bool kHasIns = (K == kInsert || K == kMixed);
    const uint32_t lane = lane_id();
    const uint32_t half = lane >> 5;
    uint32_t kmv = 0, emv = 0; // this lane's op: key votes, empty votes of its slab
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (!((todo >> (2 * q)) & 3ull))
            continue;
        const uint64_t w = pre[q];
        const uint32_t kq = L.key[2 * q + half];
        const uint64_t km = ballot((uint32_t)w == kq);
        kmv = wl(kmv, 2 * q, (uint32_t)km);
        kmv = wl(kmv, 2 * q + 1, (uint32_t)(km >> 32));
        if constexpr (kHasIns) {
            const uint64_t em = ballot(w == kEmptyPair);
            emv = wl(emv, 2 * q, (uint32_t)em);
            emv = wl(emv, 2 * q + 1, (uint32_t)(em >> 32));
        }
    }
    const bool ins = (K == kInsert) || (K == kMixed && op == (uint32_t)kInsert);
    // the op's slot is its key's first slot (with unique keys the only one); 31: absent
    const uint32_t kslot = (uint32_t)__builtin_ctz(kmv | 0x80000000u);
    // the first empty slot; 31: none, and no next slab; 32: none, and a next slab
    const uint32_t eslot = emv ? (uint32_t)__builtin_ctz(emv) : 32u;
    // with duplicates an insert takes the first empty slot whatever keys it meets
    const bool by_key = !(Dup && ins) && kslot < 31u;
    // the word of the slab the op needs: its key's value, else the next index
    const uint32_t src = ((lane & 1u) * 32u + (by_key ? kslot : 31u)) * 4u;
    // (unconditional, so that the fetches are issued back to back; pairs with no running op give
    // words that no op uses)
    uint32_t hv = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const uint32_t h = (uint32_t)__builtin_amdgcn_ds_bpermute(
            (int)src, (int)(uint32_t)(pre[q] >> 32));
        if (inverse_ballot(3ull << (2 * q)))
            hv = h;
    }
    uint32_t code, tslot = kslot, payload = hv;
    if (by_key) {
        code = (K == kSearch) ? kMsgFound : ((K == kDelete) ? kMsgSwapDel : kMsgSwapRep);
        if constexpr (K == kMixed)
            code = (op == (uint32_t)kSearch)
                       ? kMsgFound
                       : ((op == (uint32_t)kDelete) ? kMsgSwapDel : kMsgSwapRep);
    } else if (ins && eslot < 31u) {
        code = kMsgSwapIns;
        tslot = eslot;
        // with duplicates empty slots need not be a suffix: the op carries them all
        if constexpr (Dup)
            payload = emv & (uint32_t)kSlotMask;
    } else {
        code = hv != kEmpty ? kMsgMove : (ins ? kMsgGrow : kMsgEnd);
    }
    return ((uint64_t)((code << 8) | tslot) << 32) | payload;
}

// One chunk of up to 2 NQ ops (lane l < count holds op base + l, with inputs `c`) on table T,
// processed in rounds until every op has finished (see the description above). NQ is the
// number of op pairs, and so the length of each round's straight run of loads.
template <int K, bool Dup, bool KO, int NQ = 32>
__device__ void run_chunk(const View &T, Alloc &al, Counters &cnt, WaveLds &L, ChunkIn c,
                          uint32_t *__restrict__ vout, uint8_t *__restrict__ sout, uint64_t base,
                          uint32_t count, uint32_t flags)
{
    constexpr bool kCoherent = (K != kSearch);
    constexpr bool kHasIns = (K == kInsert || K == kMixed);
    // unique-key pair inserts write their pair into a new tail slab before linking it
    constexpr bool kPrefill = !Dup && !KO;
    const uint32_t lane = lane_id();
    const uint32_t half = lane >> 5, slot = lane & 31;
    const bool is31 = slot == 31;
    const uint32_t below = (1u << slot) - 1u; // slots of my half below mine
    const uint32_t hshift = lane & 32;
    const uint64_t i = base + lane;
    const bool in = lane < count;
    const uint32_t key = c.key, val = c.val, op = c.op;
    // key-only slabs reserve a second key, the deleted-entry marker
    const bool reserved = in && (key == kEmpty || (KO && key == kTombKey));
    const uint64_t res_m = ballot(reserved);
    if (res_m)
        raise_error(T, SH_ERR_RESERVED_KEY, lane, ffs0(res_m));
    const bool act = in && !reserved && op <= 2;
    const uint32_t bkt = act ? bucket_of(key, T.a, T.b, T.B) : 0u;
    L.key[lane] = key;
    if constexpr (K == kMixed && KO)
        L.op[lane] = op;

    uint32_t rv = kEmpty, rs = 0; // this lane's results
    uint32_t loc = kEmpty;        // this lane's cursor
    uint64_t todo = ballot(act);
    bool first_round = true;
    while (todo) {
        todo = uniform64(todo);
        ++cnt.rounds;
        // ---- 1. load ----
        L.p[lane] = reinterpret_cast<uint64_t>(((todo >> lane) & 1) ? cursor_slab(T, loc, bkt)
                                                                     : T.base);
        __builtin_amdgcn_wave_barrier();
        uint64_t pre[NQ];
        if (K != kSearch || first_round) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const uint64_t *sp = reinterpret_cast<const uint64_t *>(L.p[2 * q + half]);
                pre[q] = load_slot<kCoherent>(sp + slot);
            }
        } else {
            // a search's later rounds usually run a few ops: read only the slabs of pairs still
            // running
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                pre[q] = 0;
                if ((todo >> (2 * q)) & 3ull) {
                    const uint64_t *sp = reinterpret_cast<const uint64_t *>(L.p[2 * q + half]);
                    pre[q] = load_slot<kCoherent>(sp + slot);
                }
            }
        }
        first_round = false;
        // ---- 2. decide ----
        uint64_t outcome = 0;
        if constexpr (!KO) {
            outcome = decide_kv<K, Dup, NQ>(pre, todo, L, op);
        } else {
            // Key-only slabs (two entries per lane, entries 2 slot in lo and 2 slot + 1 in hi):
            // the target lane of each op writes the op's outcome to the op's LDS cell.
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (!((todo >> (2 * q)) & 3ull))
                    continue;
                const uint64_t w = pre[q];
                const uint32_t lo = (uint32_t)w;
                uint32_t hi = (uint32_t)(w >> 32);
                // keep `hi` a 32-bit register value, so tests on it stay 32-bit compares
                asm("" : "+v"(hi));
                const uint32_t kq = L.key[2 * q + half];
                // votes come straight from the compares (slot 31 holds the next index)
                const uint64_t mlo_m = ballot(lo == kq) & kSlotLanes;
                const uint64_t mhi_m = ballot(hi == kq) & kSlotLanes;
                const bool mlo = inverse_ballot(mlo_m);
                const bool mhi = inverse_ballot(mhi_m);
                const bool match = mlo || mhi;
                const uint32_t kh = (uint32_t)((mlo_m | mhi_m) >> hshift); // my half's key votes
                // the op's entry is the first match of the slab (with unique keys the only one)
                const bool is_key = Dup ? (match && (kh & below) == 0u) : match;
                const uint32_t kslot = mlo ? 2 * slot : 2 * slot + 1;
                bool ins = (K == kInsert);
                uint32_t code_key = (K == kSearch) ? kMsgFound
                                                   : ((K == kDelete) ? kMsgSwapDel : kMsgSwapRep);
                if constexpr (K == kMixed) {
                    const uint32_t oq = L.op[2 * q + half];
                    ins = oq == kInsert;
                    code_key = (oq == kSearch) ? kMsgFound
                                               : ((oq == kDelete) ? kMsgSwapDel : kMsgSwapRep);
                }
                bool target;
                uint32_t code, tslot = slot;
                uint32_t empties = 0;
                if constexpr (kHasIns) {
                    const uint64_t elo_m = ballot(lo == kEmpty) & kSlotLanes;
                    const uint64_t ehi_m = ballot(hi == kEmpty) & kSlotLanes;
                    const bool elo = inverse_ballot(elo_m);
                    const bool ehi = inverse_ballot(ehi_m);
                    const bool is_empty = elo || ehi;
                    const uint32_t eh = (uint32_t)((elo_m | ehi_m) >> hshift);
                    empties = eh;
                    const bool first_empty = ins && is_empty && (eh & below) == 0u;
                    const bool tail = is31 && (!ins || eh == 0u);
                    // with duplicates an insert takes the first empty entry whatever keys it
                    // meets
                    const bool hit = Dup ? (is_key && !ins) : is_key;
                    const uint32_t khe = (Dup && ins) ? 0u : kh;
                    target = hit || (khe == 0u && (first_empty || tail));
                    code = hit ? code_key
                               : (first_empty ? kMsgSwapIns
                                              : (hi != kEmpty ? kMsgMove
                                                              : (ins ? kMsgGrow : kMsgEnd)));
                    if (hit)
                        tslot = kslot;
                    else if (first_empty)
                        tslot = elo ? 2 * slot : 2 * slot + 1;
                } else {
                    target = is_key || (kh == 0u && is31);
                    code = is_key ? code_key : (hi != kEmpty ? kMsgMove : kMsgEnd);
                    if (is_key)
                        tslot = kslot;
                }
                // the payload: the key itself when found (a search reports it as the value),
                // the next index, or for an insert into an empty entry with duplicates, the
                // lanes of the slab that showed an empty entry (they need not be a suffix)
                const uint32_t payload =
                    (Dup && code == kMsgSwapIns) ? empties : (is_key ? kq : hi);
                if (target)
                    L.msg[2 * q + half] = ((uint64_t)((code << 8) | tslot) << 32) | payload;
            }
            __builtin_amdgcn_wave_barrier();
            outcome = L.msg[lane];
        }
        // ---- 3. act on the outcome ----
        const bool mine = (todo >> lane) & 1;
        const uint64_t msg = mine ? outcome : 0ull;
        const uint32_t payload = (uint32_t)msg;
        const uint32_t code = mine ? (uint32_t)(msg >> 40) : 0u;
        const uint32_t tslot = (uint32_t)(msg >> 32) & 255u;
        if (code == kMsgFound) {
            rv = payload;
            rs = 1;
        }
        if (code == kMsgMove)
            loc = payload;
        bool done = code == kMsgFound || code == kMsgEnd;
        uint64_t alloc_m = 0;
        uint32_t claim_m = 0, claim_old = 0; // bitmap bits this lane claims for new tails
        if constexpr (K != kSearch) {
            // An op at a full tail needs a new slab: it is claimed from the resident block now,
            // so the bitmap atomic is in flight together with the swaps. One op per round and
            // wavefront grows a list (the first in lane order); the others keep their cursor
            // and re-read their tail next round, where they usually find it linked. So a
            // wavefront never holds more than one slab it may have to give back, and slabs
            // held by links about to be lost cannot make a pool under heavy contention look
            // exhausted.
            alloc_m = ballot(code == kMsgGrow);
            alloc_m &= 0ull - alloc_m;
            if (alloc_m) {
                claim_m = claim_plan(al, lane, 1u);
                if (claim_m)
                    claim_old = or32(&al.row[lane], claim_m);
            }
            bool won = false, lost = false;
            if (KO && code >= kMsgSwapIns) {
                // key-only slab: 32-bit swaps on single entries
                uint32_t *ent = reinterpret_cast<uint32_t *>(cursor_slab(T, loc, bkt));
                uint32_t e = tslot;
                if (code == kMsgSwapRep) {
                    rs = 2u; // the key is already there: nothing to replace
                    won = true;
                } else if (code == kMsgSwapDel) {
                    won = cas32(ent + e, key, Dup ? kEmpty : kTombKey) == key;
                    rs = won ? 1u : 0u;
                    lost = !won;
                } else {
                    uint32_t old = cas32(ent + e, kEmpty, key);
                    if (old == kEmpty) {
                        rs = 1u;
                        won = true;
                    } else if (!Dup) {
                        // entries fill in order: walk on with the occupants the swaps return
                        for (;;) {
                            if (old == key) {
                                rs = 2u; // inserted meanwhile by another op
                                won = true;
                                break;
                            }
                            if (++e >= kKeyEntries) {
                                lost = true;
                                break;
                            }
                            old = cas32(ent + e, kEmpty, key);
                            if (old == kEmpty) {
                                rs = 1u;
                                won = true;
                                break;
                            }
                        }
                    } else {
                        // the rest of this lane, then the lanes that showed an empty entry
                        if (!(e & 1u) && cas32(ent + e + 1, kEmpty, key) == kEmpty) {
                            rs = 1u;
                            won = true;
                        }
                        uint32_t m = payload & ~((2u << (e >> 1)) - 1u);
                        while (!won && m) {
                            const uint32_t l = (uint32_t)__builtin_ctz(m);
                            m &= m - 1u;
                            if (cas32(ent + 2 * l, kEmpty, key) == kEmpty ||
                                cas32(ent + 2 * l + 1, kEmpty, key) == kEmpty) {
                                rs = 1u;
                                won = true;
                            }
                        }
                        lost = !won;
                    }
                }
            } else if (code >= kMsgSwapIns) {
                uint32_t cslot = tslot;
                uint64_t *slab = cursor_slab(T, loc, bkt);
                // a delete leaves a tombstone, or with duplicates an empty slot
                const uint64_t desired = (code == kMsgSwapDel)
                                             ? (Dup ? kEmptyPair : kTombPair)
                                             : (((uint64_t)val << 32) | key);
                uint64_t expect = (code == kMsgSwapIns) ? kEmptyPair
                                                        : (((uint64_t)payload << 32) | key);
                uint64_t old = cas64(slab + cslot, expect, desired);
                if (old == expect) {
                    rs = (code == kMsgSwapRep) ? 2u : 1u;
                    won = true;
                } else if (code == kMsgSwapIns && Dup) {
                    // try the empty slots after the lost one that the slab read showed
                    uint32_t m = payload & ~((2u << cslot) - 1u);
                    while (m) {
                        cslot = (uint32_t)__builtin_ctz(m);
                        m &= m - 1u;
                        if (cas64(slab + cslot, kEmptyPair, desired) == kEmptyPair) {
                            rs = 1u;
                            won = true;
                            break;
                        }
                    }
                    lost = !won; // all taken: the next round re-reads the slab
                } else if (code == kMsgSwapIns) {
                    // Walk forward from the lost empty slot using the occupants the swaps
                    // return; at most the 31 slots of this slab. (With duplicates, empty slots
                    // need not be a suffix, so a lost insert re-reads its slab next round.)
                    for (;;) {
                        if ((uint32_t)old == key) { // the same key was inserted: replace it
                            expect = old;
                            old = cas64(slab + cslot, expect, desired);
                            if (old == expect) {
                                rs = 2u;
                                won = true;
                            } else {
                                lost = true;
                            }
                            break;
                        }
                        if (++cslot >= 31) {
                            lost = true; // slab filled up: the next round follows `next`
                            break;
                        }
                        old = cas64(slab + cslot, kEmptyPair, desired);
                        if (old == kEmptyPair) {
                            rs = 1u;
                            won = true;
                            break;
                        }
                    }
                } else {
                    lost = true;
                }
            }
            done = done || won;
            if (flags & kFlagCounters)
                cnt.cas_lost += (uint32_t)__popcll(ballot(lost));
        }
        todo &= ~ballot(done);
        if constexpr (K != kSearch) {
            // ---- 4. allocate and link new tail slabs ----
            if (alloc_m) {
                // the slab claimed with the swaps, if the claim won its bit
                const uint32_t got_m = claim_m & ~claim_old;
                if (claim_m)
                    al.word = claim_old | claim_m;
                al.lost += (uint32_t)__popcll(ballot((claim_m & claim_old) != 0u));
                uint32_t served;
                uint32_t at = rotated_scan((uint32_t)__popc(got_m), lane, al.rot, &served);
                uint32_t *claimed = L.claimed;
                for (uint32_t w = got_m; w; w &= w - 1u)
                    claimed[at++] = al.code + lane * 32 + (uint32_t)__builtin_ctz(w);
                if (served)
                    al.moves = 0;
                __builtin_amdgcn_wave_barrier();
                const bool grows = (alloc_m >> lane) & 1;
                const uint32_t g = (uint32_t)__popcll(alloc_m & ((1ull << lane) - 1ull));
                uint32_t idx = (grows && g < served) ? claimed[g] : kEmpty;
                // if the claim could not serve it (the resident block's free bits were taken):
                // the allocator proper, moving on through the blocks
                uint64_t rest = alloc_m & ~ballot(idx != kEmpty);
                while (rest) {
                    const uint32_t j = ffs0(rest);
                    rest &= rest - 1;
                    const uint32_t x = wave_alloc(T, al, lane);
                    if (x == kEmpty) {
                        raise_error(T, SH_ERR_POOL_EXHAUSTED, lane, 0);
                        todo &= ~(1ull << j); // status stays 0
                        continue;
                    }
                    idx = wl(idx, j, x);
                }
                // The op links its slab: a swap of its tail's next index from empty to the new
                // slab. On unique-key pair tables the op's pair goes into slot 0 of the new slab
                // with a swap issued together with the link: a reader that follows the link
                // before the pair lands sees an empty slot, which is the state before the
                // insert, and if another insert fills slot 0 first this op takes the next round
                // on the new slab. A link lost to another wavefront leaves the new slab private,
                // so its pair went in; it is taken out again (a free slab must be empty) before
                // the slab is returned, and the op follows the winner's slab.
                const bool has = grows && idx != kEmpty;
                bool linked_done = false, link_lost = false;
                if (has) {
                    uint64_t *tail = cursor_slab(T, loc, bkt);
                    uint32_t *link = reinterpret_cast<uint32_t *>(tail + 31) + 1;
                    uint64_t *fresh = pool_slab(T, idx);
                    const uint64_t pair = ((uint64_t)val << 32) | key;
                    uint64_t put = 0;
                    if constexpr (kPrefill)
                        put = cas64(fresh, kEmptyPair, pair);
                    const uint32_t lold = cas32(link, kEmpty, idx);
                    if (lold == kEmpty) {
                        if (kPrefill && put == kEmptyPair) {
                            rs = 1u; // a new key, in slot 0 of the new tail
                            linked_done = true;
                        } else {
                            loc = idx;
                        }
                    } else {
                        link_lost = true;
                        uint32_t freed = idx;
                        if (kPrefill && put == kEmptyPair) {
                            const uint32_t back = cas64(fresh, pair, kEmptyPair) == pair;
                            asm volatile("" : "+v"(freed) : "v"(back));
                        }
                        slab_free(T, freed);
                        loc = lold;
                    }
                }
                if (flags & kFlagCounters) {
                    const uint64_t hm = ballot(has);
                    cnt.allocs += (uint32_t)__popcll(hm);
                    cnt.link_lost += (uint32_t)__popcll(ballot(link_lost));
                }
                todo &= ~ballot(linked_done);
            }
        }
        // Every load of this round has been consumed; saying so lets the compiler issue the
        // next round's loads back to back instead of waiting before each one.
        wait_vm_all();
    }

    if (in) {
        if (vout)
            vout[i] = rv;
        if (sout)
            sout[i] = (uint8_t)rs;
    }
}

__device__ __forceinline__ void flush_counters(const View &T, const Counters &cnt,
                                               const Alloc &al, uint32_t wave)
{
    if (lane_id() == 0) {
        auto cs = gmem(T.counters + (size_t)(wave % kCounterSlots) * 8);
        const unsigned long long add[6] = {cnt.rounds, cnt.cas_lost, cnt.allocs, cnt.link_lost,
                                           al.total_moves, al.lost};
#pragma unroll
        for (int f = 0; f < 6; ++f)
            __hip_atomic_fetch_add(cs + f, add[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void alloc_init(Alloc &al, uint32_t wave, uint32_t seq)
{
    al.blk = kEmpty;
    al.word = 0;
    al.row = nullptr;
    al.code = 0;
    al.nact = 0;
    al.moves = 0;
    al.total_moves = 0;
    al.lost = 0;
    al.full = false;
    al.start = mix32(wave * 0x9E3779B9u + seq);
    al.rot = mix32(al.start) & 63u;
}

template <int K, bool Dup, bool KO, int NQ>
__global__ __launch_bounds__(kBlock) void ops_kernel(View T, const uint8_t *__restrict__ ops,
                                                     const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ vals,
                                                     uint64_t n, uint32_t *__restrict__ vout,
                                                     uint8_t *__restrict__ sout, uint32_t seq,
                                                     uint32_t flags)
{
    constexpr uint32_t C = 2 * NQ; // ops per chunk, two per load of the straight run
    __shared__ WaveLds lds[kWavesPerBlock];
    const uint32_t wl_ = threadIdx.x >> 6;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + wl_;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Alloc al;
    alloc_init(al, wave, seq);
    if constexpr (K == kInsert || K == kMixed)
        alloc_preload(T, al, lane_id());
    Counters cnt = {0, 0, 0, 0};
    const uint64_t nchunks = (n + C - 1) / C;
    for (uint64_t c = wave; c < nchunks; c += nwaves) {
        const uint64_t base = c * C;
        const uint32_t count = (uint32_t)((n - base < C) ? n - base : C);
        const ChunkIn cur = load_chunk<K, KO>(ops, keys, vals, base, count);
        run_chunk<K, Dup, KO, NQ>(T, al, cnt, lds[wl_], cur, vout, sout, base, count, flags);
    }
    if (flags & kFlagCounters)
        flush_counters(T, cnt, al, wave);
}

// Batched form: many tables, one launch. d_desc[d] hands ops [offset, offset + length) of the
// shared op arrays (n_ops long) to table `table` (< T); descriptors naming another table are
// skipped and ranges are clipped to the arrays, so no descriptor makes the kernel read or write
// outside them. Each block turns the descriptors' chunk counts into an
// exclusive prefix sum in LDS; wavefront w then takes global chunks w, w + W, ... of the
// concatenated chunk space and finds each chunk's descriptor by binary search. Nothing is
// counted with atomics, so the launch can be captured in a graph and replayed as is.
template <int NQ>
__global__ __launch_bounds__(kBlock) void multi_kernel(const View *__restrict__ dir, uint32_t T,
                                                       const sh_batch_desc_t *__restrict__ desc,
                                                       uint32_t nb, uint64_t n_ops,
                                                       const uint8_t *__restrict__ ops,
                                                       const uint32_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ vals,
                                                       uint32_t *__restrict__ vout,
                                                       uint8_t *__restrict__ sout, uint32_t seq,
                                                       uint32_t flags)
{
    constexpr uint32_t C = 2 * NQ; // ops per chunk, two per load of the straight run
    __shared__ WaveLds lds[kWavesPerBlock];
    // chunk counts in 64 bits (up to 4096 descriptors of up to 2^32 - 1 ops each); pre[] holds
    // nb + 1 entries in the launch's dynamic LDS
    extern __shared__ uint64_t pre[];
    __shared__ uint64_t part[kBlock];
    const uint32_t tid = threadIdx.x;
    // exclusive prefix of chunk counts: each thread sums a contiguous segment, then the
    // segment sums are scanned across the block
    const uint32_t seg = (nb + kBlock - 1) / kBlock;
    const uint32_t s0 = tid * seg, s1 = (s0 + seg < nb) ? s0 + seg : nb;
    uint64_t local = 0;
    for (uint32_t d = s0; d < s1; ++d)
        local += ((uint64_t)desc[d].length + C - 1) / C;
    part[tid] = local;
    __syncthreads();
    for (uint32_t off = 1; off < kBlock; off <<= 1) {
        const uint64_t v = (tid >= off) ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - local; // exclusive start of this thread's segment
    for (uint32_t d = s0; d < s1; ++d) {
        pre[d] = run;
        run += ((uint64_t)desc[d].length + C - 1) / C;
    }
    if (tid == kBlock - 1)
        pre[nb] = part[kBlock - 1];
    __syncthreads();

    const uint32_t wl_ = tid >> 6;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + wl_;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    const uint64_t total = pre[nb];
    Alloc al;
    alloc_init(al, wave, seq);
    Counters cnt = {0, 0, 0, 0};
    uint32_t cur_t = kEmpty;
    for (uint64_t c = wave; c < total; c += nwaves) {
        // largest d with pre[d] <= c (descriptors with no ops have pre[d] == pre[d + 1])
        uint32_t lo = 0, hi = nb;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pre[mid] <= c)
                lo = mid;
            else
                hi = mid;
        }
        const sh_batch_desc_t dd = desc[lo];
        if (dd.table >= T)
            continue; // no such table: the batch is skipped
        if (dd.table != cur_t) {
            if ((flags & kFlagCounters) && cur_t != kEmpty) {
                flush_counters(dir[cur_t], cnt, al, wave);
                cnt = Counters{0, 0, 0, 0};
            }
            alloc_init(al, wave, seq); // another table: another pool
            cur_t = dd.table;
        }
        const View Tv = dir[cur_t];
        alloc_preload(Tv, al, lane_id()); // once per table switch
        // first < dd.length: chunk c is one of this descriptor's
        const uint64_t first = (c - pre[lo]) * C;
        uint64_t base = 0, count = 0; // a range outside the op arrays reads and writes nothing
        if (dd.offset < n_ops && first < n_ops - dd.offset) {
            base = dd.offset + first;
            count = (dd.length - first < C) ? dd.length - first : C;
            if (count > n_ops - base)
                count = n_ops - base;
        }
        run_chunk<kMixed, false, false, NQ>(
            Tv, al, cnt, lds[wl_],
            load_chunk<kMixed, false>(ops, keys, vals, base, (uint32_t)count), vout, sout, base,
            (uint32_t)count, flags);
    }
    if ((flags & kFlagCounters) && cur_t != kEmpty)
        flush_counters(dir[cur_t], cnt, al, wave);
}

// ---------------------------------------------------------------------------------------------
// Structure walk: one wavefront per bucket (grid-stride). Counts live, deleted and slabs per
// bucket, checks the invariants the insertion rule guarantees, optionally emits live pairs.

__device__ __forceinline__ bool bitmap_has(const View &T, uint32_t idx)
{
    return (*bitmap_word(T, idx) >> (idx & 31)) & 1u;
}

template <bool KO>
__global__ __launch_bounds__(kBlock) void walk_kernel(View T, uint32_t *__restrict__ dbkt,
                                                      uint32_t *__restrict__ dkey,
                                                      uint32_t *__restrict__ dval, uint64_t cap,
                                                      uint32_t *__restrict__ counts, int emit)
{
    const bool dup = (T.mode & SH_TABLE_DUPLICATES) != 0;
    const uint32_t lane = lane_id();
    const uint32_t slot = lane & 31;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    unsigned long long live_t = 0, tomb_t = 0, slabs_t = 0;
    uint32_t viol = 0;
    for (uint32_t b = wave; b < T.B; b += nwaves) {
        const uint64_t *cur = T.base + (size_t)b * 32;
        uint32_t nl = 0, nt = 0, ns = 0;
        for (;;) {
            const uint64_t w = cur[slot];
            const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
            ++ns;
            uint64_t E, L;
            if constexpr (KO) {
                // two entries per lane (2 slot in lo, 2 slot + 1 in hi); lane 31: aux and next
                const bool s31 = slot == 31;
                const bool elo = !s31 && lo == kEmpty, ehi = !s31 && hi == kEmpty;
                const uint64_t Llo = ballot(!s31 && lo != kEmpty && lo != kTombKey) & kSlotMask;
                const uint64_t Lhi = ballot(!s31 && hi != kEmpty && hi != kTombKey) & kSlotMask;
                nl += __popcll(Llo) + __popcll(Lhi);
                nt += __popcll(ballot(!s31 && lo == kTombKey) & kSlotMask) +
                      __popcll(ballot(!s31 && hi == kTombKey) & kSlotMask);
                const uint64_t Eall = ballot(elo && ehi) & kSlotMask;
                const uint64_t Ehi = ballot(!elo && ehi) & kSlotMask;
                const uint64_t Ebad = ballot(elo && !ehi) & kSlotMask;
                E = Eall | Ehi | Ebad;
                L = Llo | Lhi;
                if (!dup) {
                    // empty entries form a suffix: full lanes, at most one lane with only its
                    // high entry empty, then empty lanes
                    const uint64_t full = kSlotMask & ~E;
                    const uint32_t nf = (uint32_t)__popcll(full);
                    if (Ebad || full != (1ull << nf) - 1 || (Ehi && Ehi != (1ull << nf)))
                        ++viol;
                }
                if (emit && L) {
                    unsigned long long pos0 = 0;
                    const uint32_t ne = (uint32_t)(__popcll(Llo) + __popcll(Lhi));
                    if (lane == 0)
                        pos0 = atomicAdd(&T.hdr->dump_count, (unsigned long long)ne);
                    pos0 = ((unsigned long long)rl((uint32_t)(pos0 >> 32), 0) << 32) |
                           rl((uint32_t)pos0, 0);
                    if (lane < 32) {
                        const uint64_t lb = (1ull << lane) - 1;
                        const bool ilo = (Llo >> lane) & 1, ihi = (Lhi >> lane) & 1;
                        const uint64_t p =
                            pos0 + __popcll(Llo & lb) + __popcll(Lhi & lb);
                        if (ilo && p < cap) {
                            dbkt[p] = b;
                            dkey[p] = lo;
                            dval[p] = lo;
                        }
                        if (ihi && p + ilo < cap) {
                            dbkt[p + ilo] = b;
                            dkey[p + ilo] = hi;
                            dval[p + ilo] = hi;
                        }
                    }
                }
            } else {
                E = ballot(w == kEmptyPair) & kSlotMask;
                L = ballot(lo != kEmpty) & kSlotMask;
                const uint64_t Tm = ballot(w == kTombPair) & kSlotMask;
                const uint64_t bad =
                    ballot(lo == kEmpty && hi != kEmpty && hi != 0u) & kSlotMask;
                nl += __popcll(L);
                nt += __popcll(Tm);
                if (bad)
                    ++viol;
                if (!dup && E && E != (kSlotMask & ~((1ull << ffs0(E)) - 1)))
                    ++viol; // empty slots must form a suffix (with unique keys)
            }
            const uint32_t aux = rl(lo, 31), next = rl(hi, 31);
            if (aux != kEmpty)
                ++viol;
            if (!KO && emit && L) {
                unsigned long long pos0 = 0;
                if (lane == 0)
                    pos0 = atomicAdd(&T.hdr->dump_count, (unsigned long long)__popcll(L));
                pos0 = ((unsigned long long)rl((uint32_t)(pos0 >> 32), 0) << 32) |
                       rl((uint32_t)pos0, 0);
                if (lane < 32 && ((L >> lane) & 1)) {
                    const uint64_t pos = pos0 + __popcll(L & ((1ull << lane) - 1));
                    if (pos < cap) {
                        dbkt[pos] = b;
                        dkey[pos] = lo;
                        dval[pos] = hi;
                    }
                }
            }
            if (next == kEmpty)
                break;
            if (E && !dup)
                ++viol; // a slab with a successor must be full (with unique keys)
            if (!pool_in_range(T, next) || !bitmap_has(T, next) ||
                ns > T.total_blocks * SH_BLOCK_SLABS) {
                ++viol;
                break;
            }
            cur = pool_slab(T, next);
        }
        if (counts && lane == 0) {
            counts[(size_t)3 * b] = nl;
            counts[(size_t)3 * b + 1] = nt;
            counts[(size_t)3 * b + 2] = ns;
        }
        live_t += nl;
        tomb_t += nt;
        slabs_t += ns;
    }
    if (lane == 0) {
        atomicAdd(&T.hdr->live, live_t);
        atomicAdd(&T.hdr->tomb, tomb_t);
        atomicAdd(&T.hdr->slabs, slabs_t);
        if (viol)
            atomicAdd(&T.hdr->violations, viol);
    }
}

// FLUSH ("Flush" subsection): each half-wavefront takes one bucket of [first, first + count)
// (lanes 0..31 bucket 2p, lanes 32..63 bucket 2p + 1, p grid-stride), so a wavefront walks two
// lists at once. A half walks its bucket's list head to tail and moves its live pairs, in the order it
// meets them, to the front of the list. The slab that receives the last live pair (the base
// slab if there is none) becomes the tail: its remaining slots are emptied and its next index
// cleared. The slabs after it are reset to all ones, so a later allocation finds them empty, and
// returned to the allocator. The write position never passes the end of the slab being read
// (a slab holds at most 31 live pairs), so every slab is read before anything is written into
// it; the next index of a slab is never written before the walk has passed it. This is a kernel
// of its own: no operation touches the table while it runs. A next index outside the pool (a
// well-formed table has none; the structure walk of sh_stats reports one) leaves the rest of
// that bucket as it is.
template <bool KO>
__global__ __launch_bounds__(kBlock) void flush_kernel(View T, uint32_t first, uint32_t count)
{
    // slots per slab: 31 pairs, or 62 keys of a key-only slab (entries 2 slot and 2 slot + 1)
    constexpr uint32_t kCap = KO ? kKeyEntries : 31u;
    const uint32_t lane = lane_id();
    const uint32_t slot = lane & 31;
    const uint32_t half = lane >> 5, hshift = lane & 32;
    const uint32_t below = (1u << slot) - 1u;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    // slot 31 of this half's slab (its next index lives in the high word)
    auto last_of_half = [&](uint32_t v) { return half ? rl(v, 63) : rl(v, 31); };
    for (uint32_t p = wave; (uint64_t)2 * p < count; p += nwaves) {
        const uint32_t i = 2 * p + half;
        if (i >= count)
            continue; // an odd count leaves the last wavefront's upper half idle
        const uint32_t bkt = first + i;
        uint64_t *rp = T.base + (size_t)bkt * 32; // the slab being read
        uint64_t *wp = rp;                        // write position: slot ws of slab wp
        uint32_t ws = 0, seen = 0, nxt = kEmpty;
        const uint32_t limit = T.total_blocks * SH_BLOCK_SLABS;
        uint64_t w = 0;
        bool ok = true;
        for (;;) {
            w = rp[slot];
            nxt = last_of_half((uint32_t)(w >> 32));
            const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
            const bool live = slot < 31 && lo != kEmpty && (!KO || lo != kTombKey);
            const bool live_hi = KO && slot < 31 && hi != kEmpty && hi != kTombKey;
            const uint32_t lm = (uint32_t)(ballot(live) >> hshift); // this half's slots
            const uint32_t hm = (uint32_t)(ballot(live_hi) >> hshift);
            const uint32_t cnt = (uint32_t)(__popc(lm) + __popc(hm));
            if (cnt) {
                // entries past the last slot of wp go to the slab after it, which the walk has
                // passed
                uint64_t *sp = wp;
                if (ws + cnt > kCap) {
                    const uint32_t spill = (uint32_t)(wp[31] >> 32);
                    if (!pool_in_range(T, spill)) {
                        ok = false;
                        break;
                    }
                    sp = pool_slab(T, spill);
                }
                const uint32_t pos = ws + (uint32_t)(__popc(lm & below) + __popc(hm & below));
                uint64_t *dp = (pos < kCap) ? wp : sp;
                const uint32_t ds = (pos < kCap) ? pos : pos - kCap;
                if constexpr (KO) {
                    const uint32_t pos2 = pos + (live ? 1u : 0u); // the high entry's position
                    uint64_t *dp2 = (pos2 < kCap) ? wp : sp;
                    const uint32_t ds2 = (pos2 < kCap) ? pos2 : pos2 - kCap;
                    if (live && (dp != rp || ds != 2 * slot)) // entries in place stay
                        reinterpret_cast<uint32_t *>(dp)[ds] = lo;
                    if (live_hi && (dp2 != rp || ds2 != 2 * slot + 1))
                        reinterpret_cast<uint32_t *>(dp2)[ds2] = hi;
                } else {
                    if (live && (dp != rp || ds != slot)) // pairs in place stay
                        dp[ds] = w;
                }
                if (ws + cnt > kCap) {
                    wp = sp;
                    ws = ws + cnt - kCap;
                } else {
                    ws += cnt;
                }
            }
            if (nxt == kEmpty)
                break;
            if (!pool_in_range(T, nxt) || ++seen > limit) {
                ok = false;
                break;
            }
            rp = pool_slab(T, nxt);
        }
        if (!ok)
            continue;
        // the tail: its old next index (already in hand if the tail is the last slab read),
        // then its slots after the write position are emptied and its next index cleared (word
        // 31 becomes all ones: auxiliary half and "no next"); words already so are not written
        uint32_t rest = nxt;
        if (wp != rp)
            rest = last_of_half((uint32_t)(wp[slot] >> 32));
        // the last slab read still holds its own words in w; an earlier tail is rewritten whole
        if constexpr (KO) {
            uint32_t *ent = reinterpret_cast<uint32_t *>(wp);
            const bool same = wp == rp;
            if (2 * slot >= ws && !(same && (uint32_t)w == kEmpty))
                ent[2 * slot] = kEmpty;
            if (2 * slot + 1 >= ws && !(same && (uint32_t)(w >> 32) == kEmpty))
                ent[2 * slot + 1] = kEmpty;
        } else {
            const bool keep = wp == rp && w == kEmptyPair;
            if (slot >= ws && !keep)
                wp[slot] = kEmptyPair;
        }
        // the slabs that followed the tail go back to the pool, emptied
        uint32_t f = rest;
        seen = 0;
        while (f != kEmpty) {
            if (!pool_in_range(T, f) || ++seen > limit)
                break;
            uint64_t *fp = pool_slab(T, f);
            const uint32_t nf = last_of_half((uint32_t)(fp[slot] >> 32));
            fp[slot] = kEmptyPair;
            if (slot == 0)
                slab_free(T, f);
            f = nf;
        }
    }
}

// SEARCHALL and DELETEALL ("Supported Operations"): every live element with the key, in list
// order, so each op walks its whole list. A wavefront holds a chunk of up to 2 NQ ops, reads
// their base slabs in one straight run of NQ loads (two ops per load, as in run_chunk), then takes the ops
// a pair at a time: lanes 0..31 walk op 2q's list and lanes 32..63 op 2q+1's, each slab voted
// on at once. SEARCHALL writes the values of the matching slots in list order from
// offsets[op], never past `limit` of the op (the next op's offset, or the output's capacity);
// DELETEALL swaps each matching slot to `gone` (a tombstone, or an empty slot with duplicates),
// retrying a slot whose value a concurrent replace changed. counts[op] receives the number of
// matches found (SEARCHALL) or deleted (DELETEALL).
template <bool Del, bool KO, int NQ>
__global__ __launch_bounds__(kBlock) void all_kernel(View T, const uint32_t *__restrict__ keys,
                                                     uint64_t n, uint32_t *__restrict__ counts,
                                                     const uint64_t *__restrict__ offsets,
                                                     uint32_t *__restrict__ vout,
                                                     uint64_t vcap, uint64_t gone)
{
    __shared__ uint32_t ku[kWavesPerBlock][2][64];
    const uint32_t lane = lane_id();
    const uint32_t half = lane >> 5, slot = lane & 31;
    const uint32_t below = (1u << slot) - 1u;
    const uint32_t wl_ = threadIdx.x >> 6;
    const uint64_t wave = blockIdx.x * (uint64_t)kWavesPerBlock + wl_;
    const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
    constexpr uint32_t C = 2 * NQ; // ops per chunk, two per load
    const uint64_t nchunks = (n + C - 1) / C;
    uint32_t *kk = ku[wl_][0], *uu = ku[wl_][1];
    for (uint64_t c = wave; c < nchunks; c += nwaves) {
        const uint64_t base = c * C;
        const uint32_t count = (n - base < C) ? (uint32_t)(n - base) : C;
        const bool in = lane < count;
        const uint32_t key = in ? keys[base + lane] : kEmpty;
        const uint64_t res_m = ballot(in && (key == kEmpty || (KO && key == kTombKey)));
        if (res_m)
            raise_error(T, SH_ERR_RESERVED_KEY, lane, ffs0(res_m));
        kk[lane] = key;
        uu[lane] = (in && key != kEmpty && !(KO && key == kTombKey))
                       ? bucket_of(key, T.a, T.b, T.B)
                       : 0u;
        // each op's output range, read once per chunk by the op's own lane (the pairs below
        // take theirs from that lane)
        uint64_t my_out0 = 0, my_lim = 0;
        if (!Del && vout && in) {
            my_out0 = offsets[base + lane];
            my_lim = (base + lane + 1 < n) ? offsets[base + lane + 1] : vcap;
        }
        __builtin_amdgcn_wave_barrier();
        uint64_t pre[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            pre[q] = load_slot<Del>(T.base + (size_t)uu[2 * q + half] * 32 + slot);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (2 * (uint32_t)q >= count)
                break;
            const uint32_t op = 2 * q + half;
            const uint32_t kq = kk[op];
            bool go = op < count && kq != kEmpty && !(KO && kq == kTombKey);
            uint64_t lim = 0, out0 = 0;
            if (!Del && vout) {
                const uint32_t lo0 = (uint32_t)__shfl((int)(uint32_t)my_out0, (int)op, 64);
                const uint32_t hi0 = (uint32_t)__shfl((int)(uint32_t)(my_out0 >> 32), (int)op, 64);
                const uint32_t lo1 = (uint32_t)__shfl((int)(uint32_t)my_lim, (int)op, 64);
                const uint32_t hi1 = (uint32_t)__shfl((int)(uint32_t)(my_lim >> 32), (int)op, 64);
                out0 = ((uint64_t)hi0 << 32) | lo0;
                lim = ((uint64_t)hi1 << 32) | lo1;
            }
            uint64_t w = pre[q];
            uint64_t *up = T.base + (size_t)uu[op] * 32; // the slab being read
            uint32_t found = 0, steps = 0;
            const uint32_t limit = T.total_blocks * SH_BLOCK_SLABS;
            for (;;) {
                const bool m = go && slot < 31 && (uint32_t)w == kq;
                const bool m2 = KO && go && slot < 31 && (uint32_t)(w >> 32) == kq;
                const uint32_t mm = (uint32_t)(ballot(m) >> (lane & 32u));
                const uint32_t mm2 = (uint32_t)(ballot(m2) >> (lane & 32u));
                uint32_t hits = (uint32_t)(__popc(mm) + __popc(mm2));
                if constexpr (Del) {
                    bool ok = false, ok2 = false;
                    if constexpr (KO) {
                        // key-only entries: the key is the whole entry, so one swap decides
                        uint32_t *e = reinterpret_cast<uint32_t *>(up) + 2 * slot;
                        if (m)
                            ok = cas32(e, kq, (uint32_t)gone) == kq;
                        if (m2)
                            ok2 = cas32(e + 1, kq, (uint32_t)gone) == kq;
                    } else if (m) {
                        uint64_t *p = up + slot;
                        uint64_t expect = w;
                        for (;;) {
                            const uint64_t old = cas64(p, expect, gone);
                            if (old == expect) {
                                ok = true;
                                break;
                            }
                            if ((uint32_t)old != kq)
                                break; // deleted by someone else meanwhile
                            expect = old; // a replace changed the value: delete that
                        }
                    }
                    hits = (uint32_t)(__popc((uint32_t)(ballot(ok) >> (lane & 32u))) +
                                      __popc((uint32_t)(ballot(ok2) >> (lane & 32u))));
                } else {
                    if ((m || m2) && vout) {
                        // in list order: entry 2 slot before 2 slot + 1, lanes in order
                        const uint64_t at = out0 + found + (uint32_t)__popc(mm & below) +
                                            (uint32_t)__popc(mm2 & below);
                        if (m && at < lim && at < vcap)
                            vout[at] = KO ? kq : (uint32_t)(w >> 32);
                        const uint64_t at2 = at + (m ? 1u : 0u);
                        if (m2 && at2 < lim && at2 < vcap)
                            vout[at2] = kq;
                    }
                }
                found += hits;
                const uint32_t nx = (uint32_t)__shfl((int)(uint32_t)(w >> 32),
                                                     (int)((lane & 32u) | 31u), 64);
                go = go && nx != kEmpty && pool_in_range(T, nx) && ++steps <= limit;
                if (!ballot(go))
                    break;
                if (go) {
                    up = pool_slab(T, nx);
                    w = load_slot<Del>(up + slot);
                }
            }
            if (slot == 0 && op < count && counts)
                counts[base + op] = found;
        }
    }
}

// SlabAlloc on its own ("Dynamic memory allocation"): requests 64 w .. 64 w + 63 of n belong to
// wavefront w, which serves them together (wave_alloc_many) from its resident block. The
// wavefronts partition the pool: wavefront w starts in block (w / 32) mod (blocks) at bitmap
// word 2 (w mod 32), the 64 slabs its requests need when every slab is free, so wavefronts
// sharing a block claim disjoint words and only a pool that is partly in use makes them hunt.
// out[i] receives a pool index, or kEmpty once the pool is exhausted.
__global__ __launch_bounds__(kBlock) void alloc_kernel(View T, uint64_t n,
                                                       uint32_t *__restrict__ out, uint32_t seq,
                                                       uint32_t flags)
{
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t i0 = wave * 64;
    if (i0 >= n)
        return; // the whole wavefront
    const uint32_t cnt = (n - i0 < 64) ? (uint32_t)(n - i0) : 64u;
    Alloc al;
    alloc_init(al, (uint32_t)wave, seq);
    al.start = (uint32_t)(wave / 32); // taken modulo the blocks in use
    al.rot = (uint32_t)(wave % 32) * 2u;
    const uint32_t got = wave_alloc_many(T, al, lane, cnt, out + i0);
    if (got < cnt) {
        raise_error(T, SH_ERR_POOL_EXHAUSTED, lane, 0);
        if (lane >= got && lane < cnt)
            out[i0 + lane] = kEmpty;
    }
    if (flags & kFlagCounters)
        flush_counters(T, Counters{0, 0, got, 0}, al, (uint32_t)wave);
}

// Deallocation: unset each slab's bit in its block's bitmap; entries outside the pool are skipped.
// The OR of x over the lanes of the wavefront.
__device__ __forceinline__ uint32_t wave_or(uint32_t x)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
        x |= (uint32_t)__shfl_xor((int)x, d, 64);
    return x;
}

// Frees 64 entries per wavefront at a time. Entries that name one bitmap word (slabs handed out
// together sit in few words) are cleared with one atomic AND by the first of them: up to four
// such groups per 64 entries, then whatever is left with one AND per entry, so entries spread
// over many words cost no more than before.
__global__ __launch_bounds__(kBlock) void free_kernel(View T, const uint32_t *__restrict__ idx,
                                                      uint64_t n)
{
    const uint32_t lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    for (uint64_t base = wave * 64; base < n; base += nwaves * 64) {
        const uint64_t i = base + lane;
        const uint32_t f = i < n ? idx[i] : kEmpty;
        bool mine = i < n && pool_in_range(T, f);
        uint32_t *w = mine ? bitmap_word(T, f) : nullptr;
        const uint32_t bit = 1u << (f & 31);
        uint64_t todo = ballot(mine);
        for (int g = 0; g < 4 && todo; ++g) {
            const uint32_t lead = ffs0(todo);
            const uint64_t wa = reinterpret_cast<uint64_t>(w);
            const uint64_t wl = ((uint64_t)rl((uint32_t)(wa >> 32), lead) << 32) |
                                rl((uint32_t)wa, lead);
            const bool same = mine && wa == wl;
            const uint32_t m = wave_or(same ? bit : 0u);
            if (lane == lead)
                __hip_atomic_fetch_and(gmem(w), ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            todo &= ~ballot(same);
            mine = mine && !same;
        }
        if (mine)
            __hip_atomic_fetch_and(gmem(w), ~bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Set bits of the bitmap rows of every registered super block (words numbered over all of
// them, allocator block order).
__global__ __launch_bounds__(kBlock) void popcount_kernel(View T)
{
    const size_t nw = (size_t)T.total_blocks * 64;
    unsigned long long c = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nw;
         i += (size_t)gridDim.x * kBlock) {
        uint32_t *row;
        uint32_t code;
        block_ref(T, (uint32_t)(i >> 6), row, code);
        c += __popc(row[i & 63]);
    }
    // wave reduction via ballot-free shuffle-down
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_down(c, off, 64);
    if (lane_id() == 0 && c)
        atomicAdd(&T.hdr->pool_alloc, c);
}

__global__ void clear_stats_kernel(View T, uint64_t *d_count, uint32_t *d_viol)
{
    if (threadIdx.x == 0) {
        T.hdr->violations = 0;
        T.hdr->live = T.hdr->tomb = T.hdr->slabs = T.hdr->pool_alloc = T.hdr->dump_count = 0;
    }
    (void)d_count;
    (void)d_viol;
}

__global__ void publish_dump_kernel(View T, uint64_t *d_count, uint32_t *d_viol)
{
    if (threadIdx.x == 0) {
        if (d_count)
            *d_count = T.hdr->dump_count;
        if (d_viol)
            *d_viol = T.hdr->violations;
    }
}

// Initialisation: header zero, base and pool slabs all ones (empty slots, empty next, aux all
// ones), bitmaps zero. 16-byte stores, grid-stride.
__global__ __launch_bounds__(kBlock) void init_kernel(uint4 *store, size_t hdr16, size_t ones16,
                                                      size_t zeros16)
{
    const size_t total = hdr16 + ones16 + zeros16;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const uint32_t f = (i >= hdr16 && i < hdr16 + ones16) ? kEmpty : 0u;
        store[i] = make_uint4(f, f, f, f);
    }
}

// Registration of super block sb: its directory entry in the table header.
__global__ void set_super_kernel(SuperDesc *dir, uint32_t sb, uint64_t *pool, uint32_t *bitmap,
                                 uint32_t slabs, uint32_t first)
{
    if (threadIdx.x == 0)
        dir[sb] = SuperDesc{pool, bitmap, slabs, first};
}

// Re-initialisation of a table in use. A free pool slab is always all ones: allocation hands
// slabs out untouched, a lost link takes its pair out again before returning its slab, FLUSH
// empties the slabs it frees, and slabs given back through sh_free_slabs must be empty. So the
// storage comes back to what the full initialisation writes by clearing the header (all but the
// super-block directory, which stays registered), filling the base slabs with ones, and filling
// only the pool slabs the bitmaps mark allocated, in every super block, before zeroing the
// bitmaps. Blocks [fill start, grid end) do the header and base slabs (16-byte stores,
// grid-stride over them); the others take one bitmap row (2048 pool slabs) per wavefront,
// grid-stride over the rows of all super blocks.
// The bitmap walkers take the first blocks, so they are dispatched before the fill blocks
// occupy the CUs; their dependent bitmap loads then overlap the fill instead of trailing it.
__global__ __launch_bounds__(kBlock) void reset_kernel(View T, uint4 *store, size_t hdr16,
                                                       size_t base16, uint32_t pool_blocks)
{
    if (blockIdx.x >= pool_blocks) {
        const size_t total = hdr16 + base16;
        const uint32_t fill_blocks = gridDim.x - pool_blocks;
        constexpr size_t kDir16 = kDirOffset / 16, kDirEnd16 = kGrownOffset / 16;
        for (size_t i = (size_t)(blockIdx.x - pool_blocks) * kBlock + threadIdx.x; i < total;
             i += (size_t)fill_blocks * kBlock) {
            if (i >= kDir16 && i < kDirEnd16)
                continue; // the super-block directory stays
            const uint32_t f = i >= hdr16 ? kEmpty : 0u;
            store[i] = make_uint4(f, f, f, f);
        }
        return;
    }
    const uint32_t lane = lane_id();
    const uint32_t wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const uint32_t nwaves = pool_blocks * kWavesPerBlock;
    // allocator blocks of every registered super block
    for (uint32_t r = wave; r < T.total_blocks; r += nwaves) {
        uint32_t *row, code;
        block_ref(T, r, row, code);
        uint32_t word = row[lane]; // slabs code + 32 lane + bit
        // the wavefront writes each allocated slab whole: 64 lanes x 4 bytes
        for (uint64_t m = ballot(word != 0); m; m = ballot(word != 0)) {
            const uint32_t j = ffs0(m);
            const uint32_t bit = (uint32_t)__builtin_ctz(rl(word, j));
            uint32_t *sl = reinterpret_cast<uint32_t *>(pool_slab(T, code + j * 32 + bit));
            sl[lane] = kEmpty;
            if (lane == j)
                word &= word - 1u; // that slab is done
        }
        row[lane] = 0u;
    }
}

} // namespace

// ---------------------------------------------------------------------------------------------
// Host side

struct sh_table {
    sh_params_t p;
    char *storage;
    size_t bytes;
    View v;
    uint32_t seq;
    uint32_t waves_per_cu; // 0 = the operation kind's default
    uint32_t ops_per_wave; // 0 = chosen per call
    uint32_t flags;        // SH_LAUNCH_* bits
    int num_cu;
    int embedded; // owned by a multi-table object
    struct sh_multi *owner; // that object, and this table's index in it
    uint32_t index;
    uint64_t super_slabs; // slabs of the super blocks registered beyond super block 0
};

struct sh_multi {
    uint32_t T;
    sh_table *tables; // T embedded table handles
    View *h_dir;      // host copy of the device directory
    View *d_dir;
    char *storage;
    size_t bytes;
    uint32_t seq, waves_per_cu, ops_per_wave, flags;
    int num_cu;
};

struct sh_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

struct Layout {
    size_t base, pool, bitmap, total;
};

bool layout_of(const sh_params_t *p, Layout *L)
{
    if (!p || p->num_buckets == 0 || p->pool_slabs % SH_BLOCK_SLABS != 0 ||
        p->pool_slabs > kMaxSuperSlabs || p->hash_a == 0 ||
        p->hash_a >= kPrime || p->hash_b >= kPrime ||
        (uint64_t)p->num_buckets + p->pool_slabs >= 0xFFFFFFFFull ||
        (p->flags & ~(uint32_t)(SH_TABLE_DUPLICATES | SH_TABLE_KEYS_ONLY)) != 0)
        return false;
    L->base = kHeaderBytes;
    L->pool = L->base + (size_t)p->num_buckets * SH_SLAB_BYTES;
    L->bitmap = L->pool + (size_t)p->pool_slabs * SH_SLAB_BYTES;
    L->total = L->bitmap + (size_t)(p->pool_slabs / SH_BLOCK_SLABS) * 256;
    return true;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

sh_status_t check_launch()
{
    return hipGetLastError() == hipSuccess ? SH_OK : SH_EHIP;
}

// Default launch shape of an operation kind: wavefronts per compute unit and the largest chunk
// (ops per wavefront). A persistent grid should not exceed the wavefronts that fit at once at
// the kernel's register use, or the ones that do not fit run after the others (launch_wpc
// lowers a default grid to what fits). The straight run of loads follows the chunk: on
// unique-key pair tables inserts and deletes at 16 ops per wavefront use 78 VGPRs (24
// wavefronts fit per CU) and ran fastest at 20 per CU (2^22-pair build 254 us against 330 us
// at 64 ops and 16 per CU); searches ran fastest at 32 ops, 16 per CU (72 VGPRs). Tables with
// flags (duplicates, key-only slabs) take the same shapes.
struct Shape {
    uint32_t waves_per_cu, max_ops;
};

Shape default_shape(const sh_table *, int kind)
{
    switch (kind) {
    case kSearch:
        return {16, 32};
    case kInsert:
    case kDelete:
        return {20, 16};
    default:
        return {kDefaultWavesPerCU, 64};
    }
}

uint32_t waves_per_cu_for(const sh_table *t, int kind)
{
    return t->waves_per_cu ? t->waves_per_cu : default_shape(t, kind).waves_per_cu;
}

// Ops per wavefront: the kind's largest chunk, halved (down to 8) while the batch's chunks would
// not fill the persistent grid, so small batches spread over the chip; a wavefront's straight
// run of loads shrinks with its chunk (unique-key pair tables).
uint32_t ops_per_wave_for(const sh_table *t, uint64_t n, int kind)
{
    if (t->ops_per_wave)
        return t->ops_per_wave;
    const uint64_t waves = (uint64_t)t->num_cu * waves_per_cu_for(t, kind);
    uint32_t C = default_shape(t, kind).max_ops;
    while (C > 8 && (n + C - 1) / C < waves)
        C >>= 1;
    return C;
}

// The launch sequence number that seeds the allocator's starting blocks; calls on one table may
// come from several host threads.
uint32_t next_seq(uint32_t *seq) { return __atomic_fetch_add(seq, 1u, __ATOMIC_RELAXED); }

// Wavefronts of kernel `fn` that fit on one compute unit at once (its registers and LDS, with
// `dyn_lds` bytes of dynamic LDS per block), from the occupancy API, cached per kernel and LDS
// size (one GPU model per process); 64 (no limit) if the query fails, whose error is then
// cleared so that the launch check after it does not report it.
uint32_t resident_waves_per_cu(const void *fn, size_t dyn_lds = 0)
{
    struct Entry {
        const void *fn;
        size_t lds;
        uint32_t waves;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    std::lock_guard<std::mutex> g(mu);
    for (const auto &e : cache)
        if (e.fn == fn && e.lds == dyn_lds)
            return e.waves;
    int nb = 0;
    uint32_t w = 64;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, dyn_lds) == hipSuccess &&
        nb > 0)
        w = (uint32_t)nb * kWavesPerBlock;
    else
        (void)hipGetLastError();
    try {
        cache.push_back(Entry{fn, dyn_lds, w});
    } catch (...) {
        // not cached: the next launch asks again
    }
    return w;
}

// Waves per CU of a persistent launch of `fn`: the caller's explicit choice (set > 0) as given;
// else the default, lowered to what fits at once, so no wavefront waits for another to finish
// its whole share.
uint32_t launch_wpc(uint32_t set, uint32_t dflt, const void *fn, size_t dyn_lds = 0)
{
    if (set)
        return set;
    const uint32_t r = resident_waves_per_cu(fn, dyn_lds);
    return r < dflt ? r : dflt;
}

// Dynamic LDS of a batched launch over nb descriptors: their 64-bit chunk prefix, rounded up
// to a multiple of 64 descriptors so that few distinct sizes reach the occupancy cache.
size_t multi_lds_bytes(uint32_t nb)
{
    return (size_t)(((nb + 1 + 63) / 64) * 64) * sizeof(uint64_t);
}

uint32_t grid_for(const sh_table *t, uint64_t n, uint32_t C, uint32_t wpc)
{
    const uint64_t chunks = (n + C - 1) / C;
    uint64_t waves = (uint64_t)t->num_cu * wpc;
    if (waves > chunks)
        waves = chunks;
    if (waves == 0)
        waves = 1;
    return (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
}

sh_status_t launch_init(sh_table *t, void *stream)
{
    Layout L;
    layout_of(&t->p, &L);
    const size_t hdr16 = kHeaderBytes / 16;
    const size_t ones16 = (L.bitmap - L.base) / 16;
    const size_t zeros16 = (L.total - L.bitmap) / 16;
    const size_t total = hdr16 + ones16 + zeros16;
    size_t blocks = (total + kBlock - 1) / kBlock;
    const size_t cap = (size_t)t->num_cu * 8;
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(init_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, S(stream),
                       reinterpret_cast<uint4 *>(t->storage), hdr16, ones16, zeros16);
    return check_launch();
}

using OpsFn = void (*)(View, const uint8_t *, const uint32_t *, const uint32_t *, uint64_t,
                      uint32_t *, uint8_t *, uint32_t, uint32_t);

// The operation kernel for kind K at C ops per wavefront, in one table mode: a straight run of
// C / 2 loads per round, one per op pair.
template <int K, bool Dup, bool KO>
OpsFn ops_fn_mode(uint32_t C)
{
    return C == 64 ? ops_kernel<K, Dup, KO, 32>
                   : C == 32 ? ops_kernel<K, Dup, KO, 16>
                             : C == 16 ? ops_kernel<K, Dup, KO, 8> : ops_kernel<K, Dup, KO, 4>;
}

// The operation kernel for kind K on table t at C ops per wavefront.
template <int K>
OpsFn ops_fn(const sh_table *t, uint32_t C)
{
    switch (t->v.mode) {
    case 0:
        return ops_fn_mode<K, false, false>(C);
    case SH_TABLE_DUPLICATES:
        return ops_fn_mode<K, true, false>(C);
    case SH_TABLE_KEYS_ONLY:
        return ops_fn_mode<K, false, true>(C);
    default:
        return ops_fn_mode<K, true, true>(C);
    }
}

using AllFn = void (*)(View, const uint32_t *, uint64_t, uint32_t *, const uint64_t *,
                      uint32_t *, uint64_t, uint64_t);
// SEARCHALL/DELETEALL at C ops per chunk: a straight run of C / 2 loads, one per op pair.
// Each pair's list is then walked on its own, so a wavefront's time goes to dependent latency:
// by default short chunks (8 ops) and as many wavefronts as fit, up to 32 per CU (2^20 SEARCHALL
// counts over 4 copies of each key: 83 us at 32 per CU and 8 ops against 116 us at 16 per CU
// and 32 ops).
constexpr uint32_t kAllOps = 8;
constexpr uint32_t kAllWavesPerCU = 32;

template <bool Del, bool KO>
AllFn all_fn(uint32_t C)
{
    return C == 64 ? all_kernel<Del, KO, 32>
                   : C == 32 ? all_kernel<Del, KO, 16>
                             : C == 16 ? all_kernel<Del, KO, 8> : all_kernel<Del, KO, 4>;
}

template <int K>
sh_status_t launch_ops(sh_table *t, const uint8_t *ops, const uint32_t *keys,
                       const uint32_t *vals, uint64_t n, uint32_t *vout, uint8_t *sout,
                       void *stream)
{
    if (!t)
        return SH_EINVAL;
    if (n == 0)
        return SH_OK;
    if (n >= (1ull << 32) || !keys)
        return SH_EINVAL;
    const uint32_t C = ops_per_wave_for(t, n, K);
    const OpsFn fn = ops_fn<K>(t, C);
    const uint32_t wpc =
        launch_wpc(t->waves_per_cu, default_shape(t, K).waves_per_cu, reinterpret_cast<const void *>(fn));
    const dim3 grid(grid_for(t, n, C, wpc));
    const uint32_t seq = next_seq(&t->seq);
    hipLaunchKernelGGL(fn, grid, dim3(kBlock), 0, S(stream), t->v, ops, keys, vals, n, vout, sout,
                       seq, t->flags);
    return check_launch();
}

sh_status_t walk(sh_table *t, uint32_t *dbkt, uint32_t *dkey, uint32_t *dval, uint64_t cap,
                 uint32_t *counts, int emit, uint64_t *d_count, uint32_t *d_viol, void *stream)
{
    hipLaunchKernelGGL(clear_stats_kernel, dim3(1), dim3(64), 0, S(stream), t->v, d_count,
                       d_viol);
    if (check_launch() != SH_OK)
        return SH_EHIP;
    uint64_t waves = (uint64_t)t->num_cu * 16;
    if (waves > t->p.num_buckets)
        waves = t->p.num_buckets;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    if (t->v.mode & SH_TABLE_KEYS_ONLY)
        hipLaunchKernelGGL(walk_kernel<true>, dim3(blocks), dim3(kBlock), 0, S(stream), t->v,
                           dbkt, dkey, dval, cap, counts, emit);
    else
        hipLaunchKernelGGL(walk_kernel<false>, dim3(blocks), dim3(kBlock), 0, S(stream), t->v,
                           dbkt, dkey, dval, cap, counts, emit);
    if (check_launch() != SH_OK)
        return SH_EHIP;
    if (t->v.total_blocks) {
        uint32_t pb = (uint32_t)(((size_t)t->v.total_blocks * 64 + kBlock - 1) / kBlock);
        if (pb > (uint32_t)t->num_cu * 4)
            pb = (uint32_t)t->num_cu * 4;
        hipLaunchKernelGGL(popcount_kernel, dim3(pb), dim3(kBlock), 0, S(stream), t->v);
        if (check_launch() != SH_OK)
            return SH_EHIP;
    }
    if (d_count || d_viol) {
        hipLaunchKernelGGL(publish_dump_kernel, dim3(1), dim3(64), 0, S(stream), t->v, d_count,
                           d_viol);
        if (check_launch() != SH_OK)
            return SH_EHIP;
    }
    return SH_OK;
}

sh_status_t device_cus(int *ncu)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return SH_EHIP;
    if (*ncu <= 0)
        *ncu = 1;
    return SH_OK;
}

// Fill a host handle for a table whose storage (already validated) starts at `storage`.
void bind_table(sh_table *t, const sh_params_t *p, char *storage, size_t bytes, int ncu)
{
    Layout L;
    layout_of(p, &L);
    t->p = *p;
    t->storage = storage;
    t->bytes = bytes;
    t->num_cu = ncu;
    t->waves_per_cu = 0; // 0: the operation kind's default
    t->ops_per_wave = 0;
    t->flags = 0;
    t->seq = 0;
    t->v.hdr = reinterpret_cast<Header *>(storage);
    t->v.counters = reinterpret_cast<unsigned long long *>(storage + 256);
    t->v.base = reinterpret_cast<uint64_t *>(storage + L.base);
    t->v.pool = reinterpret_cast<uint64_t *>(storage + L.pool);
    t->v.bitmap = reinterpret_cast<uint32_t *>(storage + L.bitmap);
    t->v.B = p->num_buckets;
    t->v.a = p->hash_a;
    t->v.b = p->hash_b;
    t->v.pool_slabs = p->pool_slabs;
    t->v.nblk = p->pool_slabs / SH_BLOCK_SLABS;
    t->v.dir = reinterpret_cast<const SuperDesc *>(storage + kDirOffset);
    t->v.grown = reinterpret_cast<uint32_t *>(storage + kGrownOffset);
    t->v.nsuper = 1;
    t->v.total_blocks = t->v.nblk;
    t->v.mode = p->flags & (SH_TABLE_DUPLICATES | SH_TABLE_KEYS_ONLY);
    t->super_slabs = 0;
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Directory first, then each table's storage, all 256-byte aligned. offs[t] (if given) gets the
// byte offset of table t. Returns 0 for invalid input.
size_t multi_layout(uint32_t T, const sh_params_t *p, size_t *offs)
{
    if (T == 0 || !p)
        return 0;
    size_t off = round256((size_t)T * sizeof(View));
    for (uint32_t t = 0; t < T; ++t) {
        Layout L;
        if (!layout_of(&p[t], &L) || p[t].flags != 0)
            return 0; // the batched kernel runs the unique-key operations on pairs only
        if (offs)
            offs[t] = off;
        off += round256(L.total);
    }
    return off;
}

// One batched launch. n_ops bounds the op arrays; work_ops (the ops the descriptors actually
// hold, or n_ops if unknown) sizes the grid and the ops per wavefront.
uint32_t blocks_for(uint64_t waves)
{
    const uint64_t b = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return b ? (uint32_t)b : 1u;
}

using MultiFn = void (*)(const View *, uint32_t, const sh_batch_desc_t *, uint32_t, uint64_t,
                        const uint8_t *, const uint32_t *, const uint32_t *, uint32_t *,
                        uint8_t *, uint32_t, uint32_t);

// One batched launch; wpc = 0 takes the default waves per CU (lowered to what fits at once).
sh_status_t launch_multi_raw(const View *d_dir, uint32_t T, const sh_batch_desc_t *d_desc,
                             uint32_t nb, const uint8_t *d_ops, const uint32_t *d_keys,
                             const uint32_t *d_vals_in, uint32_t *d_vals_out, uint8_t *d_status,
                             uint64_t n_ops, uint64_t work_ops, int num_cu, uint32_t wpc,
                             uint32_t ops_per_wave, uint32_t seq, uint32_t flags,
                             hipStream_t stream)
{
    uint32_t C = ops_per_wave;
    if (!C) {
        const uint64_t waves = (uint64_t)num_cu * (wpc ? wpc : kDefaultWavesPerCU);
        C = 64;
        while (C > 8 && (work_ops + C - 1) / C < waves)
            C >>= 1;
    }
    // the straight run of loads is as long as a chunk's op pairs
    const MultiFn fn = C == 64 ? multi_kernel<32>
                               : C == 32 ? multi_kernel<16>
                                         : C == 16 ? multi_kernel<8> : multi_kernel<4>;
    uint64_t w = (uint64_t)num_cu * launch_wpc(wpc, kDefaultWavesPerCU,
                                               reinterpret_cast<const void *>(fn),
                                               multi_lds_bytes(nb));
    const uint64_t chunks = (work_ops + C - 1) / C + nb; // at most one partial chunk each
    if (w > chunks)
        w = chunks;
    hipLaunchKernelGGL(fn, dim3(blocks_for(w)), dim3(kBlock), multi_lds_bytes(nb), stream,
                       d_dir, T, d_desc, nb,
                       n_ops, d_ops, d_keys, d_vals_in, d_vals_out, d_status, seq, flags);
    return check_launch();
}

sh_status_t launch_multi(sh_multi *m, const sh_batch_desc_t *d_desc, uint32_t nb,
                         const uint8_t *d_ops, const uint32_t *d_keys, const uint32_t *d_vals_in,
                         uint32_t *d_vals_out, uint8_t *d_status, uint64_t n_ops,
                         hipStream_t stream)
{
    return launch_multi_raw(m->d_dir, m->T, d_desc, nb, d_ops, d_keys, d_vals_in, d_vals_out,
                            d_status, n_ops, n_ops, m->num_cu, m->waves_per_cu, m->ops_per_wave,
                            next_seq(&m->seq), m->flags, stream);
}

} // namespace

extern "C" {

size_t sh_storage_bytes(const sh_params_t *p)
{
    Layout L;
    return layout_of(p, &L) ? L.total : 0;
}

sh_status_t sh_create(const sh_params_t *p, void *d_storage, size_t bytes, void *stream,
                      sh_table_t **out)
{
    Layout L;
    if (!out || !d_storage || !layout_of(p, &L) || bytes < L.total ||
        (reinterpret_cast<uintptr_t>(d_storage) & 255u))
        return SH_EINVAL;
    int ncu = 0;
    if (device_cus(&ncu) != SH_OK)
        return SH_EHIP;
    sh_table *t = static_cast<sh_table *>(calloc(1, sizeof(sh_table)));
    if (!t)
        return SH_ENOMEM;
    bind_table(t, p, static_cast<char *>(d_storage), bytes, ncu);
    sh_status_t s = launch_init(t, stream);
    if (s != SH_OK) {
        free(t);
        return s;
    }
    *out = t;
    return SH_OK;
}

sh_status_t sh_reset(sh_table_t *t, void *stream)
{
    if (!t)
        return SH_EINVAL;
    Layout L;
    layout_of(&t->p, &L);
    const size_t hdr16 = kHeaderBytes / 16;
    const size_t base16 = (L.pool - L.base) / 16;
    size_t fill = (hdr16 + base16 + kBlock - 1) / kBlock;
    const size_t cap = (size_t)t->num_cu * 8;
    if (fill > cap)
        fill = cap;
    // one wavefront per bitmap row, at most the rows of every super block
    const size_t rows = t->v.total_blocks;
    size_t pool_blocks = (rows + kWavesPerBlock - 1) / kWavesPerBlock;
    if (pool_blocks > cap)
        pool_blocks = cap;
    hipLaunchKernelGGL(reset_kernel, dim3((uint32_t)(fill + pool_blocks)), dim3(kBlock), 0,
                       S(stream), t->v, reinterpret_cast<uint4 *>(t->storage), hdr16, base16,
                       (uint32_t)pool_blocks);
    return check_launch();
}

size_t sh_super_block_bytes(uint32_t slabs)
{
    if (slabs == 0 || slabs % SH_BLOCK_SLABS != 0 || slabs > kMaxSuperSlabs)
        return 0;
    return (size_t)slabs * SH_SLAB_BYTES + (size_t)(slabs / SH_BLOCK_SLABS) * 256;
}

sh_status_t sh_add_super_block(sh_table_t *t, void *d_mem, size_t bytes, void *stream)
{
    if (!t || !d_mem || (reinterpret_cast<uintptr_t>(d_mem) & 255u) ||
        t->v.nsuper >= kMaxSupers)
        return SH_EINVAL;
    // the most slabs (a multiple of a block, at most kMaxSuperSlabs) whose slabs and bitmap
    // rows fit in `bytes`
    const size_t per_block = (size_t)SH_BLOCK_SLABS * SH_SLAB_BYTES + 256;
    uint64_t blocks = bytes / per_block;
    if (blocks > kMaxSuperSlabs / SH_BLOCK_SLABS)
        blocks = kMaxSuperSlabs / SH_BLOCK_SLABS;
    if (blocks == 0 || (uint64_t)t->v.total_blocks + blocks > (1ull << 31))
        return SH_EINVAL;
    const uint32_t slabs = (uint32_t)(blocks * SH_BLOCK_SLABS);
    char *mem = static_cast<char *>(d_mem);
    uint64_t *pool = reinterpret_cast<uint64_t *>(mem);
    uint32_t *bitmap = reinterpret_cast<uint32_t *>(mem + (size_t)slabs * SH_SLAB_BYTES);
    // slabs all ones (empty), bitmap rows zero (free), then the directory entry
    const size_t ones16 = (size_t)slabs * SH_SLAB_BYTES / 16, zeros16 = blocks * 256 / 16;
    size_t nb = (ones16 + zeros16 + kBlock - 1) / kBlock;
    if (nb > (size_t)t->num_cu * 8)
        nb = (size_t)t->num_cu * 8;
    const uint32_t sb = t->v.nsuper;
    hipLaunchKernelGGL(init_kernel, dim3((uint32_t)nb), dim3(kBlock), 0, S(stream),
                       reinterpret_cast<uint4 *>(mem), (size_t)0, ones16, zeros16);
    hipLaunchKernelGGL(set_super_kernel, dim3(1), dim3(64), 0, S(stream),
                       const_cast<SuperDesc *>(t->v.dir), sb, pool, bitmap, slabs,
                       t->v.total_blocks);
    if (check_launch() != SH_OK)
        return SH_EHIP;
    t->v.nsuper = sb + 1;
    t->v.total_blocks += (uint32_t)blocks;
    t->super_slabs += slabs;
    if (t->owner) {
        // the batched kernel reads the tables' views from the multi-table directory
        sh_multi *m = t->owner;
        m->h_dir[t->index] = t->v;
        if (hipMemcpyAsync(m->d_dir + t->index, m->h_dir + t->index, sizeof(View),
                           hipMemcpyHostToDevice, S(stream)) != hipSuccess)
            return SH_EHIP;
    }
    return SH_OK;
}

sh_status_t sh_flush(sh_table_t *t, uint32_t first_bucket, uint32_t num_buckets, void *stream)
{
    if (!t || first_bucket > t->p.num_buckets || num_buckets > t->p.num_buckets - first_bucket)
        return SH_EINVAL;
    if (num_buckets == 0)
        return SH_OK;
    // a light kernel bound by the latency of walking each list: twice the operation kernels'
    // wavefronts per compute unit, two buckets per wavefront
    uint64_t waves = (uint64_t)t->num_cu * 2 * kDefaultWavesPerCU;
    const uint64_t pairs = ((uint64_t)num_buckets + 1) / 2;
    if (waves > pairs)
        waves = pairs;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    if (t->v.mode & SH_TABLE_KEYS_ONLY)
        hipLaunchKernelGGL(flush_kernel<true>, dim3(blocks), dim3(kBlock), 0, S(stream), t->v,
                           first_bucket, num_buckets);
    else
        hipLaunchKernelGGL(flush_kernel<false>, dim3(blocks), dim3(kBlock), 0, S(stream), t->v,
                           first_bucket, num_buckets);
    return check_launch();
}

static sh_status_t launch_all(sh_table *t, bool del, const uint32_t *keys, uint64_t n,
                              uint32_t *counts, const uint64_t *offsets, uint32_t *vals,
                              uint64_t cap, void *stream)
{
    const bool dup = (t->v.mode & SH_TABLE_DUPLICATES) != 0;
    const bool ko = (t->v.mode & SH_TABLE_KEYS_ONLY) != 0;
    // what a deleted slot becomes: a tombstone, or with duplicates an empty slot
    const uint64_t gone = ko ? (dup ? kEmpty : kTombKey) : (dup ? kEmptyPair : kTombPair);
    // ops per chunk: the table's setting, else the default; the straight run has one load per
    // op pair
    const uint32_t C = t->ops_per_wave ? t->ops_per_wave : kAllOps;
    const AllFn fn = del ? (ko ? all_fn<true, true>(C) : all_fn<true, false>(C))
                         : (ko ? all_fn<false, true>(C) : all_fn<false, false>(C));
    // the default grid is what fits at once at the kernel's register use
    uint64_t waves = (uint64_t)t->num_cu *
                     launch_wpc(t->waves_per_cu, kAllWavesPerCU,
                                reinterpret_cast<const void *>(fn));
    const uint64_t chunks = (n + C - 1) / C;
    if (waves > chunks)
        waves = chunks;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    if (del)
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, S(stream), t->v, keys, n, counts,
                           nullptr, nullptr, 0, gone);
    else
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, S(stream), t->v, keys, n, counts,
                           offsets, vals, cap, 0);
    return check_launch();
}

sh_status_t sh_search_all(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_counts,
                          const uint64_t *d_offsets, uint32_t *d_vals_out, uint64_t d_vals_cap,
                          void *stream)
{
    if (!t || n >= (1ull << 32) || (n && (!d_keys || !d_counts)) ||
        (d_offsets == nullptr) != (d_vals_out == nullptr))
        return SH_EINVAL;
    if (n == 0)
        return SH_OK;
    return launch_all(t, false, d_keys, n, d_counts, d_offsets, d_vals_out,
                      d_vals_out ? d_vals_cap : 0, stream);
}

sh_status_t sh_delete_all(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_counts,
                          void *stream)
{
    if (!t || n >= (1ull << 32) || (n && !d_keys))
        return SH_EINVAL;
    if (n == 0)
        return SH_OK;
    return launch_all(t, true, d_keys, n, d_counts, nullptr, nullptr, 0, stream);
}

sh_status_t sh_alloc_slabs(sh_table_t *t, uint64_t n, uint32_t *d_out, void *stream)
{
    if (!t || (n && !d_out) || n >= (1ull << 32))
        return SH_EINVAL;
    if (n == 0)
        return SH_OK;
    const uint64_t blocks = (n + kBlock - 1) / kBlock; // one request per lane
    hipLaunchKernelGGL(alloc_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, S(stream), t->v, n,
                       d_out, next_seq(&t->seq), t->flags);
    return check_launch();
}

sh_status_t sh_free_slabs(sh_table_t *t, const uint32_t *d_idx, uint64_t n, void *stream)
{
    if (!t || (n && !d_idx) || n >= (1ull << 32))
        return SH_EINVAL;
    if (n == 0)
        return SH_OK;
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)t->num_cu * 8;
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(free_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, S(stream), t->v,
                       d_idx, n);
    return check_launch();
}

sh_status_t sh_destroy(sh_table_t *t)
{
    if (!t || t->embedded)
        return SH_EINVAL;
    free(t);
    return SH_OK;
}

sh_status_t sh_set_launch(sh_table_t *t, const sh_launch_t *shape)
{
    if (!t)
        return SH_EINVAL;
    if (!shape) {
        t->waves_per_cu = 0;
        t->ops_per_wave = 0;
        t->flags = 0;
        return SH_OK;
    }
    const uint32_t c = shape->ops_per_wave;
    if (shape->waves_per_cu > 64 || (c != 0 && c != 8 && c != 16 && c != 32 && c != 64) ||
        (shape->flags & ~(uint32_t)SH_LAUNCH_COUNTERS))
        return SH_EINVAL;
    t->waves_per_cu = shape->waves_per_cu; // 0: the operation kind's default
    t->ops_per_wave = c;
    t->flags = shape->flags;
    return SH_OK;
}

sh_status_t sh_launch_shape(const sh_table_t *t, int kind, uint64_t n, uint32_t *waves_per_cu,
                            uint32_t *ops_per_wave)
{
    if (!t || !waves_per_cu || !ops_per_wave || kind < kSearch || kind > kMixed)
        return SH_EINVAL;
    const uint32_t C = ops_per_wave_for(t, n, kind);
    const OpsFn fn = kind == kSearch   ? ops_fn<kSearch>(t, C)
                     : kind == kInsert ? ops_fn<kInsert>(t, C)
                     : kind == kDelete ? ops_fn<kDelete>(t, C)
                                       : ops_fn<kMixed>(t, C);
    *waves_per_cu = launch_wpc(t->waves_per_cu, default_shape(t, kind).waves_per_cu,
                               reinterpret_cast<const void *>(fn));
    *ops_per_wave = C;
    return SH_OK;
}

sh_status_t sh_build(sh_table_t *t, const uint32_t *d_keys, const uint32_t *d_vals, uint64_t n,
                     uint8_t *d_status, void *stream)
{
    const bool ko = t && (t->v.mode & SH_TABLE_KEYS_ONLY);
    if (n && !d_vals && !ko) // a key-only table has no values to read
        return SH_EINVAL;
    return launch_ops<kInsert>(t, nullptr, d_keys, d_vals, n, nullptr, d_status, stream);
}

sh_status_t sh_insert(sh_table_t *t, const uint32_t *d_keys, const uint32_t *d_vals,
                      uint64_t n, uint8_t *d_status, void *stream)
{
    return sh_build(t, d_keys, d_vals, n, d_status, stream);
}

sh_status_t sh_delete(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint8_t *d_status,
                      void *stream)
{
    return launch_ops<kDelete>(t, nullptr, d_keys, nullptr, n, nullptr, d_status, stream);
}

sh_status_t sh_search(sh_table_t *t, const uint32_t *d_keys, uint64_t n, uint32_t *d_vals_out,
                      uint8_t *d_found, void *stream)
{
    if (n && !d_vals_out)
        return SH_EINVAL;
    return launch_ops<kSearch>(t, nullptr, d_keys, nullptr, n, d_vals_out, d_found, stream);
}

sh_status_t sh_mixed(sh_table_t *t, const uint8_t *d_ops, const uint32_t *d_keys,
                     const uint32_t *d_vals_in, uint64_t n, uint32_t *d_vals_out,
                     uint8_t *d_status, void *stream)
{
    const bool ko = t && (t->v.mode & SH_TABLE_KEYS_ONLY);
    if (n && (!d_ops || (!d_vals_in && !ko) || !d_vals_out || !d_status))
        return SH_EINVAL;
    return launch_ops<kMixed>(t, d_ops, d_keys, d_vals_in, n, d_vals_out, d_status, stream);
}

sh_status_t sh_stats(sh_table_t *t, sh_stats_t *h_out, void *stream)
{
    if (!t || !h_out)
        return SH_EINVAL;
    sh_status_t s = walk(t, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, stream);
    if (s != SH_OK)
        return s;
    Header h;
    unsigned long long cs[kCounterSlots * 8];
    if (hipMemcpyAsync(&h, t->v.hdr, sizeof(Header), hipMemcpyDeviceToHost, S(stream)) !=
            hipSuccess ||
        hipMemcpyAsync(cs, t->v.counters, sizeof(cs), hipMemcpyDeviceToHost, S(stream)) !=
            hipSuccess ||
        hipStreamSynchronize(S(stream)) != hipSuccess)
        return SH_EHIP;
    unsigned long long sum[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t k = 0; k < kCounterSlots; ++k)
        for (int f = 0; f < 6; ++f)
            sum[f] += cs[k * 8 + f];
    memset(h_out, 0, sizeof(*h_out));
    h_out->live = h.live;
    h_out->tombstones = h.tomb;
    h_out->slabs_total = h.slabs;
    h_out->pool_allocated = h.pool_alloc;
    h_out->pool_capacity = t->p.pool_slabs + t->super_slabs;
    h_out->error_word = h.err;
    h_out->violations = h.violations;
    h_out->num_buckets = t->p.num_buckets;
    h_out->hash_a = t->p.hash_a;
    h_out->hash_b = t->p.hash_b;
    h_out->hash_p = kPrime;
    h_out->rounds = sum[0];
    h_out->cas_lost = sum[1];
    h_out->allocs = sum[2];
    h_out->link_lost = sum[3];
    h_out->block_moves = sum[4];
    h_out->alloc_lost = sum[5];
    return SH_OK;
}

sh_status_t sh_dump(sh_table_t *t, uint32_t *d_bucket, uint32_t *d_key, uint32_t *d_val,
                    uint64_t cap, uint32_t *d_bucket_counts, uint64_t *d_count,
                    uint32_t *d_violations, void *stream)
{
    if (!t || !d_count || (cap && (!d_bucket || !d_key || !d_val)))
        return SH_EINVAL;
    return walk(t, d_bucket, d_key, d_val, cap, d_bucket_counts, 1, d_count, d_violations,
                stream);
}

size_t sh_multi_storage_bytes(uint32_t T, const sh_params_t *h_params)
{
    return multi_layout(T, h_params, nullptr);
}

sh_status_t sh_multi_create(uint32_t T, const sh_params_t *h_params, void *d_storage,
                            size_t bytes, void *stream, sh_multi_t **out)
{
    if (!out || !d_storage || (reinterpret_cast<uintptr_t>(d_storage) & 255u))
        return SH_EINVAL;
    const size_t need = multi_layout(T, h_params, nullptr);
    if (need == 0 || bytes < need)
        return SH_EINVAL;
    int ncu = 0;
    if (device_cus(&ncu) != SH_OK)
        return SH_EHIP;
    sh_multi *m = static_cast<sh_multi *>(calloc(1, sizeof(sh_multi)));
    size_t *offs = static_cast<size_t *>(calloc(T, sizeof(size_t)));
    if (m) {
        m->tables = static_cast<sh_table *>(calloc(T, sizeof(sh_table)));
        m->h_dir = static_cast<View *>(calloc(T, sizeof(View)));
    }
    if (!m || !offs || !m->tables || !m->h_dir) {
        if (m) {
            free(m->tables);
            free(m->h_dir);
        }
        free(m);
        free(offs);
        return SH_ENOMEM;
    }
    multi_layout(T, h_params, offs);
    m->T = T;
    m->storage = static_cast<char *>(d_storage);
    m->bytes = bytes;
    m->d_dir = reinterpret_cast<View *>(d_storage);
    m->num_cu = ncu;
    m->waves_per_cu = 0; // the default
    sh_status_t s = SH_OK;
    for (uint32_t t = 0; t < T && s == SH_OK; ++t) {
        Layout L;
        layout_of(&h_params[t], &L);
        bind_table(&m->tables[t], &h_params[t], m->storage + offs[t], L.total, ncu);
        m->tables[t].embedded = 1;
        m->tables[t].owner = m;
        m->tables[t].index = t;
        m->h_dir[t] = m->tables[t].v;
        s = launch_init(&m->tables[t], stream);
    }
    free(offs);
    if (s == SH_OK &&
        (hipMemcpyAsync(m->d_dir, m->h_dir, (size_t)T * sizeof(View), hipMemcpyHostToDevice,
                        S(stream)) != hipSuccess ||
         hipStreamSynchronize(S(stream)) != hipSuccess))
        s = SH_EHIP;
    if (s != SH_OK) {
        free(m->tables);
        free(m->h_dir);
        free(m);
        return s;
    }
    *out = m;
    return SH_OK;
}

sh_status_t sh_multi_table(sh_multi_t *m, uint32_t t, sh_table_t **out)
{
    if (!m || !out || t >= m->T)
        return SH_EINVAL;
    *out = &m->tables[t];
    return SH_OK;
}

sh_status_t sh_multi_set_launch(sh_multi_t *m, const sh_launch_t *shape)
{
    if (!m)
        return SH_EINVAL;
    if (!shape) {
        m->waves_per_cu = 0;
        m->ops_per_wave = 0;
        m->flags = 0;
        return SH_OK;
    }
    const uint32_t c = shape->ops_per_wave;
    if (shape->waves_per_cu > 64 || (c != 0 && c != 8 && c != 16 && c != 32 && c != 64) ||
        (shape->flags & ~(uint32_t)SH_LAUNCH_COUNTERS))
        return SH_EINVAL;
    m->waves_per_cu = shape->waves_per_cu; // 0: the default
    m->ops_per_wave = c;
    m->flags = shape->flags;
    return SH_OK;
}

sh_status_t sh_multi_mixed(sh_multi_t *m, const sh_batch_desc_t *d_desc, uint32_t nb,
                           const uint8_t *d_ops, const uint32_t *d_keys,
                           const uint32_t *d_vals_in, uint32_t *d_vals_out, uint8_t *d_status,
                           uint64_t n_ops, void *stream)
{
    if (!m || nb > kMaxBatches || n_ops >= (1ull << 40))
        return SH_EINVAL;
    if (nb == 0 || n_ops == 0)
        return SH_OK;
    if (!d_desc || !d_ops || !d_keys || !d_vals_in || !d_vals_out || !d_status)
        return SH_EINVAL;
    return launch_multi(m, d_desc, nb, d_ops, d_keys, d_vals_in, d_vals_out, d_status, n_ops,
                        S(stream));
}

sh_status_t sh_multi_mixed_each(sh_multi_t *m, const sh_batch_desc_t *h_desc, uint32_t nb,
                                const uint8_t *d_ops, const uint32_t *d_keys,
                                const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                uint8_t *d_status, uint64_t n_ops, void *stream)
{
    if (!m || (nb && (!h_desc || !d_ops || !d_keys || !d_vals_in || !d_vals_out || !d_status)))
        return SH_EINVAL;
    for (uint32_t d = 0; d < nb; ++d)
        if (h_desc[d].table >= m->T || h_desc[d].offset > n_ops ||
            h_desc[d].length > n_ops - h_desc[d].offset)
            return SH_EINVAL;
    for (uint32_t d = 0; d < nb; ++d) {
        const sh_batch_desc_t &b = h_desc[d];
        const uint64_t o = b.offset;
        const sh_status_t s =
            launch_ops<kMixed>(&m->tables[b.table], d_ops + o, d_keys + o, d_vals_in + o, b.length,
                               d_vals_out + o, d_status + o, stream);
        if (s != SH_OK)
            return s;
    }
    return SH_OK;
}

sh_status_t sh_multi_graph(sh_multi_t *m, const sh_batch_desc_t *d_desc, uint32_t nb,
                           const uint8_t *d_ops, const uint32_t *d_keys,
                           const uint32_t *d_vals_in, uint32_t *d_vals_out, uint8_t *d_status,
                           uint64_t n_ops, sh_graph_t **out)
{
    if (!m || !out || nb == 0 || nb > kMaxBatches || n_ops == 0 || n_ops >= (1ull << 40) ||
        !d_desc || !d_ops || !d_keys || !d_vals_in || !d_vals_out || !d_status)
        return SH_EINVAL;
    sh_graph *g = static_cast<sh_graph *>(calloc(1, sizeof(sh_graph)));
    if (!g)
        return SH_ENOMEM;
    hipStream_t cs = nullptr;
    sh_status_t s = SH_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        free(g);
        return SH_EHIP;
    }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        s = SH_EHIP;
    } else {
        s = launch_multi(m, d_desc, nb, d_ops, d_keys, d_vals_in, d_vals_out, d_status, n_ops,
                         cs);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (s == SH_OK && e != hipSuccess)
            s = SH_EHIP;
        if (s == SH_OK) {
            g->graph = graph;
            if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
                s = SH_EHIP;
        } else if (graph) {
            (void)hipGraphDestroy(graph); // best effort on the error path
        }
    }
    (void)hipStreamDestroy(cs);
    if (s != SH_OK) {
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        free(g);
        return s;
    }
    *out = g;
    return SH_OK;
}

sh_status_t sh_capture_begin(void *stream)
{
    if (!stream)
        return SH_EINVAL; // the NULL stream cannot be captured
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(S(stream), &st) != hipSuccess)
        return SH_EHIP;
    if (st != hipStreamCaptureStatusNone)
        return SH_EINVAL;
    return hipStreamBeginCapture(S(stream), hipStreamCaptureModeThreadLocal) == hipSuccess
               ? SH_OK
               : SH_EHIP;
}

sh_status_t sh_capture_end(void *stream, sh_graph_t **out)
{
    if (!stream || !out)
        return SH_EINVAL;
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(S(stream), &graph) != hipSuccess || !graph) {
        if (graph)
            (void)hipGraphDestroy(graph); // best effort on the error path
        return SH_EHIP;
    }
    sh_graph *g = static_cast<sh_graph *>(calloc(1, sizeof(sh_graph)));
    if (!g) {
        (void)hipGraphDestroy(graph);
        return SH_ENOMEM;
    }
    g->graph = graph;
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        free(g);
        return SH_EHIP;
    }
    *out = g;
    return SH_OK;
}

sh_status_t sh_graph_launch(sh_graph_t *g, void *stream)
{
    if (!g)
        return SH_EINVAL;
    return hipGraphLaunch(g->exec, S(stream)) == hipSuccess ? SH_OK : SH_EHIP;
}

sh_status_t sh_graph_destroy(sh_graph_t *g)
{
    if (!g)
        return SH_EINVAL;
    bool ok = hipGraphExecDestroy(g->exec) == hipSuccess;
    ok = (hipGraphDestroy(g->graph) == hipSuccess) && ok;
    free(g);
    return ok ? SH_OK : SH_EHIP;
}

sh_status_t sh_multi_destroy(sh_multi_t *m)
{
    if (!m)
        return SH_EINVAL;
    free(m->tables);
    free(m->h_dir);
    free(m);
    return SH_OK;
}

const char *sh_strerror(sh_status_t s)
{
    switch (s) {
    case SH_OK:
        return "ok";
    case SH_EINVAL:
        return "invalid argument";
    case SH_ENOMEM:
        return "host allocation failed";
    case SH_EHIP:
        return "HIP runtime error";
    case SH_EBUSY:
        return "busy";
    }
    return "unknown status";
}

} // extern "C"

// ---------------------------------------------------------------------------------------------
// Served form: a native request loop doing continuous batching (see include/slabhash.h).

namespace {

constexpr uint32_t kMaxLaunches = 8;
constexpr size_t kCounterBytes = (size_t)kCounterSlots * 8 * sizeof(unsigned long long);

uint64_t clock_now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr size_t kTicketWindow = size_t(1) << 20; // finished requests a server remembers
constexpr uint32_t kReplayBurst = 1024;         // submissions between scans of a load driver

struct ServerReq {
    sh_request_t r;
    uint64_t t_admit;
    uint64_t t_done; // 0 = not finished (guarded by the server mutex)
    bool read;       // its finish has been reported (poll or load driver)
};

struct LaunchSlot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    sh_batch_desc_t *h_desc = nullptr;   // pinned staging for this launch's descriptors
    unsigned long long *h_cnt = nullptr; // pinned copy of the table's counter slots
    sh_batch_desc_t *d_desc = nullptr;   // in the caller's scratch
    std::vector<uint64_t> tickets;
    bool busy = false;
};

} // namespace

struct sh_server {
    sh_table *t = nullptr;
    sh_server_cfg_t cfg{};
    const uint8_t *ops = nullptr;
    const uint32_t *keys = nullptr, *vals = nullptr;
    uint32_t *vout = nullptr;
    uint8_t *sout = nullptr;
    uint64_t n_ops = 0;
    View *d_dir = nullptr;
    int device = 0;
    LaunchSlot slots[kMaxLaunches];
    uint32_t nslots = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<ServerReq> reqs;   // request of ticket t at reqs[t - reqs_base]
    uint64_t reqs_base = 0;       // ticket of reqs.front(); older tickets have expired
    std::deque<uint64_t> pending; // admitted, not yet launched
    uint64_t unfinished = 0;      // admitted, not yet finished
    int64_t reserved = 0;         // slabs promised to unfinished requests
    int64_t allocated = 0;        // pool slabs in use, as last read from the device
    int64_t base_allocated = 0;
    long long base_net = 0;
    uint32_t seq = 0;
    bool stop = false;
    std::atomic<int> error{0};
    std::atomic<uint64_t> completions{0}; // requests finished so far (read without the lock)
    std::thread thr;
};

namespace {

long long counters_net(const unsigned long long *cs)
{
    long long net = 0; // slabs allocated minus slabs given back after a lost link
    for (uint32_t k = 0; k < kCounterSlots; ++k)
        net += (long long)cs[k * 8 + 2] - (long long)cs[k * 8 + 3];
    return net;
}

void server_loop(sh_server *s)
{
    if (hipSetDevice(s->device) != hipSuccess)
        s->error.store(1);
    for (;;) {
        bool progressed = false, any_busy = false;
        // completed launches: stamp their requests, release reservations, refresh occupancy
        for (uint32_t k = 0; k < s->nslots; ++k) {
            LaunchSlot &L = s->slots[k];
            if (!L.busy)
                continue;
            const hipError_t q = hipEventQuery(L.ev);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            if (q != hipSuccess)
                s->error.store(1);
            const uint64_t now = clock_now_ns();
            const long long net = counters_net(L.h_cnt);
            std::lock_guard<std::mutex> g(s->mu);
            for (uint64_t tk : L.tickets) {
                ServerReq &R = s->reqs[tk - s->reqs_base];
                s->reserved -= R.r.inserts;
                --s->unfinished;
                R.t_done = now;
            }
            s->completions.fetch_add(L.tickets.size(), std::memory_order_release);
            const int64_t a = s->base_allocated + (int64_t)(net - s->base_net);
            if (a > s->allocated)
                s->allocated = a; // snapshots can lag one another; occupancy only grows
            L.tickets.clear();
            L.busy = false;
            progressed = true;
        }
        // free slots take everything admitted and not yet launched
        for (uint32_t k = 0; k < s->nslots; ++k) {
            LaunchSlot &L = s->slots[k];
            if (L.busy)
                continue;
            uint32_t nb = 0;
            uint64_t work = 0;
            {
                std::lock_guard<std::mutex> g(s->mu);
                while (!s->pending.empty() && nb < kMaxBatches) {
                    const ServerReq &R = s->reqs[s->pending.front() - s->reqs_base];
                    if (nb > 0 && work + R.r.length > s->cfg.max_batch_ops)
                        break;
                    L.h_desc[nb].offset = R.r.offset;
                    L.h_desc[nb].length = R.r.length;
                    L.h_desc[nb].table = 0;
                    L.tickets.push_back(s->pending.front());
                    s->pending.pop_front();
                    work += R.r.length;
                    ++nb;
                }
            }
            if (nb == 0)
                break;
            bool ok = hipMemcpyAsync(L.d_desc, L.h_desc, nb * sizeof(sh_batch_desc_t),
                                     hipMemcpyHostToDevice, L.stream) == hipSuccess;
            ok = ok && launch_multi_raw(s->d_dir, 1, L.d_desc, nb, s->ops, s->keys, s->vals,
                                        s->vout, s->sout, s->n_ops, work, s->t->num_cu,
                                        s->t->waves_per_cu, s->t->ops_per_wave,
                                        s->seq++,
                                        kFlagCounters, L.stream) == SH_OK;
            ok = ok && hipMemcpyAsync(L.h_cnt, s->t->v.counters, kCounterBytes,
                                      hipMemcpyDeviceToHost, L.stream) == hipSuccess;
            ok = ok && hipEventRecord(L.ev, L.stream) == hipSuccess;
            if (!ok)
                s->error.store(1);
            L.busy = true;
            any_busy = true;
            progressed = true;
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->pending.empty() && !any_busy)
                break;
            if (!any_busy && s->pending.empty())
                s->cv.wait_for(lk, std::chrono::microseconds(200));
            // with launches in flight the loop keeps polling their events
        }
    }
}

// Release a server's slots (best effort: nothing is left to report a failure to).
void server_free(sh_server *s)
{
    for (uint32_t k = 0; k < s->nslots; ++k) {
        LaunchSlot &L = s->slots[k];
        if (L.ev)
            (void)hipEventDestroy(L.ev);
        if (L.stream)
            (void)hipStreamDestroy(L.stream);
        if (L.h_desc)
            (void)hipHostFree(L.h_desc);
        if (L.h_cnt)
            (void)hipHostFree(L.h_cnt);
    }
    delete s;
}

sh_server_cfg_t server_cfg(const sh_server_cfg_t *c)
{
    sh_server_cfg_t r{};
    if (c)
        r = *c;
    if (r.max_launches == 0)
        r.max_launches = 4;
    if (r.max_batch_ops == 0)
        r.max_batch_ops = 1u << 20;
    if (r.max_requests == 0)
        r.max_requests = 4096;
    return r;
}

} // namespace

extern "C" {

uint64_t sh_clock_ns(void) { return clock_now_ns(); }

size_t sh_server_scratch_bytes(const sh_server_cfg_t *cfg)
{
    const sh_server_cfg_t c = server_cfg(cfg);
    if (c.max_launches > kMaxLaunches)
        return 0;
    return 256 + (size_t)c.max_launches * kMaxBatches * sizeof(sh_batch_desc_t);
}

sh_status_t sh_server_start(sh_table_t *t, const sh_server_cfg_t *cfg, const uint8_t *d_ops,
                            const uint32_t *d_keys, const uint32_t *d_vals_in,
                            uint32_t *d_vals_out, uint8_t *d_status, uint64_t n_ops,
                            void *d_scratch, size_t scratch_bytes, void *stream,
                            sh_server_t **out)
{
    const sh_server_cfg_t c = server_cfg(cfg);
    const size_t need = sh_server_scratch_bytes(&c);
    if (!t || !out || !d_ops || !d_keys || !d_vals_in || !d_vals_out || !d_status ||
        n_ops == 0 || n_ops >= (1ull << 40) || !d_scratch || need == 0 ||
        scratch_bytes < need || (reinterpret_cast<uintptr_t>(d_scratch) & 255u) || t->v.mode)
        return SH_EINVAL;
    sh_server *s = nullptr;
    try {
        s = new sh_server(); // its containers may allocate as they are built
    } catch (...) {
        return SH_ENOMEM;
    }
    s->t = t;
    s->cfg = c;
    s->ops = d_ops;
    s->keys = d_keys;
    s->vals = d_vals_in;
    s->vout = d_vals_out;
    s->sout = d_status;
    s->n_ops = n_ops;
    s->d_dir = reinterpret_cast<View *>(d_scratch);
    char *sc = static_cast<char *>(d_scratch) + 256;
    sh_status_t st = (hipGetDevice(&s->device) == hipSuccess) ? SH_OK : SH_EHIP;
    for (uint32_t k = 0; k < c.max_launches && st == SH_OK; ++k) {
        LaunchSlot &L = s->slots[k];
        s->nslots = k + 1;
        L.d_desc = reinterpret_cast<sh_batch_desc_t *>(sc + (size_t)k * kMaxBatches *
                                                                 sizeof(sh_batch_desc_t));
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&L.h_desc),
                          kMaxBatches * sizeof(sh_batch_desc_t), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&L.h_cnt), kCounterBytes,
                          hipHostMallocDefault) != hipSuccess)
            st = SH_EHIP;
    }
    sh_stats_t stt;
    if (st == SH_OK &&
        hipMemcpyAsync(s->d_dir, &t->v, sizeof(View), hipMemcpyHostToDevice, S(stream)) !=
            hipSuccess)
        st = SH_EHIP;
    if (st == SH_OK)
        st = sh_stats(t, &stt, stream); // synchronises `stream`, so the directory copy is done
    if (st == SH_OK &&
        (hipMemcpyAsync(s->slots[0].h_cnt, t->v.counters, kCounterBytes, hipMemcpyDeviceToHost,
                        S(stream)) != hipSuccess ||
         hipStreamSynchronize(S(stream)) != hipSuccess))
        st = SH_EHIP;
    if (st != SH_OK) {
        server_free(s);
        return st;
    }
    s->base_allocated = (int64_t)stt.pool_allocated;
    s->allocated = s->base_allocated;
    s->base_net = counters_net(s->slots[0].h_cnt);
    try {
        // a launch takes at most kMaxBatches requests: the server thread never grows these
        for (uint32_t k = 0; k < s->nslots; ++k)
            s->slots[k].tickets.reserve(kMaxBatches);
        s->thr = std::thread(server_loop, s);
    } catch (...) {
        server_free(s);
        return SH_ENOMEM;
    }
    *out = s;
    return SH_OK;
}

sh_status_t sh_server_submit(sh_server_t *s, const sh_request_t *req, uint64_t *ticket)
{
    if (!s || !req || !ticket || req->length == 0 || req->offset > s->n_ops ||
        req->length > s->n_ops - req->offset || req->inserts > req->length)
        return SH_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop)
        return SH_EINVAL;
    const int64_t avail =
        (int64_t)(s->t->p.pool_slabs + s->t->super_slabs) - s->allocated -
        (int64_t)s->cfg.reserve_slabs;
    if ((int64_t)req->inserts > avail)
        return s->unfinished == 0 ? SH_ENOMEM : SH_EBUSY;
    if (s->unfinished >= s->cfg.max_requests || (int64_t)req->inserts > avail - s->reserved)
        return SH_EBUSY;
    // Finished requests beyond the last kTicketWindow tickets are forgotten once their finish
    // has been reported (their tickets expire), and beyond four windows even if it has not, so
    // a long-running server holds bounded memory.
    while (s->reqs.size() >= kTicketWindow && s->reqs.front().t_done != 0 &&
           (s->reqs.front().read || s->reqs.size() >= 4 * kTicketWindow)) {
        s->reqs.pop_front();
        ++s->reqs_base;
    }
    // the two containers grow first; if either cannot, the request is refused and nothing
    // else has changed
    const uint64_t tk = s->reqs_base + s->reqs.size();
    try {
        s->reqs.emplace_back();
        try {
            s->pending.push_back(tk);
        } catch (...) {
            s->reqs.pop_back();
            throw;
        }
    } catch (...) {
        return SH_ENOMEM;
    }
    ServerReq &R = s->reqs.back();
    R.r = *req;
    R.t_admit = clock_now_ns();
    R.t_done = 0;
    R.read = false;
    s->reserved += req->inserts;
    ++s->unfinished;
    *ticket = tk;
    s->cv.notify_one();
    return SH_OK;
}

sh_status_t sh_server_poll(sh_server_t *s, uint64_t ticket, int *done, uint64_t *t_admit_ns,
                           uint64_t *t_done_ns)
{
    if (!s || !done)
        return SH_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (ticket < s->reqs_base || ticket - s->reqs_base >= s->reqs.size())
        return SH_EINVAL;
    ServerReq &R = s->reqs[ticket - s->reqs_base];
    *done = R.t_done != 0;
    if (*done)
        R.read = true;
    if (t_admit_ns)
        *t_admit_ns = R.t_admit;
    if (t_done_ns)
        *t_done_ns = R.t_done;
    return s->error.load() ? SH_EHIP : SH_OK;
}

static sh_status_t replay_run(sh_server_t *s, const sh_request_t *h_reqs,
                              const uint64_t *h_arrival_ns, uint64_t n, uint64_t *h_admit_ns,
                              uint64_t *h_done_ns)
{
    if (!s || (n && (!h_reqs || !h_arrival_ns || !h_admit_ns || !h_done_ns)))
        return SH_EINVAL;
    for (uint64_t i = 1; i < n; ++i)
        if (h_arrival_ns[i] < h_arrival_ns[i - 1])
            return SH_EINVAL;
    std::vector<uint64_t> ticket(n, UINT64_MAX);
    std::vector<uint64_t> outstanding;
    std::deque<uint64_t> backlog;
    uint64_t next = 0, finished = 0;
    uint64_t seen = s->completions.load(std::memory_order_acquire);
    // after a refusal for lack of room, admission can only succeed once requests finish
    uint64_t refused_at = UINT64_MAX;
    const uint64_t t0 = clock_now_ns();
    while (finished < n) {
        const uint64_t now = clock_now_ns() - t0;
        while (next < n && h_arrival_ns[next] <= now)
            backlog.push_back(next++);
        // submit in bursts so the scan below runs (and reads finished tickets) between them
        for (uint32_t burst = 0; burst < kReplayBurst && !backlog.empty() &&
                                 s->completions.load(std::memory_order_acquire) != refused_at;
             ++burst) {
            const uint64_t i = backlog.front();
            uint64_t tk = 0;
            const uint64_t before = s->completions.load(std::memory_order_acquire);
            const sh_status_t st = sh_server_submit(s, &h_reqs[i], &tk);
            if (st == SH_EBUSY) {
                refused_at = before;
                break;
            }
            refused_at = UINT64_MAX;
            backlog.pop_front();
            if (st == SH_OK) {
                ticket[i] = tk;
                h_admit_ns[i] = clock_now_ns() - t0;
                outstanding.push_back(i);
            } else if (st == SH_ENOMEM) {
                h_admit_ns[i] = h_done_ns[i] = UINT64_MAX;
                ++finished;
            } else {
                return st;
            }
        }
        // scan the outstanding requests only when the server has finished some since the last
        // scan: the lock is the server thread's too
        const uint64_t done_now = s->completions.load(std::memory_order_acquire);
        if (!outstanding.empty() && done_now == seen)
            std::this_thread::yield();
        if (!outstanding.empty() && done_now != seen) {
            seen = done_now;
            std::lock_guard<std::mutex> g(s->mu);
            for (size_t j = 0; j < outstanding.size();) {
                const uint64_t i = outstanding[j];
                // a ticket of this driver expires only if millions of later requests finished
                // before it was scanned; it then counts as finished now
                const bool gone = ticket[i] < s->reqs_base;
                ServerReq *R = gone ? nullptr : &s->reqs[ticket[i] - s->reqs_base];
                const uint64_t td = gone ? clock_now_ns() : R->t_done;
                if (td) {
                    if (R)
                        R->read = true;
                    h_done_ns[i] = td - t0;
                    ++finished;
                    outstanding[j] = outstanding.back();
                    outstanding.pop_back();
                } else {
                    ++j;
                }
            }
        }
        if (s->error.load())
            return SH_EHIP;
    }
    return SH_OK;
}

sh_status_t sh_server_replay(sh_server_t *s, const sh_request_t *h_reqs,
                             const uint64_t *h_arrival_ns, uint64_t n, uint64_t *h_admit_ns,
                             uint64_t *h_done_ns)
{
    // the driver's bookkeeping grows with n; if it cannot, the call ends with SH_ENOMEM
    // (requests already submitted still run on the server)
    try {
        return replay_run(s, h_reqs, h_arrival_ns, n, h_admit_ns, h_done_ns);
    } catch (...) {
        return SH_ENOMEM;
    }
}

sh_status_t sh_server_stop(sh_server_t *s)
{
    if (!s)
        return SH_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_one();
    if (s->thr.joinable())
        s->thr.join();
    const int err = s->error.load();
    server_free(s);
    return err ? SH_EHIP : SH_OK;
}

} // extern "C"

// Slab hash for MI355X (gfx950, wave64): kernels and the C ABI declared in include/slabhash.h.
//
// Paper: Ashkiani, Farach-Colton, Owens, "A Dynamic Hash Table for the GPU".
//
// Memory layout of one table (one caller-owned device allocation, 256-byte aligned):
//   [header 256 B][B base slabs][P pool slabs][P/2048 bitmap rows of 256 B]
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
// Work sharing ("Our warp-cooperative work sharing strategy"): every lane holds one operation,
// and the whole wavefront processes the queued operations one at a time in lane order, with
// ballots and lane reads. Per chunk of 64 operations the kernel runs
//   pass 1: the base slabs of all 64 operations are loaded up front (32 two-slab loads), then
//           each operation is decided on its base slab in lane order. Searches and deletes that
//           resolve there finish; inserts and deletes that resolve there record a compare-and-
//           swap, and the chunk's swaps are issued together as one vector atomic.
//   pass 2: every operation not finished by pass 1 (chain continues, swap lost, new slab
//           needed) goes through the paper's loop (Fig. "Pseudocode for search, insert and
//           delete"): read slab, ballot, swap or follow the next index, allocate at the tail.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "slabhash.h"

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kEmptyPair = ~0ull;
constexpr uint64_t kTombPair = 0x00000000FFFFFFFFull; // key half all ones, value half 0
constexpr uint64_t kSlotMask = 0x7FFFFFFFull;         // slots 0..30 of a half wavefront
constexpr uint32_t kPrime = SH_HASH_PRIME;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr size_t kHeaderBytes = 256;
constexpr uint32_t kDefaultWavesPerCU = 16;

enum Kind { kSearch = 0, kInsert = 1, kDelete = 2, kMixed = 3 };

struct Header {
    uint32_t err;
    uint32_t violations;
    unsigned long long live, tomb, slabs, pool_alloc, dump_count;
};

struct View {
    uint64_t *base;   // B slabs of 32 words
    uint64_t *pool;   // P slabs of 32 words
    uint32_t *bitmap; // P/2048 rows of 64 words
    Header *hdr;
    uint32_t B, a, b, pool_slabs, nblk;
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

// Give lane `j` the wave-uniform value v, leaving other lanes' x unchanged.
__device__ __forceinline__ void put(uint32_t &x, uint32_t lane, uint32_t j, uint32_t v)
{
    x = (lane == j) ? v : x;
}

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

template <bool Coherent>
__device__ __forceinline__ uint64_t load_slot(const uint64_t *p)
{
    if constexpr (Coherent)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

__device__ __forceinline__ uint32_t load_word_coherent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t cas64(uint64_t *p, uint64_t expected, uint64_t desired)
{
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected; // the value found at p (equal to `expected` on success)
}

__device__ __forceinline__ uint32_t cas32(uint32_t *p, uint32_t expected, uint32_t desired)
{
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected;
}

// One lane (`who`) performs the swap; every lane gets the old value.
__device__ __forceinline__ uint64_t cas64_by(uint64_t *p, uint64_t expected, uint64_t desired,
                                             uint32_t lane, uint32_t who)
{
    uint64_t old = 0;
    if (lane == who)
        old = cas64(p, expected, desired);
    return ((uint64_t)rl((uint32_t)(old >> 32), who) << 32) | rl((uint32_t)old, who);
}

__device__ __forceinline__ void raise_error(const View &T, uint32_t bits, uint32_t lane,
                                            uint32_t who)
{
    if (lane == who)
        __hip_atomic_fetch_or(&T.hdr->err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// SlabAlloc for wave64 ("Dynamic memory allocation"). The pool is one contiguous array of
// blocks of 2048 slabs; a block's occupancy is one 256-byte bitmap row, which a wavefront holds
// in registers as one 32-bit word per lane (lane l covers slabs 32l .. 32l+31 of the block).
// The wavefront's "resident" block serves its allocations: lanes with a free bit vote, the
// lowest such lane claims its lowest free bit with an atomic OR on the row in memory and, if the
// bit was still free, broadcasts the slab index. A lost race refreshes that lane's word. When
// the resident block is full the wavefront moves to the next block, reading its row with one
// coalesced load; after a full cycle of blocks without success the pool counts as exhausted.

struct Alloc {
    uint32_t blk;   // resident block (wave-uniform), kEmpty = none yet
    uint32_t word;  // this lane's bitmap word of the resident block
    uint32_t moves; // block moves since the last successful allocation
    uint32_t start; // first block tried
    bool full;      // this wavefront found the pool exhausted
};

__device__ uint32_t wave_alloc(const View &T, Alloc &s, uint32_t lane)
{
    if (T.nblk == 0 || s.full)
        return kEmpty;
    if (s.blk == kEmpty) {
        s.blk = s.start % T.nblk;
        s.moves = 0;
        s.word = load_word_coherent(&T.bitmap[(size_t)s.blk * 64 + lane]);
    }
    for (;;) {
        const uint64_t free_lanes = ballot(s.word != kEmpty);
        if (free_lanes) {
            const uint32_t l = ffs0(free_lanes);
            uint32_t got = kEmpty;
            if (lane == l) {
                const uint32_t bit = (uint32_t)__builtin_ctz(~s.word);
                const uint32_t m = 1u << bit;
                const uint32_t old =
                    __hip_atomic_fetch_or(&T.bitmap[(size_t)s.blk * 64 + l], m,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s.word = old | m;
                if (!(old & m))
                    got = s.blk * SH_BLOCK_SLABS + l * 32 + bit;
            }
            const uint32_t idx = rl(got, l);
            if (idx != kEmpty) {
                s.moves = 0;
                return idx;
            }
            continue;
        }
        if (++s.moves > T.nblk) {
            s.full = true;
            return kEmpty;
        }
        s.blk = (s.blk + 1 == T.nblk) ? 0 : s.blk + 1;
        s.word = load_word_coherent(&T.bitmap[(size_t)s.blk * 64 + lane]);
    }
}

__device__ __forceinline__ void slab_free(const View &T, uint32_t idx)
{
    __hip_atomic_fetch_and(&T.bitmap[(size_t)(idx >> 11) * 64 + ((idx >> 5) & 63)],
                           ~(1u << (idx & 31)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------------------------
// The per-operation loop (pass 2). One queued operation at a time: the source lane's key is
// broadcast, the wavefront reads the current slab, votes for the key (and for empty slots when
// inserting), and either finishes, swaps, follows the next index, or allocates and links a new
// tail slab. `start` is kEmpty to begin at the base slab, else a pool slab index to resume at.

template <bool Coherent>
__device__ void wave_op(const View &T, Alloc &al, uint32_t lane, uint32_t op, uint32_t k,
                        uint32_t v, uint32_t bkt, uint32_t start, uint32_t &res_v,
                        uint32_t &res_s)
{
    const uint32_t slot = lane & 31;
    uint64_t *cur = (start == kEmpty) ? T.base + (size_t)bkt * 32 : T.pool + (size_t)start * 32;
    res_v = kEmpty;
    res_s = 0;
    for (;;) {
        const uint64_t w = load_slot<Coherent>(cur + slot);
        const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
        const uint64_t match = ballot(lo == k) & kSlotMask;
        const uint32_t next = rl(hi, 31);
        if (op == kSearch) {
            if (match) {
                res_v = rl(hi, ffs0(match));
                res_s = 1;
                return;
            }
        } else if (op == kDelete) {
            if (match) {
                const uint32_t d = ffs0(match);
                const uint64_t expect = ((uint64_t)rl(hi, d) << 32) | k;
                if (cas64_by(cur + d, expect, kTombPair, lane, 0) == expect) {
                    res_s = 1;
                    return;
                }
                continue; // the slot changed under us: read the same slab again
            }
        } else {
            uint32_t d = 32, st = 0;
            uint64_t expect = kEmptyPair;
            if (match) {
                d = ffs0(match);
                expect = ((uint64_t)rl(hi, d) << 32) | k;
                st = 2;
            } else {
                const uint64_t empty = ballot(w == kEmptyPair) & kSlotMask;
                if (empty) {
                    d = ffs0(empty);
                    st = 1;
                }
            }
            if (d < 32) {
                const uint64_t desired = ((uint64_t)v << 32) | k;
                if (cas64_by(cur + d, expect, desired, lane, 0) == expect) {
                    res_s = st;
                    return;
                }
                continue;
            }
            if (next == kEmpty) {
                // Tail slab is full: allocate, then link with a swap on the next index.
                const uint32_t idx = wave_alloc(T, al, lane);
                if (idx == kEmpty) {
                    raise_error(T, SH_ERR_POOL_EXHAUSTED, lane, 0);
                    return;
                }
                uint32_t *link = reinterpret_cast<uint32_t *>(cur + 31) + 1;
                uint32_t old = 0;
                if (lane == 0)
                    old = cas32(link, kEmpty, idx);
                old = rl(old, 0);
                if (old == kEmpty) {
                    cur = T.pool + (size_t)idx * 32;
                } else {
                    if (lane == 0)
                        slab_free(T, idx); // another wavefront linked first
                    cur = T.pool + (size_t)old * 32;
                }
                continue;
            }
        }
        if (next == kEmpty)
            return; // end of the list: not found / nothing to delete
        cur = T.pool + (size_t)next * 32;
    }
}

// ---------------------------------------------------------------------------------------------
// Operation kernel. Persistent grid: wavefront w takes chunks w, w + W, w + 2W, ... of 64 ops.

template <int K>
__global__ __launch_bounds__(kBlock) void ops_kernel(View T, const uint8_t *__restrict__ ops,
                                                     const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ vals,
                                                     uint64_t n, uint32_t *__restrict__ vout,
                                                     uint8_t *__restrict__ sout, uint32_t seq)
{
    constexpr bool kCoherent = (K != kSearch);
    const uint32_t lane = lane_id();
    const uint32_t half = lane >> 5, slot = lane & 31;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Alloc al;
    al.blk = kEmpty;
    al.word = 0;
    al.moves = 0;
    al.full = false;
    al.start = mix32(wave * 0x9E3779B9u + seq);

    const uint64_t nchunks = (n + 63) >> 6;
    for (uint64_t c = wave; c < nchunks; c += nwaves) {
        const uint64_t i = (c << 6) + lane;
        const bool in = i < n;
        const uint32_t key = in ? keys[i] : kEmpty;
        uint32_t val = 0;
        if constexpr (K == kInsert || K == kMixed)
            val = in ? vals[i] : 0;
        uint32_t op = (uint32_t)K;
        if constexpr (K == kMixed)
            op = in ? (uint32_t)ops[i] : 0u;
        const bool reserved = in && key == kEmpty;
        const uint64_t res_m = ballot(reserved);
        if (res_m)
            raise_error(T, SH_ERR_RESERVED_KEY, lane, ffs0(res_m));
        const bool act = in && !reserved && op <= 2;
        const uint32_t bkt = act ? bucket_of(key, T.a, T.b, T.B) : 0u;
        const uint64_t act_m = ballot(act);

        uint32_t rv = kEmpty, rs = 0; // this lane's results
        uint64_t pend = 0;            // ops left for pass 2
        uint32_t pnext = kEmpty;      // where pass 2 resumes (kEmpty = base slab)
        uint32_t cmode = 0, cslot = 0, cvobs = 0; // recorded swap: 1 insert, 2 replace, 3 delete

        // ---- pass 1: prefetch all 64 base slabs, two per load instruction ----
        uint64_t pre[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const uint32_t b0 = rl(bkt, 2 * q), b1 = rl(bkt, 2 * q + 1);
            const uint32_t bs = half ? b1 : b0;
            pre[q] = load_slot<kCoherent>(T.base + (size_t)bs * 32 + slot);
        }
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            if (!((act_m >> j) & 1))
                continue;
            const int h = (j & 1) * 32;
            const uint32_t lo = (uint32_t)pre[j >> 1], hi = (uint32_t)(pre[j >> 1] >> 32);
            const uint32_t kj = rl(key, j);
            const uint32_t oj = (K == kMixed) ? rl(op, j) : (uint32_t)K;
            const uint64_t match = (ballot(lo == kj) >> h) & kSlotMask;
            if (oj == kSearch) {
                if (match) {
                    put(rv, lane, j, rl(hi, ffs0(match) + h));
                    put(rs, lane, j, 1);
                } else {
                    const uint32_t nx = rl(hi, 31 + h);
                    if (nx != kEmpty) {
                        pend |= 1ull << j;
                        put(pnext, lane, j, nx);
                    }
                }
            } else if (oj == kDelete) {
                if (match) {
                    const uint32_t d = ffs0(match);
                    put(cmode, lane, j, 3);
                    put(cslot, lane, j, d);
                    put(cvobs, lane, j, rl(hi, d + h));
                } else {
                    const uint32_t nx = rl(hi, 31 + h);
                    if (nx != kEmpty) {
                        pend |= 1ull << j;
                        put(pnext, lane, j, nx);
                    }
                }
            } else {
                if (match) {
                    const uint32_t d = ffs0(match);
                    put(cmode, lane, j, 2);
                    put(cslot, lane, j, d);
                    put(cvobs, lane, j, rl(hi, d + h));
                } else {
                    const uint64_t empty = (ballot(pre[j >> 1] == kEmptyPair) >> h) & kSlotMask;
                    if (empty) {
                        put(cmode, lane, j, 1);
                        put(cslot, lane, j, ffs0(empty));
                    } else {
                        // Base slab full: continue down the chain, or allocate at the base.
                        pend |= 1ull << j;
                        put(pnext, lane, j, rl(hi, 31 + h));
                    }
                }
            }
        }
        if constexpr (K != kSearch) {
            // Commit the recorded swaps of the chunk together; losers redo the op in pass 2.
            bool lost = false;
            if (cmode) {
                uint64_t *sp = T.base + (size_t)bkt * 32 + cslot;
                const uint64_t expect =
                    (cmode == 1) ? kEmptyPair : (((uint64_t)cvobs << 32) | key);
                const uint64_t desired = (cmode == 3) ? kTombPair : (((uint64_t)val << 32) | key);
                if (cas64(sp, expect, desired) == expect)
                    rs = (cmode == 2) ? 2u : 1u;
                else
                    lost = true;
            }
            const uint64_t lost_m = ballot(lost);
            pend |= lost_m;
            if (lost)
                pnext = kEmpty;
        }

        // ---- pass 2: the remaining ops, one at a time in lane order ----
        while (pend) {
            const uint32_t j = ffs0(pend);
            pend &= pend - 1;
            uint32_t ov, os;
            wave_op<kCoherent>(T, al, lane, (K == kMixed) ? rl(op, j) : (uint32_t)K, rl(key, j),
                               rl(val, j), rl(bkt, j), rl(pnext, j), ov, os);
            put(rv, lane, j, ov);
            put(rs, lane, j, os);
        }

        if (in) {
            if (vout)
                vout[i] = rv;
            if (sout)
                sout[i] = (uint8_t)rs;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Structure walk: one wavefront per bucket (grid-stride). Counts live, deleted and slabs per
// bucket, checks the invariants the insertion rule guarantees, optionally emits live pairs.

__device__ __forceinline__ bool bitmap_has(const View &T, uint32_t idx)
{
    const uint32_t w = T.bitmap[(size_t)(idx >> 11) * 64 + ((idx >> 5) & 63)];
    return (w >> (idx & 31)) & 1u;
}

__global__ __launch_bounds__(kBlock) void walk_kernel(View T, uint32_t *__restrict__ dbkt,
                                                      uint32_t *__restrict__ dkey,
                                                      uint32_t *__restrict__ dval, uint64_t cap,
                                                      uint32_t *__restrict__ counts, int emit)
{
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
            const uint64_t E = ballot(w == kEmptyPair) & kSlotMask;
            const uint64_t L = ballot(lo != kEmpty) & kSlotMask;
            const uint64_t Tm = ballot(w == kTombPair) & kSlotMask;
            const uint64_t bad = ballot(lo == kEmpty && hi != kEmpty && hi != 0u) & kSlotMask;
            nl += __popcll(L);
            nt += __popcll(Tm);
            if (bad)
                ++viol;
            if (E && E != (kSlotMask & ~((1ull << ffs0(E)) - 1)))
                ++viol; // empty slots must form a suffix
            const uint32_t aux = rl(lo, 31), next = rl(hi, 31);
            if (aux != kEmpty)
                ++viol;
            if (emit && L) {
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
            if (E)
                ++viol; // a slab with a successor must be full
            if (next >= T.pool_slabs || !bitmap_has(T, next) || ns > T.pool_slabs) {
                ++viol;
                break;
            }
            cur = T.pool + (size_t)next * 32;
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

__global__ __launch_bounds__(kBlock) void popcount_kernel(View T)
{
    const size_t nw = (size_t)T.nblk * 64;
    unsigned long long c = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nw;
         i += (size_t)gridDim.x * kBlock)
        c += __popc(T.bitmap[i]);
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

} // namespace

// ---------------------------------------------------------------------------------------------
// Host side

struct sh_table {
    sh_params_t p;
    char *storage;
    size_t bytes;
    View v;
    uint32_t seq;
    uint32_t waves_per_cu;
    int num_cu;
};

namespace {

struct Layout {
    size_t base, pool, bitmap, total;
};

bool layout_of(const sh_params_t *p, Layout *L)
{
    if (!p || p->num_buckets == 0 || p->pool_slabs % SH_BLOCK_SLABS != 0 || p->hash_a == 0 ||
        p->hash_a >= kPrime || p->hash_b >= kPrime)
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

uint32_t grid_for(const sh_table *t, uint64_t n)
{
    const uint64_t chunks = (n + 63) / 64;
    uint64_t waves = (uint64_t)t->num_cu * t->waves_per_cu;
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
    hipLaunchKernelGGL(ops_kernel<K>, dim3(grid_for(t, n)), dim3(kBlock), 0, S(stream), t->v,
                       ops, keys, vals, n, vout, sout, t->seq++);
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
    hipLaunchKernelGGL(walk_kernel, dim3(blocks), dim3(kBlock), 0, S(stream), t->v, dbkt, dkey,
                       dval, cap, counts, emit);
    if (check_launch() != SH_OK)
        return SH_EHIP;
    if (t->v.nblk) {
        uint32_t pb = (uint32_t)(((size_t)t->v.nblk * 64 + kBlock - 1) / kBlock);
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
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return SH_EHIP;
    sh_table *t = static_cast<sh_table *>(calloc(1, sizeof(sh_table)));
    if (!t)
        return SH_ENOMEM;
    t->p = *p;
    t->storage = static_cast<char *>(d_storage);
    t->bytes = bytes;
    t->num_cu = ncu > 0 ? ncu : 1;
    t->waves_per_cu = kDefaultWavesPerCU;
    t->seq = 0;
    t->v.hdr = reinterpret_cast<Header *>(t->storage);
    t->v.base = reinterpret_cast<uint64_t *>(t->storage + L.base);
    t->v.pool = reinterpret_cast<uint64_t *>(t->storage + L.pool);
    t->v.bitmap = reinterpret_cast<uint32_t *>(t->storage + L.bitmap);
    t->v.B = p->num_buckets;
    t->v.a = p->hash_a;
    t->v.b = p->hash_b;
    t->v.pool_slabs = p->pool_slabs;
    t->v.nblk = p->pool_slabs / SH_BLOCK_SLABS;
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
    return launch_init(t, stream);
}

sh_status_t sh_destroy(sh_table_t *t)
{
    if (!t)
        return SH_EINVAL;
    free(t);
    return SH_OK;
}

sh_status_t sh_set_launch(sh_table_t *t, const sh_launch_t *shape)
{
    if (!t)
        return SH_EINVAL;
    if (!shape || shape->waves_per_cu == 0) {
        t->waves_per_cu = kDefaultWavesPerCU;
        return SH_OK;
    }
    if (shape->waves_per_cu > 64)
        return SH_EINVAL;
    t->waves_per_cu = shape->waves_per_cu;
    return SH_OK;
}

sh_status_t sh_build(sh_table_t *t, const uint32_t *d_keys, const uint32_t *d_vals, uint64_t n,
                     uint8_t *d_status, void *stream)
{
    if (n && !d_vals)
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
    if (n && (!d_ops || !d_vals_in || !d_vals_out || !d_status))
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
    if (hipMemcpyAsync(&h, t->v.hdr, sizeof(Header), hipMemcpyDeviceToHost, S(stream)) !=
            hipSuccess ||
        hipStreamSynchronize(S(stream)) != hipSuccess)
        return SH_EHIP;
    memset(h_out, 0, sizeof(*h_out));
    h_out->live = h.live;
    h_out->tombstones = h.tomb;
    h_out->slabs_total = h.slabs;
    h_out->pool_allocated = h.pool_alloc;
    h_out->pool_capacity = t->p.pool_slabs;
    h_out->error_word = h.err;
    h_out->violations = h.violations;
    h_out->num_buckets = t->p.num_buckets;
    h_out->hash_a = t->p.hash_a;
    h_out->hash_b = t->p.hash_b;
    h_out->hash_p = kPrime;
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

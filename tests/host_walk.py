"""Host-side reading of a table's raw device storage, independent of the library's own structure
walk: the storage tensor is copied to the host and its slab lists are followed in numpy.

Storage layout (one allocation): a 4 KB header, B base slabs, P pool slabs, then P / 2048 bitmap
rows of 64 32-bit words (bit b of word l of row r covers pool slab 2048 r + 32 l + b). A slab is
32 eight-byte words: words 0..30 are slots (key in the low half, value in the high half); word
31 holds the auxiliary half and, in its high half, the next pool slab (0xFFFFFFFF = none).

check_structure() asserts, in this order, the invariants that hold whenever no operation is in
flight, so a failure names the first one broken:
  1. every next index is inside the pool and every list ends (no cycle);
  2. no pool slab is referenced twice (by two lists, or twice by one);
  3. every referenced pool slab is marked allocated;
  4. every allocated pool slab is referenced (no slab leaked by a lost link race);
  5. every free pool slab is all ones (an allocation may hand it out without clearing it);
  6. the allocator's set bits equal the sum over buckets of (slabs - 1).
It returns per-bucket (live, tombstones, slabs) as numpy arrays."""
import numpy as np

HEADER = 4096
SLAB = 256
BLOCK = 2048
EMPTY32 = 0xFFFFFFFF
EMPTY64 = np.uint64(0xFFFFFFFFFFFFFFFF)
TOMB64 = np.uint64(0x00000000FFFFFFFF)


SUPER_SHIFT = 27


def super_slabs(nbytes):
    """Slabs of a super block registered with `nbytes` bytes: the most whole blocks whose slabs
    and bitmap rows fit, at most 2^27 - 2048 slabs."""
    return min(nbytes // (BLOCK * SLAB + 256), (1 << SUPER_SHIFT) // BLOCK - 1) * BLOCK


def raw_parts(t, supers=()):
    """(base [B,32] u64, pools, bitmaps) of a table with its own storage, copied from the device:
    pools[s] [P_s, 32] u64 and bitmaps[s] [P_s/2048, 64] u32 for super block s (0 = the table's
    own pool, then the device tensors in `supers` in registration order)."""
    B, P = int(t.params.num_buckets), int(t.params.pool_slabs)
    raw = t.storage.cpu().numpy()
    o_pool = HEADER + B * SLAB
    o_bm = o_pool + P * SLAB
    base = raw[HEADER:o_pool].view(np.uint64).reshape(B, 32)
    pools = [raw[o_pool:o_bm].view(np.uint64).reshape(P, 32)]
    bms = [raw[o_bm:o_bm + (P // BLOCK) * 256].view(np.uint32).reshape(-1, 64)]
    for mem in supers:
        r = mem.cpu().numpy()
        n = super_slabs(r.size)
        pools.append(r[:n * SLAB].view(np.uint64).reshape(n, 32))
        bms.append(r[n * SLAB:n * SLAB + (n // BLOCK) * 256].view(np.uint32).reshape(-1, 64))
    return base, pools, bms


def _counts(rows, keys_only):
    """Live and tombstone entries of slab rows [n, 32] (slots 0..30)."""
    w = rows[:, :31]
    if keys_only:
        lo = (w & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        hi = (w >> np.uint64(32)).astype(np.uint32)
        live = ((lo != EMPTY32) & (lo != 0xFFFFFFFE)).sum(1) + \
            ((hi != EMPTY32) & (hi != 0xFFFFFFFE)).sum(1)
        tomb = (lo == 0xFFFFFFFE).sum(1) + (hi == 0xFFFFFFFE).sum(1)
    else:
        key = (w & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        live = (key != EMPTY32).sum(1)
        tomb = (w == TOMB64).sum(1)
    return live.astype(np.int64), tomb.astype(np.int64)


def check_structure(t, keys_only=False, supers=None):
    """Pool slab addresses carry their super block in the top 5 bits (0 = the table's own
    pool); `supers` defaults to the table's registered super blocks (t.supers)."""
    if supers is None:
        supers = getattr(t, "supers", [])
    base, pools, bms = raw_parts(t, supers)
    B = base.shape[0]
    sizes = np.array([p.shape[0] for p in pools], np.int64)
    first = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    pool = np.concatenate(pools) if len(pools) > 1 else pools[0]
    P = pool.shape[0]

    def flat(addr):
        """Global row of each pool address (-1 if it names no registered slab)."""
        sb = (addr >> np.uint32(SUPER_SHIFT)).astype(np.int64)
        i = (addr & np.uint32((1 << SUPER_SHIFT) - 1)).astype(np.int64)
        ok = (sb < sizes.size)
        ok[ok] &= i[ok] < sizes[sb[ok]]
        out = np.full(addr.shape, -1, np.int64)
        out[ok] = first[sb[ok]] + i[ok]
        return out

    live, tomb = _counts(base, keys_only)
    slabs = np.ones(B, np.int64)
    refs = np.zeros(P, np.int64)
    nxt = (base[:, 31] >> np.uint64(32)).astype(np.uint32)
    owner = np.arange(B)
    depth = 0
    while True:
        on = nxt != EMPTY32
        if not on.any():
            break
        idx = flat(nxt[on])
        assert (idx >= 0).all(), "1: a next index points outside the pool (bucket %d)" % \
            int(owner[on][idx < 0][0])
        depth += 1
        assert depth <= P, "1: a slab list does not end"
        np.add.at(refs, idx, 1)
        rows = pool[idx]
        l, d = _counts(rows, keys_only)
        b_on = owner[on]
        np.add.at(live, b_on, l)
        np.add.at(tomb, b_on, d)
        np.add.at(slabs, b_on, 1)
        owner = b_on
        nxt = (rows[:, 31] >> np.uint64(32)).astype(np.uint32)
    bits = np.concatenate([
        np.unpackbits(bm.reshape(-1).view(np.uint8), bitorder="little").astype(bool)[:n]
        for bm, n in zip(bms, sizes)])
    assert refs.max(initial=0) <= 1, "2: pool slab row %d is referenced %d times" % (
        int(refs.argmax()), int(refs.max()))
    ref = refs == 1
    bad = np.flatnonzero(ref & ~bits)
    assert bad.size == 0, "3: pool slab %d is in a list but marked free" % int(bad[0])
    bad = np.flatnonzero(bits & ~ref)
    assert bad.size == 0, "4: pool slab %d is allocated but in no list (%d such)" % (
        int(bad[0]), bad.size)
    free_rows = pool[~bits]
    bad = np.flatnonzero((free_rows != EMPTY64).any(1))
    assert bad.size == 0, "5: free pool slab %d is not empty" % int(np.flatnonzero(~bits)[bad[0]])
    assert int(bits.sum()) == int((slabs - 1).sum()), "6: allocator bits != sum(slabs - 1)"
    return live, tomb, slabs

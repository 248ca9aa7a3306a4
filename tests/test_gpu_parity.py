"""GPU parity: the HIP slab hash (through the C ABI) against the CPU oracle on the same seeded
inputs. Integer results must match bit for bit; concurrent mixed batches must be linearizable
against the oracle with an identical final table."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import host_walk as HW
import linearize as LZ

pytestmark = pytest.mark.gpu

M = S.SH_SLAB_PAIRS
EMPTY = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def make(oracle_mod, B, a, b, pool):
    t = S.SlabHash(B, pool, a, b)
    o = oracle_mod.Oracle(B, M, a, b, pool_slabs=None)
    return t, o


def assert_same_table(t, o, check_counts=True):
    b, k, v, counts, viol = t.dump()
    if getattr(t, "storage", None) is not None:
        # the raw storage read on the host: lists, allocator bits and free slabs, and the
        # library walk's per-bucket counts against it
        ko = bool(t.params.flags & S.SH_TABLE_KEYS_ONLY)
        h_live, h_tomb, h_slabs = HW.check_structure(t, keys_only=ko)
        assert (counts[:, 0] == h_live).all() and (counts[:, 1] == h_tomb).all()
        assert (counts[:, 2] == h_slabs).all()
    assert viol == 0, "structure invariant violated"
    ob, ok, ov = o.dump()
    order = np.lexsort((ov, ok, ob))  # the live multiset: equal keys may sit in any order
    assert b.size == ob.size
    assert (b == ob[order]).all() and (k == ok[order]).all() and (v == ov[order]).all()
    st = t.stats()
    if check_counts:
        live, tomb, slabs = o.bucket_stats()
        assert (counts[:, 0] == live).all()
        assert (counts[:, 1] == tomb).all()
        assert (counts[:, 2] == slabs).all()
        assert st["pool_allocated"] == o.pool_used == int((slabs - 1).sum())
        assert st["slabs_total"] == o.total_slabs
    assert st["live"] == ob.size and st["violations"] == 0
    return st


def search_both(t, o, q_np):
    v, f = t.search(S.to_dev(q_np))
    ov, of, _ = o.search(q_np)
    gv, gf = S.to_host_u32(v), f.cpu().numpy()
    assert (gf == of).all(), "found flags differ"
    assert (gv == ov).all(), "values differ"


def test_config1_phased(oracle_mod):
    """2^16 keys into 2^12 buckets, 2^16 searches half present, delete 25%, search again."""
    say("case: config1 seed=1 n=65536 B=4096")
    wl = W.phased(seed=1, n=1 << 16, n_queries=1 << 16, hit_fraction=0.5,
                  delete_fraction=0.25, prime=S.SH_HASH_PRIME)
    B = 1 << 12
    t, o = make(oracle_mod, B, wl.hash_a, wl.hash_b, S.pool_slabs_bound(1 << 16))
    st = t.build(S.to_dev(wl["keys"]), S.to_dev(wl["vals"]))
    assert (st.cpu().numpy() == o.replace(wl["keys"], wl["vals"])).all()
    search_both(t, o, wl["queries"])
    ds = t.delete(S.to_dev(wl["deletes"]))
    assert (ds.cpu().numpy() == o.delete(wl["deletes"])).all()
    search_both(t, o, wl["queries"])
    st = assert_same_table(t, o)
    assert st["error_word"] == 0 and st["tombstones"] == wl["deletes"].size


@pytest.mark.parametrize("n", [1, 2, 31, 63, 64, 65, 127, 129, 1000, 4097, 20011])
def test_ragged_sizes(oracle_mod, n):
    say("case: ragged n=%d B=97" % n)
    rng = W.SplitMix64(n)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, n)
    vals = W.value_of(keys)
    miss = W.unique_keys(rng, n, exclude=keys)
    t, o = make(oracle_mod, 97, a, b, S.pool_slabs_bound(n))
    st = t.build(S.to_dev(keys), S.to_dev(vals))
    assert (st.cpu().numpy() == o.replace(keys, vals)).all()
    search_both(t, o, np.concatenate([keys, miss]))
    half = keys[: (n + 1) // 2]
    ds = t.delete(S.to_dev(half))
    assert (ds.cpu().numpy() == o.delete(half)).all()
    search_both(t, o, np.concatenate([miss, keys]))
    # replace existing values (status 2) and re-insert deleted keys (status 1, appended)
    newv = (vals ^ np.uint32(0x5A5A5A5A)).astype(np.uint32)
    st = t.insert(S.to_dev(keys), S.to_dev(newv))
    assert (st.cpu().numpy() == o.replace(keys, newv)).all()
    search_both(t, o, keys)
    assert_same_table(t, o)


@pytest.mark.parametrize("opw", [8, 16, 32, 64])
def test_every_chunk_width(oracle_mod, opw):
    """Each chunk width, with a ragged last chunk: lanes past a chunk's end hold no op and must
    touch nothing. (A 32-op chunk once let lanes 32..63 act whenever op 31 was pending; their
    default key and value then filled bucket 0's list with (EMPTY, 0) pairs.)"""
    say("case: chunk width %d" % opw)
    n = 37 * 64 + 33
    rng = W.SplitMix64(700 + opw)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, 2 * n)
    ins, extra = keys[:n], keys[n:]
    t, o = make(oracle_mod, 61, a, b, S.pool_slabs_bound(3 * n))
    t.set_launch(0, opw)
    st = t.build(S.to_dev(ins), S.to_dev(W.value_of(ins)))
    assert (st.cpu().numpy() == o.replace(ins, W.value_of(ins))).all()
    assert_same_table(t, o)
    search_both(t, o, keys)
    gone = ins[::3]
    assert (t.delete(S.to_dev(gone)).cpu().numpy() == o.delete(gone)).all()
    assert_same_table(t, o)
    present = np.setdiff1d(ins, gone)
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(n, W.GAMMAS["gamma1"])
    ops, mk, mv = W.mixed_batch(rng, present, extra[:n_ins], extra[n_ins:], n_ins, n_del, n_hit,
                                n_miss)
    pre_v, pre_f, _ = o.search(mk)
    gv, gs = t.mixed(S.to_dev(ops), S.to_dev(mk), S.to_dev(mv))
    ov, ost = o.mixed(ops, mk, mv)
    post_v, post_f, _ = o.search(mk)
    LZ.check_single_mutation_batch(ops, mk, S.to_host_u32(gv), gs.cpu().numpy(), pre_f, pre_v,
                                   post_f, post_v, ost)
    st = assert_same_table(t, o)
    assert st["tombstones"] == int(o.bucket_stats()[1].sum())


def test_launch_shape_reports_the_shape_used():
    """The shape query follows sh_set_launch and the per-kind defaults: a set shape is reported
    as set; by default small batches get the smallest chunk (whose kernel fits at least as many
    wavefronts per CU as the largest), default grids never exceed 20 wavefronts per CU, and bad
    arguments are refused."""
    t = S.SlabHash(97, 2048, 3, 5)
    kinds = (S.SH_OP_SEARCH, S.SH_OP_INSERT, S.SH_OP_DELETE, S.SH_KIND_MIXED)
    for kind in kinds:
        w, c = t.launch_shape(kind, 1 << 22)
        assert 1 <= w <= 20 and c in (8, 16, 32, 64)
        w8, c8 = t.launch_shape(kind, 100)
        assert c8 == 8 and w <= w8 <= 20
    t.set_launch(12, 32)
    assert all(t.launch_shape(k, n) == (12, 32) for k in kinds for n in (1, 1 << 22))
    t.set_launch()
    assert t.launch_shape(S.SH_OP_INSERT, 100)[1] == 8
    with pytest.raises(S.SlabHashError):
        t.launch_shape(4, 10)
    with pytest.raises(S.SlabHashError):
        t.launch_shape(-1, 10)


@pytest.mark.parametrize("dup,ko", [(False, False), (True, False), (False, True)])
def test_reset_restores_the_initial_storage(oracle_mod, dup, ko):
    """After inserts, deletes, a FLUSH and slabs taken through the allocator alone, a reset
    leaves the storage byte for byte as a fresh table's initialisation does, and the table
    works again."""
    say("case: reset, duplicates=%s keys_only=%s" % (dup, ko))
    rng = W.SplitMix64(1401)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n, B = 50000, 61
    pool = S.pool_slabs_bound(3 * n)
    fresh = S.SlabHash(B, pool, a, b, duplicates=dup, keys_only=ko)
    t = S.SlabHash(B, pool, a, b, duplicates=dup, keys_only=ko)
    keys = W.unique_keys(rng, n)
    keys = keys[keys != np.uint32(0xFFFFFFFE)]
    dev = lambda x: None if ko else S.to_dev(W.value_of(x))
    t.insert(S.to_dev(keys), dev(keys))
    t.delete(S.to_dev(keys[::3]))
    t.flush()
    t.insert(S.to_dev(keys[::3]), dev(keys[::3]))
    spare = torch.empty(100, dtype=torch.int32, device="cuda")
    S.sh_alloc_slabs(t.handle, 100, spare)       # allocated, in no list
    assert t.stats()["pool_allocated"] > 100
    t.reset()
    torch.cuda.synchronize()
    assert torch.equal(t.storage, fresh.storage)
    o = oracle_mod.Oracle(B, 62 if ko else M, a, b, duplicates=dup)
    t.insert(S.to_dev(keys), dev(keys))
    o.replace(keys, keys if ko else W.value_of(keys))
    assert_same_table(t, o)


def test_empty_calls_are_noops(oracle_mod):
    say("case: empty inputs")
    t, o = make(oracle_mod, 16, 3, 5, 0)
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
    S.sh_build(t.handle, e32, e32, e8)
    S.sh_search(t.handle, e32, e32, e8)
    S.sh_delete(t.handle, e32, e8)
    S.sh_mixed(t.handle, e8, e32, e32, e32, e8)
    st = assert_same_table(t, o)
    assert st["live"] == 0 and st["slabs_total"] == 16 and st["pool_allocated"] == 0


@pytest.mark.parametrize("B,n", [(1, 3000), (4, 20000), (61, 50000)])
def test_long_chains_and_contention(oracle_mod, B, n):
    """Few buckets: long slab lists, many wavefronts racing on the same tail slabs."""
    say("case: contention B=%d n=%d" % (B, n))
    rng = W.SplitMix64(77 + B)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, n)
    vals = W.value_of(keys)
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(n))
    st = t.insert(S.to_dev(keys), S.to_dev(vals))
    assert (st.cpu().numpy() == o.replace(keys, vals)).all()
    search_both(t, o, keys[::3])
    dels = keys[1::4]
    ds = t.delete(S.to_dev(dels))
    assert (ds.cpu().numpy() == o.delete(dels)).all()
    search_both(t, o, keys)
    assert_same_table(t, o)


def test_duplicate_keys_in_one_batch(oracle_mod):
    """Repeated keys in one insert batch: one insert wins as new (status 1), the rest replace
    (status 2), and the final value is one of the batch's values for that key."""
    say("case: duplicates")
    rng = W.SplitMix64(5)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    base = W.unique_keys(rng, 3000)
    keys = base[rng.below(20000, base.size)].astype(np.uint32)
    vals = (rng.next(20000) >> np.uint64(32)).astype(np.uint32)
    t = S.SlabHash(29, S.pool_slabs_bound(20000), a, b)
    st = t.insert(S.to_dev(keys), S.to_dev(vals)).cpu().numpy()
    uk = np.unique(keys)
    ones = np.bincount(np.searchsorted(uk, keys), weights=(st == 1)).astype(int)
    assert (ones == 1).all() and ((st == 1) | (st == 2)).all()
    bb, kk, vv, counts, viol = t.dump()
    assert viol == 0 and (np.sort(kk) == uk).all()
    allowed = set(zip(keys.tolist(), vals.tolist()))
    assert all((k, v) in allowed for k, v in zip(kk.tolist(), vv.tolist()))
    assert t.stats()["live"] == uk.size


def test_reserved_key_flagged(oracle_mod):
    say("case: reserved key")
    t, o = make(oracle_mod, 8, 11, 13, S.pool_slabs_bound(100))
    keys = np.array([1, 2, EMPTY, 3, EMPTY], np.uint32)
    vals = np.array([10, 20, 30, 40, 50], np.uint32)
    st = t.insert(S.to_dev(keys), S.to_dev(vals)).cpu().numpy()
    assert (st == o.replace(keys, vals)).all() and st.tolist() == [1, 1, 0, 1, 0]
    v, f = t.search(S.to_dev(keys))
    assert f.cpu().numpy().tolist() == [1, 1, 0, 1, 0]
    assert S.to_host_u32(v).tolist() == [10, 20, EMPTY, 40, EMPTY]
    assert t.stats()["error_word"] & S.SH_ERR_RESERVED_KEY
    assert_same_table(t, o)


def test_pool_exhaustion(oracle_mod):
    """A pool of one block: inserts beyond its capacity fail with status 0 and the error bit;
    nothing that reported success is lost and nothing that failed is present."""
    say("case: pool exhaustion")
    B, pool = 8, 2048
    rng = W.SplitMix64(31337)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n = (B + pool) * M + 4000
    keys = W.unique_keys(rng, n)
    vals = W.value_of(keys)
    t = S.SlabHash(B, pool, a, b)
    st = t.insert(S.to_dev(keys), S.to_dev(vals)).cpu().numpy()
    assert set(np.unique(st).tolist()) <= {0, 1}
    assert (st == 0).sum() >= 4000 - B * M
    s = t.stats()
    assert s["error_word"] & S.SH_ERR_POOL_EXHAUSTED
    assert s["pool_allocated"] == pool and s["violations"] == 0
    v, f = t.search(S.to_dev(keys))
    f = f.cpu().numpy()
    assert (f == (st == 1)).all()
    assert (S.to_host_u32(v)[st == 1] == vals[st == 1]).all()
    assert s["live"] == int((st == 1).sum())


def _grow_and_mix(oracle_mod, n_keys, B, n_batches, batch, seed, gamma=(0.2, 0.2, 0.3, 0.3)):
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, n_keys)
    vals = W.value_of(keys)
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(batch, gamma)
    fresh = W.unique_keys(rng, n_ins * n_batches + n_miss, exclude=keys)
    absent = fresh[n_ins * n_batches:]
    pool = S.pool_slabs_bound(n_keys + n_ins * n_batches)
    t, o = make(oracle_mod, B, a, b, pool)
    # incremental growth in batches
    g = 1 << 16
    for s in range(0, n_keys, g):
        st = t.insert(S.to_dev(keys[s:s + g]), S.to_dev(vals[s:s + g]))
        assert (st.cpu().numpy() == 1).all()
    o.replace(keys, vals)
    present = keys.copy()
    for bi in range(n_batches):
        ops, bk, bv = W.mixed_batch(rng, present, fresh[bi * n_ins:(bi + 1) * n_ins], absent,
                                    n_ins, n_del, n_hit, n_miss)
        pre_v, pre_f, _ = o.search(bk)
        gv, gs = t.mixed(S.to_dev(ops), S.to_dev(bk), S.to_dev(bv))
        ov, ost = o.mixed(ops, bk, bv)
        post_v, post_f, _ = o.search(bk)
        LZ.check_single_mutation_batch(ops, bk, S.to_host_u32(gv), gs.cpu().numpy(), pre_f,
                                       pre_v, post_f, post_v, ost)
        dels = bk[ops == 2]
        present = np.concatenate([present[~np.isin(present, dels)], bk[ops == 1]])
    return t, o


def test_mixed_batches_linearizable(oracle_mod):
    say("case: mixed 2^18 keys, 4 batches of 2^16")
    t, o = _grow_and_mix(oracle_mod, 1 << 18, (1 << 18) // 20, 4, 1 << 16, seed=3)
    assert_same_table(t, o)


def test_mixed_with_repeated_keys_linearizable(oracle_mod):
    """Many mutations per key in one batch, on a few buckets: the general per-key check."""
    say("case: mixed repeated keys")
    rng = W.SplitMix64(12)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    dom = W.unique_keys(rng, 400)
    t, o = make(oracle_mod, 7, a, b, S.pool_slabs_bound(20000))
    init = dom[:200]
    t.insert(S.to_dev(init), S.to_dev(W.value_of(init)))
    o.replace(init, W.value_of(init))
    for it in range(3):
        n = 2000
        ops = rng.below(n, 3).astype(np.uint8)
        keys = dom[rng.below(n, dom.size)].astype(np.uint32)
        # at most 6 mutations of any key, so the brute-force order search stays small
        mut_keys = keys[ops != 0]
        uk, cnt = np.unique(mut_keys, return_counts=True)
        over = np.isin(keys, uk[cnt > 6]) & (ops != 0)
        ops[over] = 0
        vals = (rng.next(n) >> np.uint64(32)).astype(np.uint32)
        _, ok_, ov_ = o.dump()
        pre = LZ.state_lookup(ok_, ov_)
        gv, gs = t.mixed(S.to_dev(ops), S.to_dev(keys), S.to_dev(vals))
        tb, tk, tv, _, viol = t.dump()
        assert viol == 0
        post = LZ.state_lookup(tk, tv)
        LZ.check_batch(ops, keys, vals, S.to_host_u32(gv), gs.cpu().numpy(), pre, post)
        # keys not in the batch keep their state
        untouched = np.setdiff1d(ok_, keys)
        assert all(post(int(k)) == pre(int(k)) for k in untouched)
        # continue from the GPU's state: rebuild the oracle from its dump
        o = oracle_mod.Oracle(7, M, a, b)
        o.replace(tk, tv)


def test_lost_links_leave_free_slabs_empty(oracle_mod):
    """Many wavefronts growing the same four lists at once lose link races; each loser has
    already put its pair into slot 0 of its new slab, and must take it out before freeing the
    slab. Every pool slab the bitmaps mark free must then be all ones, as the reset and the
    allocator assume, and the table must equal the oracle's."""
    say("case: lost links, B=4, n=100000")
    rng = W.SplitMix64(1501)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n, B = 100000, 4
    pool = S.pool_slabs_bound(n)
    t = S.SlabHash(B, pool, a, b)
    o = oracle_mod.Oracle(B, M, a, b)
    S.sh_set_launch(t.handle, 0, 0, S.SH_LAUNCH_COUNTERS)
    keys = W.unique_keys(rng, n)
    st = t.insert(S.to_dev(keys), S.to_dev(W.value_of(keys)))
    assert (st.cpu().numpy() == o.replace(keys, W.value_of(keys))).all()
    stats = assert_same_table(t, o)
    assert stats["link_lost"] > 0, "no link race happened; the case tests nothing"
    torch.cuda.synchronize()
    raw = t.storage.view(torch.uint8).cpu().numpy()
    base = 4096
    pool_at = base + B * 256
    bitmap_at = pool_at + pool * 256
    words = raw[bitmap_at:bitmap_at + (pool // 2048) * 256].view(np.uint32)
    # slab 2048 r + 32 w + bit is marked by bit `bit` of word 64 r + w
    allocated = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1).astype(bool)
    assert int(allocated.sum()) == stats["pool_allocated"]
    slabs = raw[pool_at:bitmap_at].reshape(pool, 256)
    free_dirty = np.flatnonzero(~allocated & (slabs != 0xFF).any(axis=1))
    assert free_dirty.size == 0, "free pool slabs holding data: %s" % free_dirty[:8]


@pytest.mark.parametrize("B", [1, 3])
def test_boundary_keys_and_values(oracle_mod, B):
    """Keys at the edges of their range (0, 1, the largest valid key, the keys at and above p,
    which alias to 0..3 in the hash) with values that share a half with the empty and deleted
    codes (all ones, 0), among ordinary pairs, on one or three buckets so that lists run over
    several slabs: inserts, searches, replaces, deletes, re-inserts and a mixed batch all match
    the oracle."""
    say("case: boundary keys and values, B=%d" % B)
    p = S.SH_HASH_PRIME
    # p + 3 = 0xFFFFFFFE is the largest valid key; every key appears once (the statuses of
    # repeated keys in one batch depend on the schedule, and another test covers them)
    edge = np.unique(np.array([0, 1, 2, 3, p - 1, p, p + 1, p + 2, p + 3, 0x7FFFFFFF,
                               0x80000000], np.uint64)).astype(np.uint32)
    rng = W.SplitMix64(1501)
    a, b = W.hash_params(rng, p)
    other = W.unique_keys(rng, 400)
    other = other[~np.isin(other, edge)]
    keys = np.concatenate([edge, other])
    vals = W.value_of(keys)
    vals[0::3] = 0xFFFFFFFF                     # value half of the empty code
    vals[1::3] = 0                              # value half of the deleted code
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(4 * keys.size))
    order = rng.permutation(keys.size)
    st = t.insert(S.to_dev(keys[order]), S.to_dev(vals[order])).cpu().numpy()
    assert (st == o.replace(keys[order], vals[order])).all()
    absent = W.unique_keys(rng, 200)
    absent = absent[~np.isin(absent, keys)]
    search_both(t, o, np.concatenate([keys, absent]))
    # replace every edge key's value with all ones, then delete half the keys and re-insert some
    rv = np.full(edge.size, 0xFFFFFFFF, np.uint32)
    st = t.insert(S.to_dev(edge), S.to_dev(rv)).cpu().numpy()
    assert (st == o.replace(edge, rv)).all() and (st == 2).all()
    dk = keys[order[: keys.size // 2]]
    ds = t.delete(S.to_dev(dk)).cpu().numpy()
    assert (ds == o.delete(dk)).all() and (ds == 1).all()
    back = dk[::2]
    bv = np.zeros(back.size, np.uint32)
    st = t.insert(S.to_dev(back), S.to_dev(bv)).cpu().numpy()
    assert (st == o.replace(back, bv)).all() and (st == 1).all()
    search_both(t, o, np.concatenate([keys, absent]))
    # a mixed batch over the same keys: each key appears once, so the outcome is exact
    mk = np.concatenate([keys, absent[:50]])
    ops = np.zeros(mk.size, np.uint8)
    live = ~np.isin(mk, dk[1::2])                # keys present now
    ops[:keys.size][live[:keys.size] & (np.arange(keys.size) % 3 == 0)] = S.SH_OP_DELETE
    ops[keys.size:] = S.SH_OP_INSERT             # fresh keys
    ops[:keys.size][~live[:keys.size]] = S.SH_OP_INSERT  # deleted keys come back
    mv = W.value_of(mk)
    mv[::2] = 0xFFFFFFFF
    vo = torch.empty(mk.size, dtype=torch.int32, device="cuda")
    so = torch.empty(mk.size, dtype=torch.uint8, device="cuda")
    S.sh_mixed(t.handle, S.to_dev(ops), S.to_dev(mk), S.to_dev(mv), vo, so)
    g_st, g_v = so.cpu().numpy(), S.to_host_u32(vo)
    for i in range(mk.size):
        k = mk[i:i + 1]
        if ops[i] == S.SH_OP_INSERT:
            assert g_st[i] == o.replace(k, mv[i:i + 1])[0]
        elif ops[i] == S.SH_OP_DELETE:
            assert g_st[i] == o.delete(k)[0]
        else:
            ov, of, _ = o.search(k)
            assert g_st[i] == of[0] and (not of[0] or g_v[i] == ov[0])
    assert_same_table(t, o)
    search_both(t, o, np.concatenate([keys, absent]))

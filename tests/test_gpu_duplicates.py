"""GPU parity of the multiset operations ("Supported Operations": INSERT, DELETE with duplicates,
DELETEALL, SEARCH, SEARCHALL) against the oracle. Where concurrency leaves a choice (which
empty slot a concurrent insert takes, which of several equal keys comes first in a list filled
by one batch), the tests compare what is unique: the live multiset, per-bucket counts, counts
per key; list order is checked where it is determined (copies inserted one per batch)."""
import sys
from collections import Counter

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import dup_cases
import host_walk as HW
from test_gpu_parity import M, assert_same_table

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def make_dup(oracle_mod, B, pool, seed):
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, pool, a, b, duplicates=True)
    o = oracle_mod.Oracle(B, M, a, b, duplicates=True)
    return t, o, rng


def per_key_sum(keys, status):
    c = Counter()
    for k, s in zip(keys.tolist(), status.tolist()):
        c[k] += int(s)
    return c


@pytest.mark.parametrize("B,domain", [(1, 300), (61, 5000), (4099, 1 << 18)])
def test_insert_delete_reinsert(oracle_mod, B, domain):
    """Copies go in over six batches, each holding a key at most once, so a key's copies lie in
    batch order along its list. A batch of deletes with repeated keys must then remove, for
    each key, its first copies in that order (the oracle's), whatever the schedule."""
    say("case: dup insert/delete/reinsert B=%d domain=%d" % (B, domain))
    t, o, rng = make_dup(oracle_mod, B, S.pool_slabs_bound(8 * domain), 900 + B)
    pool_keys = W.unique_keys(rng, domain)
    for r in range(6):
        keys = pool_keys[rng.below(domain, 10) < 7]
        vals = (rng.next(keys.size) >> np.uint64(32)).astype(np.uint32)
        st = t.insert(S.to_dev(keys), S.to_dev(vals))
        assert bool((st == 1).all())
        o.replace(keys, vals)
    assert_same_table(t, o)
    n = int(o.bucket_stats()[0].sum())
    # deletes with repeats: each removes the first remaining copy in list order
    dk = pool_keys[rng.below(n // 2, domain)]
    gs = t.delete(S.to_dev(dk)).cpu().numpy()
    os_ = o.delete(dk)
    assert per_key_sum(dk, gs) == per_key_sum(dk, os_)
    assert_same_table(t, o)
    # inserts fill the emptied slots first, then the tails
    rk = pool_keys[rng.below(n // 3, domain)]
    rv = (rng.next(rk.size) >> np.uint64(32)).astype(np.uint32)
    assert bool((t.insert(S.to_dev(rk), S.to_dev(rv)) == 1).all())
    o.replace(rk, rv)
    assert_same_table(t, o)
    # SEARCHALL: counts exact, values the same multiset per key
    q = pool_keys[: min(domain, 50000)]
    gc, goff, gv = t.search_all(S.to_dev(q))
    oc, ooff, ov = o.search_all(q)
    gc, goff, gv = gc.cpu().numpy(), goff.cpu().numpy(), S.to_host_u32(gv)
    assert (gc == oc).all() and (goff == ooff).all()
    for i in range(0, q.size, max(1, q.size // 2000)):
        a0, c0 = int(ooff[i]), int(oc[i])
        assert sorted(gv[a0:a0 + c0].tolist()) == sorted(ov[a0:a0 + c0].tolist())
    # SEARCH: found exact; the value is one of the key's values
    v, f = t.search(S.to_dev(q))
    ovv, of, _ = o.search(q)
    assert (f.cpu().numpy() == of).all()


@pytest.mark.parametrize("opw", [0, 8, 16, 64])
def test_list_order_across_batches(oracle_mod, opw):
    """Copies inserted one per batch sit in batch order: SEARCH returns the first batch's value
    and SEARCHALL the values in batch order; DELETE removes the first copy. Run at the default
    chunk width and at each other one (SEARCHALL and DELETEALL have a kernel per width)."""
    say("case: dup list order across batches, %d ops per wavefront" % opw)
    t, o, rng = make_dup(oracle_mod, 97, S.pool_slabs_bound(60000), 950)
    t.set_launch(0, opw)
    keys = W.unique_keys(rng, 15000)
    for r in range(4):
        v = (W.value_of(keys) + np.uint32(r)).astype(np.uint32)
        assert bool((t.insert(S.to_dev(keys), S.to_dev(v)) == 1).all())
        o.replace(keys, v)
    assert_same_table(t, o)
    gv, gf = t.search(S.to_dev(keys))
    ov, of, _ = o.search(keys)
    assert (gf.cpu().numpy() == 1).all() and (S.to_host_u32(gv) == ov).all()
    gc, goff, gvals = t.search_all(S.to_dev(keys))
    oc, ooff, ovals = o.search_all(keys)
    assert (gc.cpu().numpy() == 4).all() and (S.to_host_u32(gvals) == ovals).all()
    # delete twice each key: the first two batches' copies go
    dk = np.concatenate([keys, keys])
    assert bool((t.delete(S.to_dev(dk)) == 1).all())
    o.delete(dk)
    assert_same_table(t, o)
    gc, goff, gvals = t.search_all(S.to_dev(keys))
    oc, ooff, ovals = o.search_all(keys)
    assert (gc.cpu().numpy() == 2).all() and (S.to_host_u32(gvals) == ovals).all()
    # DELETEALL: the rest
    c = t.delete_all(S.to_dev(keys)).cpu().numpy()
    oc2 = o.delete_all(keys)
    assert (c == 2).all() and (oc2 == 2).all()
    assert_same_table(t, o)
    v, f = t.search(S.to_dev(keys))
    assert not f.cpu().numpy().any()


@pytest.mark.parametrize("opw", [0, 64])
def test_search_all_output_ranges(oracle_mod, opw):
    """SEARCHALL into ranges the caller chose: query i writes its values in list order from
    offsets[i], never past offsets[i + 1] nor the output's capacity, and nothing else; the counts
    are the full counts whatever the room. Ranges here leave gaps, cut lists short, are empty,
    and run past the capacity at the end."""
    say("case: SEARCHALL into caller ranges, %d ops per wavefront" % opw)
    t, o, rng = make_dup(oracle_mod, 97, S.pool_slabs_bound(20000), 960)
    t.set_launch(0, opw)
    keys = W.unique_keys(rng, 3500)
    present, absent = keys[:3000], keys[3000:]
    for r in range(4):
        v = (W.value_of(present) + np.uint32(r)).astype(np.uint32)
        assert bool((t.insert(S.to_dev(present), S.to_dev(v)) == 1).all())
        o.replace(present, v)
    q = np.concatenate([present, absent])[rng.permutation(keys.size)]
    oc, ooff, ov = o.search_all(q)
    room = np.array([0, 1, 2, 3, 4, 6], np.int64)[rng.below(q.size, 6).astype(np.int64)]
    offsets = np.zeros(q.size, np.int64)
    offsets[1:] = np.cumsum(room[:-1])
    cap = int(room.sum()) - 37  # the last queries' ranges run past the output
    sentinel = np.uint32(0xDEADBEEF)
    out = S.to_dev(np.full(cap, sentinel, np.uint32))
    counts = torch.empty(q.size, dtype=torch.int32, device="cuda")
    S.sh_search_all(t.handle, S.to_dev(q), counts, torch.from_numpy(offsets).cuda(), out)
    assert (counts.cpu().numpy() == oc).all()
    want = np.full(cap, sentinel, np.uint32)
    for i in range(q.size):
        end = min(int(offsets[i + 1]) if i + 1 < q.size else cap, cap)
        k = max(0, min(int(oc[i]), end - int(offsets[i])))
        want[offsets[i]:offsets[i] + k] = ov[ooff[i]:ooff[i] + k]
    assert (S.to_host_u32(out) == want).all()


def test_duplicates_at_benchmark_size(oracle_mod):
    """The benchmark's duplicates workload at its own size, against the oracle: 2^20 keys, four
    copies each, one copy per insert batch of 2^20, into 217,316 buckets; SEARCH returns each
    key's first copy, SEARCHALL all four values in batch order (into ranges offset by 4, as the
    benchmark sizes them), DELETE takes the first copy and DELETEALL the other three, the table
    equal to the oracle's after each step. The default launch shapes, as the benchmark runs."""
    say("case: duplicates at the benchmark's size (2^20 keys x 4 copies, B=217316)")
    n, copies, B = 1 << 20, 4, 217316
    keys = W.distinct_keys(81, 0, n)
    rng = W.SplitMix64(83)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, S.pool_slabs_bound(copies * n), a, b, duplicates=True)
    o = oracle_mod.Oracle(B, M, a, b, duplicates=True)
    kd = S.to_dev(keys)
    for c in range(copies):
        v = (W.value_of(keys) + np.uint32(c)).astype(np.uint32)
        assert bool((t.insert(kd, S.to_dev(v)) == 1).all())
        o.replace(keys, v)
    assert_same_table(t, o)
    q = keys[W.SplitMix64(82).below(copies * n, n)]
    gv, gf = t.search(S.to_dev(q))
    assert bool((gf == 1).all()) and (S.to_host_u32(gv) == W.value_of(q)).all()
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    off = torch.arange(0, copies * n, copies, dtype=torch.int64, device="cuda")
    vals = torch.empty(copies * n, dtype=torch.int32, device="cuda")
    S.sh_search_all(t.handle, kd, cnt, off, vals)
    oc, ooff, ov = o.search_all(keys)
    assert (cnt.cpu().numpy() == copies).all() and (oc == copies).all()
    assert (S.to_host_u32(vals) == ov).all()
    want = (W.value_of(keys)[:, None] + np.arange(copies, dtype=np.uint32)).astype(np.uint32)
    assert (ov.reshape(n, copies) == want).all()  # batch order, pinned without the oracle
    assert bool((t.delete(kd) == 1).all())
    o.delete(keys)
    assert_same_table(t, o)
    c = t.delete_all(kd).cpu().numpy()
    assert (c == copies - 1).all() and (o.delete_all(keys) == copies - 1).all()
    assert_same_table(t, o)
    _, gf = t.search(kd)
    assert not gf.cpu().numpy().any()


def test_mixed_batch_with_duplicates(oracle_mod):
    """Inserts, deletes and searches on disjoint key roles in one concurrent batch. The storage
    is checked on the host (host_walk) after the base build and after the batch, before any
    bound, so a failure names the first invariant broken: a slab in two lists, a slab in a list
    but free, an allocated slab in no list, a free slab that is not empty, or allocator bits
    that differ from the lists' slabs."""
    say("case: dup mixed batch")
    a, b, base, bv, ops, k, v = dup_cases.mixed_batch(960)
    t = S.SlabHash(dup_cases.B, S.pool_slabs_bound(80000), a, b, duplicates=True)
    o = oracle_mod.Oracle(dup_cases.B, M, a, b, duplicates=True)
    assert bool((t.insert(S.to_dev(base), S.to_dev(bv)) == 1).all())
    o.replace(base, bv)
    _, _, slabs0 = HW.check_structure(t)
    _, _, o_slabs0 = o.bucket_stats()
    assert (slabs0 == o_slabs0).all(), "the base build linked a slab beyond its inserts"
    gv, gs = t.mixed(S.to_dev(ops), S.to_dev(k), S.to_dev(v))
    ov, ost = o.mixed(ops, k, v)
    h_live, h_tomb, h_slabs = HW.check_structure(t)
    assert (gs.cpu().numpy() == ost).all() and (S.to_host_u32(gv) == ov).all()
    st = assert_same_table(t, o, check_counts=False)
    _, _, _, counts, _ = t.dump()
    # the library's walk agrees with the host's reading of the storage
    assert (counts[:, 0] == h_live).all() and (counts[:, 1] == h_tomb).all()
    assert (counts[:, 2] == h_slabs).all()
    assert st["pool_allocated"] == int((h_slabs - 1).sum())
    live, tomb, _ = o.bucket_stats()
    assert (counts[:, 0] == live).all() and (counts[:, 1] == 0).all()
    # An insert that read its slab before a concurrent delete emptied a slot appends instead
    # of filling it (the insert linearises first). So a bucket's slab count lies between the
    # oracle's with every delete ahead of every insert (most holes refilled) and the oracle's
    # with every insert ahead of every delete (no hole refilled). The oracle's count in batch
    # order is no bound: test_dup_bounds.py shows buckets of these inputs where a schedule
    # that runs deletes first ends one slab below it.
    ins_m, del_m = ops == W.OP_INSERT, ops == W.OP_DELETE
    o_lo = oracle_mod.Oracle(dup_cases.B, M, o.a, o.b, duplicates=True)
    o_lo.replace(base, bv)
    o_lo.delete(k[del_m])
    o_lo.replace(k[ins_m], v[ins_m])
    o_hi = oracle_mod.Oracle(dup_cases.B, M, o.a, o.b, duplicates=True)
    o_hi.replace(base, bv)
    o_hi.replace(k[ins_m], v[ins_m])
    o_hi.delete(k[del_m])
    _, _, lo_slabs = o_lo.bucket_stats()
    _, _, hi_slabs = o_hi.bucket_stats()
    _, _, batch_slabs = o.bucket_stats()
    say("buckets below the batch-order count: %s; above it: %s" % (
        np.flatnonzero(counts[:, 2] < batch_slabs).tolist(),
        np.flatnonzero(counts[:, 2] > batch_slabs).tolist()))
    over = np.flatnonzero(counts[:, 2] > hi_slabs)
    assert over.size == 0, "bucket %d: %d slabs, inserts-first bound %d" % (
        int(over[0]), int(counts[over[0], 2]), int(hi_slabs[over[0]]))
    under = np.flatnonzero(counts[:, 2] < lo_slabs)
    assert under.size == 0, "bucket %d: %d slabs, deletes-first bound %d" % (
        int(under[0]), int(counts[under[0], 2]), int(lo_slabs[under[0]]))


def test_flush_drops_empty_slots(oracle_mod):
    say("case: dup flush")
    t, o, rng = make_dup(oracle_mod, 7, S.pool_slabs_bound(20000), 970)
    dom = W.unique_keys(rng, 800)
    for r in range(12):   # a key at most once per batch: its copies lie in batch order
        keys = dom[rng.below(800, 10) < 9]
        vals = (rng.next(keys.size) >> np.uint64(32)).astype(np.uint32)
        t.insert(S.to_dev(keys), S.to_dev(vals))
        o.replace(keys, vals)
    dk = dom[rng.below(6000, 800)]
    t.delete(S.to_dev(dk))
    o.delete(dk)
    t.flush()
    o.flush_all()
    assert_same_table(t, o)
    more = W.unique_keys(rng, 3000)
    mv = W.value_of(more)
    t.insert(S.to_dev(more), S.to_dev(mv))
    o.replace(more, mv)
    assert_same_table(t, o)


def test_unique_key_tables_delete_all_and_search_all(oracle_mod):
    say("case: delete_all / search_all with unique keys")
    rng = W.SplitMix64(980)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(61, S.pool_slabs_bound(40000), a, b)
    o = oracle_mod.Oracle(61, M, a, b)
    keys = W.unique_keys(rng, 20000)
    vals = W.value_of(keys)
    t.insert(S.to_dev(keys), S.to_dev(vals))
    o.replace(keys, vals)
    q = np.concatenate([keys[:5000], W.unique_keys(rng, 2000, exclude=keys)])
    gc, goff, gv = t.search_all(S.to_dev(q))
    oc, ooff, ov = o.search_all(q)
    assert (gc.cpu().numpy() == oc).all() and (S.to_host_u32(gv) == ov).all()
    dq = np.concatenate([keys[:3000], keys[:100]])          # repeats find nothing the 2nd time
    c = t.delete_all(S.to_dev(dq)).cpu().numpy()
    oc2 = o.delete_all(dq)
    assert per_key_sum(dq, c) == per_key_sum(dq, oc2)
    assert_same_table(t, o)


def test_duplicates_rejected_by_batched_and_served_forms():
    p = S.ShParams(64, 2048, 3, 5, S.SH_TABLE_DUPLICATES)
    assert S.sh_storage_bytes(p) > 0
    arr = (S.ShParams * 1)(p)
    assert S.lib().sh_multi_storage_bytes(1, arr) == 0
    t = S.SlabHash(64, 2048, 3, 5, duplicates=True)
    ops = torch.zeros(8, dtype=torch.uint8, device="cuda")
    keys = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(Exception):
        S.Server(t, ops, keys, keys)

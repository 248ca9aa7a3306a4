"""GPU parity of key-only tables (the paper's 32-bit entries: 62 keys per 256-byte slab) against
the oracle run with 62 elements per slab and each key as its own value: bulk build with
repeated keys, searches, deletes, the reserved keys, concurrent mixed batches, flush, the
multiset operations, and the benchmark's size."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import linearize as LZ
from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu
KM = 62
EMPTY, TOMB = 0xFFFFFFFF, 0xFFFFFFFE


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def make_ko(oracle_mod, B, pool, seed, duplicates=False):
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, pool, a, b, keys_only=True, duplicates=duplicates)
    o = oracle_mod.Oracle(B, KM, a, b, duplicates=duplicates)
    return t, o, rng


def no_tomb_key(k):
    return k[k != TOMB]


@pytest.mark.parametrize("B,n", [(1, 3000), (61, 40000), (4099, 300000)])
def test_build_search_delete(oracle_mod, B, n):
    say("case: key-only B=%d n=%d" % (B, n))
    t, o, rng = make_ko(oracle_mod, B, S.pool_slabs_bound(2 * n), 1100 + B)
    keys = no_tomb_key(W.unique_keys(rng, n))
    batch = np.concatenate([keys, keys[rng.below(n // 10, keys.size)]])   # some repeats
    batch = batch[rng.permutation(batch.size)]
    st = t.insert(S.to_dev(batch)).cpu().numpy()
    ost = o.replace(batch, batch)
    # one op per key reports "new", the repeats "already there"
    assert int((st == 1).sum()) == keys.size and int((st == 2).sum()) == batch.size - keys.size
    assert ((st == 1) | (st == 2)).all() and (ost == 1).sum() == keys.size
    assert_same_table(t, o)
    miss = no_tomb_key(W.unique_keys(rng, n // 2, exclude=keys))
    q = np.concatenate([keys[: n // 2], miss])
    v, f = t.search(S.to_dev(q))
    ov, of, _ = o.search(q)
    assert (f.cpu().numpy() == of).all() and (S.to_host_u32(v) == ov).all()
    dels = keys[rng.permutation(keys.size)[: keys.size // 3]]
    gs = t.delete(S.to_dev(dels)).cpu().numpy()
    assert (gs == o.delete(dels)).all()
    assert_same_table(t, o)
    v, f = t.search(S.to_dev(q))
    ov, of, _ = o.search(q)
    assert (f.cpu().numpy() == of).all() and (S.to_host_u32(v) == ov).all()


def test_reserved_keys(oracle_mod):
    say("case: key-only reserved keys")
    t, o, rng = make_ko(oracle_mod, 17, 2048, 1200)
    keys = no_tomb_key(W.unique_keys(rng, 500))
    batch = np.concatenate([keys, [TOMB, EMPTY]]).astype(np.uint32)
    st = t.insert(S.to_dev(batch)).cpu().numpy()
    assert (st[:-2] == 1).all() and (st[-2:] == 0).all()
    assert t.stats()["error_word"] & S.SH_ERR_RESERVED_KEY
    o.replace(keys, keys)
    assert_same_table(t, o)
    v, f = t.search(S.to_dev(np.array([TOMB, EMPTY], np.uint32)))
    assert not f.cpu().numpy().any()


def test_mixed_linearizable(oracle_mod):
    say("case: key-only mixed batches")
    t, o, rng = make_ko(oracle_mod, 997, S.pool_slabs_bound(200000), 1300)
    present = no_tomb_key(W.unique_keys(rng, 60000))
    t.insert(S.to_dev(present))
    o.replace(present, present)
    fresh = no_tomb_key(W.unique_keys(rng, 80000, exclude=present))
    absent = fresh[60000:]
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(1 << 15, (0.2, 0.2, 0.3, 0.3))
    for r in range(3):
        ops, k, _ = W.mixed_batch(rng, present, fresh[r * n_ins:(r + 1) * n_ins], absent,
                                  n_ins, n_del, n_hit, n_miss)
        pre_v, pre_f, _ = o.search(k)
        gv, gs = t.mixed(S.to_dev(ops), S.to_dev(k), None)
        ov, ost = o.mixed(ops, k, k)
        post_v, post_f, _ = o.search(k)
        LZ.check_single_mutation_batch(ops, k, S.to_host_u32(gv), gs.cpu().numpy(), pre_f,
                                       pre_v, post_f, post_v, ost)
        dels = k[ops == 2]
        present = np.concatenate([present[~np.isin(present, dels)], k[ops == 1]])
    assert_same_table(t, o)


def test_flush(oracle_mod):
    say("case: key-only flush")
    t, o, rng = make_ko(oracle_mod, 29, S.pool_slabs_bound(60000), 1400)
    keys = no_tomb_key(W.unique_keys(rng, 30000))
    t.insert(S.to_dev(keys))
    o.replace(keys, keys)
    dels = keys[rng.permutation(keys.size)[:18000]]
    t.delete(S.to_dev(dels))
    o.delete(dels)
    back = dels[:5000]
    t.insert(S.to_dev(back))
    o.replace(back, back)
    assert_same_table(t, o)
    t.flush(3, 11)
    o.flush(3, 11)
    assert_same_table(t, o)
    t.flush()
    o.flush_all()
    assert_same_table(t, o)
    more = no_tomb_key(W.unique_keys(rng, 20000, exclude=keys))
    t.insert(S.to_dev(more))
    o.replace(more, more)
    assert_same_table(t, o)


@pytest.mark.parametrize("opw", [0, 8, 16, 64])
def test_multiset_key_only(oracle_mod, opw):
    """Duplicates allowed on a key-only table: copies one per batch, deletes with repeats,
    SEARCHALL counts, DELETEALL, flush; at the default chunk width and each other one."""
    say("case: key-only with duplicates, %d ops per wavefront" % opw)
    t, o, rng = make_ko(oracle_mod, 53, S.pool_slabs_bound(100000), 1500, duplicates=True)
    t.set_launch(0, opw)
    dom = no_tomb_key(W.unique_keys(rng, 4000))
    for r in range(5):
        ks = dom[rng.below(dom.size, 10) < 8]
        assert bool((t.insert(S.to_dev(ks)) == 1).all())
        o.replace(ks, ks)
    assert_same_table(t, o)
    dk = dom[rng.below(6000, dom.size)]
    gs = t.delete(S.to_dev(dk)).cpu().numpy()
    os_ = o.delete(dk)
    assert int(gs.sum()) == int(os_.sum())
    assert_same_table(t, o)
    gc, goff, gv = t.search_all(S.to_dev(dom))
    oc, ooff, ov = o.search_all(dom)
    assert (gc.cpu().numpy() == oc).all() and (S.to_host_u32(gv) == ov).all()
    half = dom[: dom.size // 2]
    c = t.delete_all(S.to_dev(half)).cpu().numpy()
    assert (c == o.delete_all(half)).all()
    assert_same_table(t, o)
    t.flush()
    o.flush_all()
    assert_same_table(t, o)


def test_key_only_at_benchmark_size(oracle_mod):
    say("case: key-only 2^22")
    wl = W.bulk(seed=11, n=1 << 22, prime=S.SH_HASH_PRIME)
    keys = no_tomb_key(wl["keys"])
    rng = W.SplitMix64(1600)
    a, b = wl.hash_a, wl.hash_b
    B = 108658
    t = S.SlabHash(B, S.pool_slabs_bound(keys.size), a, b, keys_only=True)
    o = oracle_mod.Oracle(B, KM, a, b)
    assert bool((t.build(S.to_dev(keys)) == 1).all())
    o.replace(keys, keys)
    assert_same_table(t, o)
    q = np.concatenate([keys[rng.permutation(keys.size)[: 1 << 20]],
                        no_tomb_key(wl["q_miss"][: 1 << 20])])
    v, f = t.search(S.to_dev(q))
    ov, of, _ = o.search(q)
    assert (f.cpu().numpy() == of).all() and (S.to_host_u32(v) == ov).all()

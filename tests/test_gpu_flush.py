"""GPU parity of FLUSH ("Flush" subsection): after deletes and re-inserts have left deleted
spots and long lists, flushing a range of buckets (or all) must give the oracle's table after
its own flush of the same range (live set, per-bucket live / deleted / slab counts, pool use,
structure invariants), and the slabs it frees must serve later allocations as empty slabs."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_parity import M, assert_same_table, make, search_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def churn(t, o, rng, keys, del_frac, back_frac):
    """Insert keys, delete a fraction, re-insert part of the deleted ones (they go to the list
    tails: deleted spots are not reused), on both sides."""
    vals = W.value_of(keys)
    assert bool((t.insert(S.to_dev(keys), S.to_dev(vals)) == 1).all())
    o.replace(keys, vals)
    dels = keys[rng.permutation(keys.size)[: int(del_frac * keys.size)]]
    assert bool((t.delete(S.to_dev(dels)) == 1).all())
    o.delete(dels)
    back = dels[: int(back_frac * dels.size)]
    bv = (W.value_of(back) ^ np.uint32(0x5A5A5A5A)).astype(np.uint32)
    assert bool((t.insert(S.to_dev(back), S.to_dev(bv)) == 1).all())
    o.replace(back, bv)
    return dels


@pytest.mark.parametrize("B,n", [(1, 3000), (7, 20000), (61, 50000), (4099, 200000)])
def test_flush_all_after_churn(oracle_mod, B, n):
    say("case: flush all, B=%d n=%d" % (B, n))
    rng = W.SplitMix64(700 + B)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, n)
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(2 * n))
    dels = churn(t, o, rng, keys, 0.5, 0.3)
    before = assert_same_table(t, o)
    t.flush()
    o.flush_all()
    after = assert_same_table(t, o)
    assert after["tombstones"] == 0 and after["pool_allocated"] <= before["pool_allocated"]
    search_both(t, o, np.concatenate([keys, dels]))
    # the freed slabs come back through the allocator as empty slabs
    more = W.unique_keys(rng, n, exclude=keys)
    mv = W.value_of(more)
    assert bool((t.insert(S.to_dev(more), S.to_dev(mv)) == 1).all())
    o.replace(more, mv)
    assert_same_table(t, o)
    search_both(t, o, more)


def test_flush_ranges(oracle_mod):
    """Flushing one bucket, then a middle range, then the rest: buckets outside each range keep
    their deleted spots and slabs."""
    say("case: flush ranges")
    rng = W.SplitMix64(801)
    B = 97
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, 30000)
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(60000))
    churn(t, o, rng, keys, 0.6, 0.5)
    for first, count in [(5, 1), (20, 41), (0, 0), (0, 20), (61, 36), (96, 1)]:
        t.flush(first, count)
        o.flush(first, count)
        assert_same_table(t, o)


def test_flush_everything_deleted(oracle_mod):
    say("case: flush with every key deleted")
    rng = W.SplitMix64(802)
    B = 13
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    keys = W.unique_keys(rng, 9000)
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(9000))
    vals = W.value_of(keys)
    t.insert(S.to_dev(keys), S.to_dev(vals))
    o.replace(keys, vals)
    t.delete(S.to_dev(keys))
    o.delete(keys)
    t.flush()
    o.flush_all()
    st = assert_same_table(t, o)
    assert st["live"] == 0 and st["pool_allocated"] == 0 and st["slabs_total"] == B


def test_flush_noop_cases_and_arguments(oracle_mod):
    say("case: flush no-ops and argument errors")
    rng = W.SplitMix64(803)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t, o = make(oracle_mod, 31, a, b, 2048)
    t.flush()                      # empty table
    o.flush_all()
    assert_same_table(t, o)
    keys = W.unique_keys(rng, 500)
    vals = W.value_of(keys)
    t.insert(S.to_dev(keys), S.to_dev(vals))
    o.replace(keys, vals)
    t.flush()                      # nothing deleted: nothing changes
    o.flush_all()
    assert_same_table(t, o)
    for first, count in [(32, 0), (31, 1), (0, 32), (30, 2)]:
        with pytest.raises(S.SlabHashError):
            S.sh_flush(t.handle, first, count)
    S.sh_flush(t.handle, 31, 0)    # an empty range at the end is fine
    assert_same_table(t, o)


def test_flush_at_benchmark_size(oracle_mod):
    """2^22 keys at B = 217316, a quarter deleted and a tenth of those re-inserted."""
    say("case: flush at 2^22 keys")
    wl = W.bulk(seed=11, n=1 << 22, prime=S.SH_HASH_PRIME)
    rng = W.SplitMix64(804)
    t, o = make(oracle_mod, 217316, wl.hash_a, wl.hash_b, S.pool_slabs_bound(1 << 22))
    churn(t, o, rng, wl["keys"], 0.25, 0.1)
    t.flush()
    o.flush_all()
    assert_same_table(t, o)
    search_both(t, o, wl["q_hit"][:1 << 18])

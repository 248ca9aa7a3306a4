"""GPU checks of SlabAlloc on its own ("Dynamic memory allocation"): every request gets a distinct
slab of the pool until the pool is exhausted, the bitmaps count exactly the slabs handed out,
freed slabs are handed out again, and a table whose pool has been through allocation and
release still matches the oracle."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_parity import assert_same_table, make

pytestmark = pytest.mark.gpu
EMPTY = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def alloc(t, n):
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    S.sh_alloc_slabs(t.handle, n, out)
    return S.to_host_u32(out)


def test_alloc_free_realloc():
    say("case: alloc / free / realloc")
    t = S.SlabHash(1, 64 * 2048, 3, 5)
    a = alloc(t, 100003)
    assert (a < t.params.pool_slabs).all() and np.unique(a).size == a.size
    st = t.stats()
    assert st["pool_allocated"] == a.size and st["error_word"] == 0
    rng = W.SplitMix64(5)
    gone = a[rng.permutation(a.size)[:40000]]
    S.sh_free_slabs(t.handle, S.to_dev(gone))
    assert t.stats()["pool_allocated"] == a.size - gone.size
    b = alloc(t, 60000)
    held = np.setdiff1d(a, gone)
    assert (b < t.params.pool_slabs).all() and np.unique(b).size == b.size
    assert np.intersect1d(b, held).size == 0
    assert t.stats()["pool_allocated"] == held.size + b.size
    # entries outside the pool are skipped when freeing
    S.sh_free_slabs(t.handle, S.to_dev(np.array([EMPTY, t.params.pool_slabs], np.uint32)))
    assert t.stats()["pool_allocated"] == held.size + b.size


def test_alloc_exhaustion():
    say("case: alloc past the pool")
    t = S.SlabHash(1, 8 * 2048, 7, 11)
    a = alloc(t, 8 * 2048 + 777)
    ok = a != EMPTY
    assert int(ok.sum()) == 8 * 2048 and np.unique(a[ok]).size == 8 * 2048
    st = t.stats()
    assert st["pool_allocated"] == 8 * 2048 and (st["error_word"] & S.SH_ERR_POOL_EXHAUSTED)


def test_one_million_allocations():
    """The paper's allocator test: a million allocations, one per thread."""
    say("case: 2^20 allocations")
    n = 1 << 20
    t = S.SlabHash(1, n + 4 * 2048, 13, 17)
    a = alloc(t, n)
    assert (a != EMPTY).all() and np.unique(a).size == n
    assert t.stats()["pool_allocated"] == n
    S.sh_free_slabs(t.handle, S.to_dev(a))
    assert t.stats()["pool_allocated"] == 0


def test_table_after_alloc_and_release(oracle_mod):
    """Slabs taken and given back leave the pool fit for lists: a contended build afterwards
    matches the oracle."""
    say("case: table after alloc and release")
    rng = W.SplitMix64(6)
    a_, b_ = W.hash_params(rng, S.SH_HASH_PRIME)
    t, o = make(oracle_mod, 5, a_, b_, 4 * 2048)
    got = alloc(t, 7000)
    S.sh_free_slabs(t.handle, S.to_dev(got))
    keys = W.unique_keys(rng, 20000)
    vals = W.value_of(keys)
    assert bool((t.insert(S.to_dev(keys), S.to_dev(vals)) == 1).all())
    o.replace(keys, vals)
    assert_same_table(t, o)


def test_whole_pool_and_counters():
    """A pool exactly the size of the request count: the wavefronts' starting words partition
    it, every slab is handed out once, and the counters account for every allocation."""
    say("case: 2^18 allocations from a pool of 2^18")
    n = 1 << 18
    t = S.SlabHash(1, n, 19, 23)
    t.set_launch(0, 0, S.SH_LAUNCH_COUNTERS)
    a = alloc(t, n)
    assert (a != EMPTY).all() and np.unique(a).size == n
    st = t.stats()
    assert st["allocs"] == n and st["pool_allocated"] == n and st["error_word"] == 0
    # half of them back, in a scattered pattern; then the same number again: the wavefronts
    # now hunt through partly used words and blocks
    rng = W.SplitMix64(7)
    gone = a[rng.permutation(n)[: n // 2]]
    S.sh_free_slabs(t.handle, S.to_dev(gone))
    b = alloc(t, n // 2)
    assert (b != EMPTY).all() and np.unique(b).size == b.size
    assert np.intersect1d(b, np.setdiff1d(a, gone)).size == 0
    assert t.stats()["pool_allocated"] == n
    assert (alloc(t, 64) == EMPTY).all()


def test_free_mixed_patterns():
    """Frees in one call that mix runs of one bitmap word, scattered slabs and repeated entries:
    every named slab is free afterwards and no other."""
    say("case: free runs, scattered and repeated entries")
    t = S.SlabHash(1, 32 * 2048, 29, 31)
    a = alloc(t, 50000)
    assert (a != EMPTY).all() and np.unique(a).size == a.size
    rng = W.SplitMix64(8)
    runs = np.sort(a)[:5000]                     # whole words, in order
    rest = np.setdiff1d(a, runs)
    scattered = rest[rng.permutation(rest.size)[:7000]]
    gone = np.concatenate([runs, scattered])
    listed = np.concatenate([gone, gone[rng.permutation(gone.size)[:3000]]])  # some twice
    listed = listed[rng.permutation(listed.size)]
    listed[: 64 * 40] = np.sort(listed[: 64 * 40])  # the first wavefronts see sorted entries
    S.sh_free_slabs(t.handle, S.to_dev(listed.astype(np.uint32)))
    assert t.stats()["pool_allocated"] == a.size - gone.size
    # the freed slabs, and only those, come back
    b = alloc(t, t.params.pool_slabs - (a.size - gone.size))
    assert (b != EMPTY).all() and np.unique(b).size == b.size
    assert np.intersect1d(b, np.setdiff1d(a, gone)).size == 0
    assert np.intersect1d(b, gone).size == gone.size

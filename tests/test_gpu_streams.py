"""Plain calls on one table from two streams at once, which the C ABI allows: the two streams'
kernels run concurrently on the table. Their key sets are disjoint, so every per-op result is
exact however the kernels overlap, and the final table must equal the oracle's after both."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_parity import assert_same_table, make, search_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def test_two_streams_on_one_table(oracle_mod):
    """Stream A inserts 2^18 fresh keys (allocating slabs) and then searches them; stream B
    deletes half of the 2^18 keys already in the table and searches the other half. Both start
    together, after the build."""
    say("case: two streams on one table")
    rng = W.SplitMix64(1301)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n = 1 << 18
    keys = W.unique_keys(rng, 2 * n)
    k0, k1 = keys[:n], keys[n:]
    v0, v1 = W.value_of(k0), W.value_of(k1)
    t, o = make(oracle_mod, n // 20, a, b, S.pool_slabs_bound(2 * n))
    assert bool((t.build(S.to_dev(k0), S.to_dev(v0)) == 1).all())
    o.replace(k0, v0)
    half = n // 2
    dk, sk = k0[:half], k0[half:]
    d_k1, d_v1, d_dk, d_sk = S.to_dev(k1), S.to_dev(v1), S.to_dev(dk), S.to_dev(sk)
    st_a = torch.empty(n, dtype=torch.uint8, device="cuda")
    va = torch.empty(n, dtype=torch.int32, device="cuda")
    fa = torch.empty(n, dtype=torch.uint8, device="cuda")
    st_b = torch.empty(half, dtype=torch.uint8, device="cuda")
    vb = torch.empty(n - half, dtype=torch.int32, device="cuda")
    fb = torch.empty(n - half, dtype=torch.uint8, device="cuda")
    ready = torch.cuda.Event()
    ready.record()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    sa.wait_event(ready)
    sb.wait_event(ready)
    S.sh_insert(t.handle, d_k1, d_v1, st_a, sa)
    S.sh_delete(t.handle, d_dk, st_b, sb)
    S.sh_search(t.handle, d_k1, va, fa, sa)
    S.sh_search(t.handle, d_sk, vb, fb, sb)
    torch.cuda.synchronize()
    assert bool((st_a == 1).all()) and bool((st_b == 1).all())
    assert bool((fa == 1).all()) and (S.to_host_u32(va) == v1).all()
    assert bool((fb == 1).all()) and (S.to_host_u32(vb) == W.value_of(sk)).all()
    o.replace(k1, v1)
    o.delete(dk)
    st = assert_same_table(t, o)
    assert st["tombstones"] == half and st["error_word"] == 0
    search_both(t, o, keys)

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


def _updates(rng, n):
    """Inputs for a table of n built keys k0 (values v0): n fresh keys k1 (values v1), the first
    quarter of k0 to delete (dk), the second quarter to give new values (rk, rv), and the rest
    left alone (uk)."""
    keys = W.unique_keys(rng, 2 * n)
    k0, k1 = keys[:n], keys[n:]
    v0, v1 = W.value_of(k0), W.value_of(k1)
    q = n // 4
    dk, rk, uk = k0[:q], k0[q:2 * q], k0[2 * q:]
    rv = (v0[q:2 * q] ^ np.uint32(0x5A5A5A5A)).astype(np.uint32)
    return k0, v0, k1, v1, dk, rk, rv, uk


def test_search_on_another_stream_after_an_event_sees_the_updates(oracle_mod):
    """Stream A inserts, deletes and replaces; stream B waits for an event recorded after those
    calls and searches: every update is seen."""
    say("case: search on stream B after stream A's updates (event order)")
    rng = W.SplitMix64(1311)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n = 1 << 17
    k0, v0, k1, v1, dk, rk, rv, uk = _updates(rng, n)
    t, o = make(oracle_mod, n // 20, a, b, S.pool_slabs_bound(2 * n))
    assert bool((t.build(S.to_dev(k0), S.to_dev(v0)) == 1).all())
    # every device input exists (and stays referenced) before the streams start
    q = np.concatenate([k1, dk, rk, uk])
    d_k1, d_v1, d_dk, d_rk, d_rv, dq = (S.to_dev(x) for x in (k1, v1, dk, rk, rv, q))
    vo = torch.empty(q.size, dtype=torch.int32, device="cuda")
    fo = torch.empty(q.size, dtype=torch.uint8, device="cuda")
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ready = torch.cuda.Event()
    ready.record()
    sa.wait_event(ready)
    S.sh_insert(t.handle, d_k1, d_v1, None, sa)
    S.sh_delete(t.handle, d_dk, None, sa)
    S.sh_insert(t.handle, d_rk, d_rv, None, sa)
    done_a = torch.cuda.Event()
    done_a.record(sa)
    sb.wait_event(done_a)
    S.sh_search(t.handle, dq, vo, fo, sb)
    torch.cuda.synchronize()
    f, v = fo.cpu().numpy(), S.to_host_u32(vo)
    i1, i2, i3 = k1.size, k1.size + dk.size, k1.size + dk.size + rk.size
    assert f[:i1].all() and (v[:i1] == v1).all()
    assert not f[i1:i2].any()
    assert f[i2:i3].all() and (v[i2:i3] == rv).all()
    assert f[i3:].all() and (v[i3:] == v0[2 * (n // 4):]).all()
    o.replace(k0, v0)
    o.replace(k1, v1)
    o.delete(dk)
    o.replace(rk, rv)
    assert_same_table(t, o)


def test_search_concurrent_with_updates_of_the_same_keys(oracle_mod):
    """Stream B searches while stream A inserts, deletes and replaces the same keys: each search
    returns its key's state before or after the update that concerns it, never anything else;
    keys no update touches are exact; afterwards the table equals the oracle's."""
    say("case: searches concurrent with updates of the same keys")
    rng = W.SplitMix64(1321)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n = 1 << 18
    k0, v0, k1, v1, dk, rk, rv, uk = _updates(rng, n)
    t, o = make(oracle_mod, n // 20, a, b, S.pool_slabs_bound(2 * n))
    assert bool((t.build(S.to_dev(k0), S.to_dev(v0)) == 1).all())
    q = np.concatenate([k1, dk, rk, uk])
    dq = S.to_dev(q)
    d_k1, d_v1, d_dk, d_rk, d_rv = (S.to_dev(x) for x in (k1, v1, dk, rk, rv))
    vo = torch.empty(q.size, dtype=torch.int32, device="cuda")
    fo = torch.empty(q.size, dtype=torch.uint8, device="cuda")
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ready = torch.cuda.Event()
    ready.record()
    sa.wait_event(ready)
    sb.wait_event(ready)
    S.sh_insert(t.handle, d_k1, d_v1, None, sa)
    S.sh_search(t.handle, dq, vo, fo, sb)
    S.sh_delete(t.handle, d_dk, None, sa)
    S.sh_insert(t.handle, d_rk, d_rv, None, sa)
    torch.cuda.synchronize()
    f, v = fo.cpu().numpy(), S.to_host_u32(vo)
    i1, i2, i3 = k1.size, k1.size + dk.size, k1.size + dk.size + rk.size
    # fresh keys: absent, or present with their value
    assert ((f[:i1] == 0) | ((f[:i1] == 1) & (v[:i1] == v1))).all()
    # deleted keys: present with the old value, or absent
    q4 = n // 4
    assert ((f[i1:i2] == 0) | ((f[i1:i2] == 1) & (v[i1:i2] == v0[:q4]))).all()
    # replaced keys: present, with the old or the new value
    assert f[i2:i3].all() and ((v[i2:i3] == v0[q4:2 * q4]) | (v[i2:i3] == rv)).all()
    # untouched keys: exact
    assert f[i3:].all() and (v[i3:] == v0[2 * q4:]).all()
    o.replace(k0, v0)
    o.replace(k1, v1)
    o.delete(dk)
    o.replace(rk, rv)
    assert_same_table(t, o)

"""The benchmark's bucket-partitioned CPU run (CPU): ops routed to thread h(k) mod T, each thread
keeping its share in the original order, must give every per-op result and the final table of
the single-threaded oracle. Mixed batches here repeat keys many times, so a thread that
reordered a bucket's ops would change some result."""
import numpy as np
import pytest

import bench
from paper_1710_11246_amd import workload as W

PRIME = 4294967291


def run_sequential(oracle_mod, B, a, b, build, searches, batches):
    o = oracle_mod.Oracle(B, 31, a, b)
    st = o.replace(*build)
    s_out = [o.search(q)[:2] for q in searches]
    m_out = [o.mixed(*bt) for bt in batches]
    return st, s_out, m_out, o


def table_of(orcs):
    rows = [np.stack(o.dump(), axis=1) for o in orcs]
    t = np.concatenate(rows) if rows else np.empty((0, 3), np.uint32)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


@pytest.mark.parametrize("B,n,T", [(1, 500, 3), (97, 6000, 4), (211, 20000, 8), (1031, 20000, 16)])
def test_partitioned_equals_sequential(oracle_mod, B, n, T):
    rng = W.SplitMix64(900 + B)
    a, b = W.hash_params(rng, PRIME)
    keys = W.unique_keys(rng, 2 * n)
    kb, absent = keys[:n], keys[n:]
    build = (kb, W.value_of(kb))
    searches = [kb[::-1].copy(), absent]
    batches = []
    present = kb.copy()
    fresh = W.unique_keys(rng, 3 * (n // 10), exclude=keys)
    for i in range(3):
        # a Gamma1 batch of distinct keys
        L = max(8, n // 5)
        ni, nd, nh, nm = W.gamma_counts(L, (0.2, 0.2, 0.3, 0.3))
        ops, bk, bv = W.mixed_batch(rng, present, fresh[i * (n // 10):(i + 1) * (n // 10)][:ni],
                                    absent, ni, nd, nh, nm)
        batches.append((ops, bk, bv))
        present = np.concatenate([present[~np.isin(present, bk[ops == 2])], bk[ops == 1]])
    # a batch over a few keys, each repeated many times with every kind of op
    few = np.concatenate([kb[:8], absent[:8]])
    m = 4000
    r = rng.next(3 * m)
    pick = (r[:m] % np.uint64(few.size)).astype(np.int64)
    ops = (r[m:2 * m] % np.uint64(3)).astype(np.uint8)
    bk = few[pick]
    bv = (r[2 * m:] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    batches.append((ops, bk, bv))

    st0, s0, m0, o0 = run_sequential(oracle_mod, B, a, b, build, searches, batches)
    st1, s1, m1, orcs = bench.oracle_partitioned(B, a, b, build, searches, batches, T)
    assert (st0 == st1).all()
    for (v0, f0), (v1, f1) in zip(s0, s1):
        assert (f0 == f1).all()
        assert (v0[f0 == 1] == v1[f1 == 1]).all()
    for (v0, q0), (v1, q1) in zip(m0, m1):
        assert (q0 == q1).all()
        assert (v0 == v1).all()
    assert all(o.error == 0 for o in orcs)
    assert np.array_equal(table_of([o0]), table_of(orcs))


def test_host_threads_bounded():
    assert 1 <= bench.host_threads() <= 16
    assert bench.host_threads(cap=1) == 1
    info = bench.host_info()
    assert info["nproc"] >= info["usable_cpus"] >= 1


def test_repeat_for_bounds():
    calls = []
    runs, dt = bench.repeat_for(lambda: calls.append(1), min_s=0.0, max_runs=5)
    assert runs == 1 and len(calls) == 1          # one run always happens
    calls.clear()
    runs, dt = bench.repeat_for(lambda: calls.append(1), min_s=3600.0, max_runs=7)
    assert runs == 7 and len(calls) == 7 and dt < 3600.0   # the cap ends a long sample

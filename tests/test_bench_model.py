"""The benchmark's algorithmic-byte model against the oracle (CPU): the slabs a search reads come
from the built table's bucket loads, so the model must count exactly the slabs the oracle's
own searches visit, for hits (slot p of a list sits in slab p // 31) and for misses (the whole
list of the query's bucket)."""
import numpy as np
import pytest

import bench
from paper_1710_11246_amd import workload as W

PRIME = 4294967291


@pytest.mark.parametrize("B,n", [(1, 100), (13, 2000), (97, 5000), (4099, 60000)])
def test_chain_visits_match_oracle_search_visits(oracle_mod, B, n):
    rng = W.SplitMix64(600 + B)
    a, b = W.hash_params(rng, PRIME)
    keys = W.unique_keys(rng, n)
    o = oracle_mod.Oracle(B, 31, a, b)
    o.replace(keys, W.value_of(keys))
    # a freshly built table (as the benchmark measures it): hits read slabs up to their own
    live, tomb, slabs = o.bucket_stats()
    assert not tomb.any()
    _, f, s = o.search(keys)
    assert f.all()
    assert bench.chain_visits(live) == int(s.sum())
    # misses, absent keys and (after deletes) deleted ones, read their bucket's whole list
    gone = keys[::5]
    o.delete(gone)
    _, _, slabs = o.bucket_stats()
    miss = np.concatenate([W.unique_keys(rng, n, exclude=keys), gone])
    _, f2, s2 = o.search(miss)
    assert not f2.any()
    assert int(s2.sum()) == int(slabs[o.bucket_of(miss)].sum())


def test_chain_visits_closed_form():
    # one bucket of 0..100 keys: slot p sits in slab p // 31 + 1 (1-based)
    for c in range(0, 101):
        want = sum(p // 31 + 1 for p in range(c))
        assert bench.chain_visits(np.array([c])) == want


def test_op_bytes_model():
    """Bytes per op of the roofline model: an insert reads its whole list (v_miss slabs) and
    writes the 64-byte sector of its swapped slot; a delete reads to its key (v_hit) and writes
    a sector; searches read their v slabs; a mixed batch adds its per-op inputs and outputs."""
    vh, vm = 1.25, 2.5
    assert bench.op_bytes("search_hit", 1, vh, vm) == 9 + 256 * vh
    assert bench.op_bytes("search_miss", 1, vh, vm) == 9 + 256 * vm
    assert bench.op_bytes("insert", 1, vh, vm) == 8 + 64 + 1 + 256 * vm
    assert bench.op_bytes("insert", 10, vh, vm, new_slabs=3) == 10 * (73 + 256 * vm) + 24
    assert bench.op_bytes("delete", 1, vh, vm) == 4 + 64 + 1 + 256 * vh
    mix = bench.op_bytes("mixed", 10, vh, vm, mix=(2, 3, 4, 1))
    assert mix == 10 * 14 + 256 * (3 * vm + 7 * vh) + 64 * 5 + 16 / 31
    # the benchmark's build at 60% utilisation: 2^22 inserts
    b = bench.op_bytes("insert", 1 << 22, 1.0006, 1.0052, new_slabs=20000)
    assert abs(b / (1 << 22) - (73 + 256 * 1.0052)) < 0.05

"""CPU: the slab-count bounds of a concurrent duplicates-mode batch ("Supported Operations":
INSERT with duplicates; "Deletion": with duplicates a deleted element leaves an empty slot that
a later insert may fill).

Every op of one batch is concurrent with every other, so any order of the batch is a legal
linearisation. With disjoint key roles (inserted keys are never deleted, deleted keys have one
copy) every order gives the same statuses, but not the same slab count: an insert fills a hole
only if the delete that made it came first. The count therefore lies between the count with
every delete first and the count with every insert first. The count in batch order is no bound:
for the inputs of the GPU test, some buckets end one slab lower when their deletes run first.
"""
import itertools

import numpy as np
import pytest

import dup_cases
import oracle
from paper_1710_11246_amd import workload as W

M = 31


def _base(a, b, base, bv, B=dup_cases.B, m=M):
    o = oracle.Oracle(B, m, a, b, duplicates=True)
    o.replace(base, bv)
    return o


@pytest.fixture(scope="module")
def case():
    a, b, base, bv, ops, k, v = dup_cases.mixed_batch(960)
    ob = _base(a, b, base, bv)
    _, st_batch = ob.mixed(ops, k, v)
    ins_m, del_m = ops == W.OP_INSERT, ops == W.OP_DELETE
    olo = _base(a, b, base, bv)
    olo.delete(k[del_m])
    olo.replace(k[ins_m], v[ins_m])
    ohi = _base(a, b, base, bv)
    ohi.replace(k[ins_m], v[ins_m])
    ohi.delete(k[del_m])
    return dict(a=a, b=b, base=base, bv=bv, ops=ops, k=k, v=v, st=st_batch,
                bkt=ob.bucket_of(k), batch=ob.bucket_stats()[2], lo=olo.bucket_stats()[2],
                hi=ohi.bucket_stats()[2], live=ob.bucket_stats()[0])


def test_batch_order_lies_between_the_bounds(case):
    assert (case["lo"] <= case["batch"]).all() and (case["batch"] <= case["hi"]).all()


def test_deletes_first_schedule_ends_below_batch_order(case):
    """The buckets where a legal schedule ends below the batch-order count: four of them go from
    4 slabs in batch order to 3 when the bucket's deletes run first; two from 5 to 4."""
    below = np.flatnonzero(case["batch"] > case["lo"])
    pairs = sorted((int(case["batch"][x]), int(case["lo"][x])) for x in below)
    assert pairs.count((4, 3)) >= 1, pairs
    ops, k, v, bkt = case["ops"], case["k"], case["v"], case["bkt"]
    for x in below:
        # the batch, with this bucket's deletes moved ahead of its first insert
        mine = np.flatnonzero((bkt == x) & (ops != W.OP_SEARCH))
        dels = [j for j in mine if ops[j] == W.OP_DELETE]
        first = next(j for j in mine if ops[j] == W.OP_INSERT)
        rest = [j for j in range(ops.size) if not (bkt[j] == x and ops[j] == W.OP_DELETE)]
        at = rest.index(first)
        order = np.array(rest[:at] + dels + rest[at:], dtype=np.int64)
        assert order.size == ops.size and np.unique(order).size == ops.size
        o = _base(case["a"], case["b"], case["base"], case["bv"])
        _, st = o.mixed(ops[order], k[order], v[order])
        assert (st == case["st"][order]).all()      # the same statuses: a legal linearisation
        slabs = o.bucket_stats()[2]
        assert slabs[x] == case["lo"][x] < case["batch"][x]


def test_inserts_first_bound_from_counting(case):
    """An insert links a slab only after reading every slot of the list occupied; each occupied
    slot it read holds a distinct element written by the build or an insert, so a list never
    exceeds ceil((built + inserted) / M) slabs, the inserts-first count."""
    ins_per_bucket = np.bincount(case["bkt"][case["ops"] == W.OP_INSERT], minlength=dup_cases.B)
    o0 = _base(case["a"], case["b"], case["base"], case["bv"])
    built = o0.bucket_stats()[0]
    n = built + ins_per_bucket
    assert (case["hi"] == np.maximum(1, -(-n // M))).all()


@pytest.mark.parametrize("seed", range(6))
def test_every_order_within_the_bounds_brute_force(seed):
    """Every order of a small batch (one bucket, two-slot slabs) ends within
    [deletes-first, inserts-first], and both ends are reached."""
    rng = W.SplitMix64(7000 + seed)
    a, b = W.hash_params(rng, dup_cases.PRIME)
    keys = W.unique_keys(rng, 9)
    base, bv = keys[:5], W.value_of(keys[:5])
    ins = np.concatenate([keys[5:8], keys[:1]])  # new keys and a further copy of a built one
    dels = keys[1:4]
    ops = np.array([W.OP_INSERT] * ins.size + [W.OP_DELETE] * dels.size, dtype=np.uint8)
    k = np.concatenate([ins, dels]).astype(np.uint32)
    v = (rng.next(k.size) >> np.uint64(32)).astype(np.uint32)
    counts = set()
    for perm in itertools.permutations(range(k.size)):
        p = np.array(perm)
        o = _base(a, b, base, bv, B=1, m=2)
        o.mixed(ops[p], k[p], v[p])
        counts.add(int(o.bucket_stats()[2].sum()))
    lo = _base(a, b, base, bv, B=1, m=2)
    lo.delete(dels)
    lo.replace(ins, v[:ins.size])
    hi = _base(a, b, base, bv, B=1, m=2)
    hi.replace(ins, v[:ins.size])
    hi.delete(dels)
    assert min(counts) == int(lo.bucket_stats()[2].sum()) and max(counts) == int(hi.bucket_stats()[2].sum())
    assert int(hi.bucket_stats()[2].sum()) == -(-(base.size + ins.size) // 2)

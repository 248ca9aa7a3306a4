"""Seeded inputs of the duplicates-mode mixed-batch case, shared by its GPU parity test and the
CPU test of its slab-count bounds. Generators only: no operation of the table is computed here."""
import numpy as np

from paper_1710_11246_amd import workload as W

PRIME = 4294967291
B = 211


def mixed_batch(seed: int = 960):
    """Base build of 20,000 unique keys, then one batch of inserts (6,000 further copies of keys
    0..4999), deletes (3,000 of keys 5000..9999, each once) and searches (8,000 of keys 10000..),
    shuffled. Returns hash_a, hash_b, base keys, base values, ops, keys, values."""
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, PRIME)
    base = W.unique_keys(rng, 20000)
    bv = W.value_of(base)
    ins = base[rng.below(6000, 5000)]
    dels = base[5000 + rng.permutation(5000)[:3000]]
    srch = base[10000:20000][rng.below(8000, 10000)]
    ops = np.concatenate([np.full(ins.size, W.OP_INSERT), np.full(dels.size, W.OP_DELETE),
                          np.full(srch.size, W.OP_SEARCH)]).astype(np.uint8)
    k = np.concatenate([ins, dels, srch]).astype(np.uint32)
    v = (rng.next(k.size) >> np.uint64(32)).astype(np.uint32)
    perm = rng.permutation(k.size)
    return a, b, base, bv, ops[perm], k[perm], v[perm]

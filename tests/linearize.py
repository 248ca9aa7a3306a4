"""Linearizability check of one concurrent mixed batch against the oracle (test infrastructure).

Every op touches one key, so the batch is linearizable iff, for each key separately, there is an
order of that key's mutations such that (Herlihy & Wing's locality of linearizability):
  - each mutation's status is what it returns when applied in that order from the key's state
    before the batch;
  - each search returns the key's state after some prefix of that order;
  - the key's state after the batch is the state at the end of that order.
Replace of k: status 1 if k absent (k becomes v), 2 if present (value becomes v).
Delete of k: status 1 if present (k becomes absent), 0 if absent.
"""
from __future__ import annotations

import itertools

import numpy as np

ABSENT = None


def _apply(state, op, val):
    """Returns (status, new_state); state is ABSENT or a value."""
    if op == 1:
        return (1 if state is ABSENT else 2), val
    if op == 2:
        return (0 if state is ABSENT else 1), ABSENT
    raise ValueError(op)


def check_batch(ops, keys, vals, got_vals, got_status, pre, post, max_mut=7):
    """ops/keys/vals: the batch; got_*: the GPU's per-op outputs; pre(key)/post(key) give the
    key's state (value or None) before and after the batch. Raises AssertionError on the first
    key with no valid order. Returns the number of keys checked."""
    ops = np.asarray(ops)
    keys = np.asarray(keys, dtype=np.uint32)
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    bounds = np.flatnonzero(np.diff(ks.astype(np.int64))) + 1
    groups = np.split(order, bounds)
    for g in groups:
        k = int(keys[g[0]])
        s0 = pre(k)
        s_end = post(k)
        muts = [int(i) for i in g if ops[i] in (1, 2)]
        srch = [int(i) for i in g if ops[i] == 0]
        if len(muts) > max_mut:
            raise ValueError("too many mutations of key %d for the brute-force check" % k)
        ok = False
        for perm in itertools.permutations(muts):
            state = s0
            states = [s0]
            good = True
            for i in perm:
                st, state = _apply(state, int(ops[i]), int(vals[i]))
                if st != int(got_status[i]):
                    good = False
                    break
                states.append(state)
            if not good or state != s_end:
                continue
            for i in srch:
                res = ABSENT if int(got_status[i]) == 0 else int(got_vals[i])
                if int(got_status[i]) == 0 and int(got_vals[i]) != 0xFFFFFFFF:
                    good = False
                    break
                if res not in states:
                    good = False
                    break
            if good:
                ok = True
                break
        assert ok, "key %d: no linearization (pre=%r post=%r ops=%s)" % (
            k, s0, s_end, [(int(ops[i]), int(vals[i]), int(got_status[i]), int(got_vals[i]))
                           for i in g])
    return len(groups)


def state_lookup(table_keys: np.ndarray, table_vals: np.ndarray):
    """Function key -> value or None over a (key, value) listing of live pairs."""
    d = dict(zip(table_keys.tolist(), table_vals.tolist()))
    return lambda k: d.get(k, ABSENT)


def check_single_mutation_batch(ops, keys, got_vals, got_status, pre_found, pre_vals,
                                post_found, post_vals, oracle_status):
    """Vectorised form of check_batch for batches where every key has at most one mutation
    (the benchmark batches): the linear order of a key's ops is then fixed up to where its
    searches fall, so mutation statuses must equal the sequential oracle's, and a search of a
    mutated key may see the state before or after the mutation; other searches are exact.
    pre_*/post_* are the oracle's search results for each op's key before/after the batch."""
    ops = np.asarray(ops)
    keys = np.asarray(keys, dtype=np.uint32)
    mut = ops != 0
    mk = np.unique(keys[mut])
    assert mk.size == int(mut.sum()), "a key has more than one mutation in this batch"
    assert (got_status[mut] == oracle_status[mut]).all(), "mutation status differs"
    s = ~mut
    touched = np.isin(keys, mk)
    gv, gs = got_vals[s], got_status[s]
    # reported miss must carry the empty value
    assert ((gs == 1) | (gv == 0xFFFFFFFF)).all()
    eq_pre = (gs == pre_found[s]) & ((gs == 0) | (gv == pre_vals[s]))
    eq_post = (gs == post_found[s]) & ((gs == 0) | (gv == post_vals[s]))
    t = touched[s]
    assert eq_pre[~t].all(), "search of an untouched key differs from the oracle"
    assert (eq_pre[t] | eq_post[t]).all(), "search of a mutated key is neither before nor after"
    return int(t.sum())

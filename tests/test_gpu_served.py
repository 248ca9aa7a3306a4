"""GPU tests of the served form (continuous batching): results alone vs in the mix, real-time
linearizability with shared hot keys, and admission by free slabs."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import autotune as A
from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu
M = S.SH_SLAB_PAIRS
EMPTY = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def table_for(n_init, n_final, a, b):
    B = A.buckets_for_utilisation(n_final, 0.6)
    return S.SlabHash(B, A.pool_slabs_for(n_final, B), a, b)


def states(sr, init_map):
    """Per op: (pre_found, pre_val, post_found, post_val) of its key around its key's single
    mutation (pre == post for keys no request mutates)."""
    n = sr.keys.size
    pre_f = np.zeros(n, np.uint8)
    pre_v = np.full(n, EMPTY, np.uint32)
    post_f = np.zeros(n, np.uint8)
    post_v = np.full(n, EMPTY, np.uint32)
    mut_idx = {}
    for j in np.flatnonzero(sr.ops != W.OP_SEARCH).tolist():
        mut_idx[int(sr.keys[j])] = j
    for j, k in enumerate(sr.keys.tolist()):
        if k in init_map:
            pre_f[j], pre_v[j] = 1, init_map[k]
        m = mut_idx.get(k)
        if m is None:
            post_f[j], post_v[j] = pre_f[j], pre_v[j]
        elif sr.ops[m] == W.OP_INSERT:
            post_f[j], post_v[j] = 1, sr.vals[m]
    return pre_f, pre_v, post_f, post_v


def req_of(sr):
    return np.searchsorted(sr.offsets, np.arange(sr.keys.size), side="right") - 1


def test_same_alone_and_in_the_mix(oracle_mod):
    """Requests on disjoint keys: each request's results issued alone (one sh_mixed per request,
    one after another) equal its results when served together with all the others."""
    say("case: served alone vs mix")
    rng = W.SplitMix64(101)
    init = W.unique_keys(rng, 1 << 16)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    sr = W.served_requests(102, init, 300, 1, 2000, zipf_s=None, disjoint=True,
                           absent_frac=0.2)
    n_final = init.size + int(sr.inserts.sum())
    ta, tb = table_for(init.size, n_final, a, b), table_for(init.size, n_final, a, b)
    vals0 = W.value_of(init)
    for t in (ta, tb):
        assert bool((t.build(S.to_dev(init), S.to_dev(vals0)) == 1).all())
    ops, keys, vals = S.to_dev(sr.ops), S.to_dev(sr.keys), S.to_dev(sr.vals)
    va = torch.empty(keys.numel(), dtype=torch.int32, device="cuda")
    sa = torch.empty(keys.numel(), dtype=torch.uint8, device="cuda")
    for i in range(300):
        o, n = int(sr.offsets[i]), int(sr.lengths[i])
        S.sh_mixed(ta.handle, ops[o:o + n], keys[o:o + n], vals[o:o + n], va[o:o + n],
                   sa[o:o + n])
    torch.cuda.synchronize()
    with S.Server(tb, ops, keys, vals, max_launches=4, max_batch_ops=4096) as srv:
        adm, done = srv.replay(sr.offsets, sr.lengths, sr.inserts,
                               np.zeros(300, np.uint64))
        srv.stop()
        vb, sb = S.to_host_u32(srv.vals_out), srv.status.cpu().numpy()
    assert (done != np.iinfo(np.uint64).max).all()
    va, sa = S.to_host_u32(va), sa.cpu().numpy()
    mut = sr.ops != W.OP_SEARCH
    assert (sa[mut] == sb[mut]).all() and (sa[mut] == 1).all()
    own = sr.mutator_of(sr.keys) == req_of(sr)
    same = ~mut & ~own   # searches of keys their own request does not mutate
    assert (sa[same] == sb[same]).all() and (va[same] == vb[same]).all()
    pre_f, pre_v, post_f, post_v = states(sr, dict(zip(init.tolist(), vals0.tolist())))
    either = ~mut & own
    for s_, v_ in ((sa, va), (sb, vb)):
        ok_pre = (s_ == pre_f) & ((s_ == 0) | (v_ == pre_v))
        ok_post = (s_ == post_f) & ((s_ == 0) | (v_ == post_v))
        assert (ok_pre | ok_post)[either].all()
    ba, ka, xa, ca, ya = ta.dump()
    bb, kb, xb, cb, yb = tb.dump()
    assert ya == yb == 0
    assert (ba == bb).all() and (ka == kb).all() and (xa == xb).all() and (ca == cb).all()
    o = oracle_mod.Oracle(tb.num_buckets, M, a, b)
    o.replace(init, vals0)
    o.mixed(sr.ops, sr.keys, sr.vals)
    assert_same_table(tb, o)


def test_zipf_requests_linearizable_in_real_time(oracle_mod):
    """Shared hot keys (Zipf searches), Poisson arrivals: a search must see its key's state
    before the mutating request if it finished before that request was admitted, after it if
    it was admitted after that request finished, and either state otherwise."""
    say("case: served zipf")
    rng = W.SplitMix64(201)
    init = W.unique_keys(rng, 1 << 17)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    sr = W.served_requests(202, init, 400, 1, 4096, zipf_s=1.1, absent_frac=0.05)
    n_final = init.size + int(sr.inserts.sum())
    t = table_for(init.size, n_final, a, b)
    vals0 = W.value_of(init)
    assert bool((t.build(S.to_dev(init), S.to_dev(vals0)) == 1).all())
    arrivals = W.poisson_arrivals(W.SplitMix64(203), 400, 2.0e4)
    ops, keys, vals = S.to_dev(sr.ops), S.to_dev(sr.keys), S.to_dev(sr.vals)
    with S.Server(t, ops, keys, vals, max_launches=4) as srv:
        adm, done = srv.replay(sr.offsets, sr.lengths, sr.inserts, arrivals)
        srv.stop()
        gv, gs = S.to_host_u32(srv.vals_out), srv.status.cpu().numpy()
    adm, done = adm.astype(np.int64), done.astype(np.int64)
    assert (done >= adm).all() and (adm >= arrivals.astype(np.int64)).all()
    mut = sr.ops != W.OP_SEARCH
    assert (gs[mut] == 1).all()
    pre_f, pre_v, post_f, post_v = states(sr, dict(zip(init.tolist(), vals0.tolist())))
    q = req_of(sr)
    r = sr.mutator_of(sr.keys)
    srch = ~mut
    ok_pre = (gs == pre_f) & ((gs == 0) | (gv == pre_v))
    ok_post = (gs == post_f) & ((gs == 0) | (gv == post_v))
    untouched = srch & (r < 0)
    assert ok_pre[untouched].all()
    m = srch & (r >= 0)
    before = m & (done[q] < adm[np.maximum(r, 0)])
    after = m & (adm[q] > done[np.maximum(r, 0)])
    assert ok_pre[before].all(), "saw a mutation from a request admitted after it finished"
    assert ok_post[after].all(), "missed a mutation of a request that finished before it"
    assert (ok_pre | ok_post)[m].all()
    say("  searches checked: %d before, %d after, %d overlapping" % (
        int(before.sum()), int(after.sum()), int((m & ~before & ~after).sum())))
    o = oracle_mod.Oracle(t.num_buckets, M, a, b)
    o.replace(init, vals0)
    o.mixed(sr.ops, sr.keys, sr.vals)
    assert_same_table(t, o)


def test_admission(oracle_mod):
    say("case: served admission")
    rng = W.SplitMix64(301)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(4, 2048, a, b)
    k = W.unique_keys(rng, 6000)
    ops = np.full(6000, W.OP_INSERT, np.uint8)
    dk, dv = S.to_dev(k), S.to_dev(W.value_of(k))
    with S.Server(t, S.to_dev(ops), dk, dv, max_requests=1) as srv:
        assert srv.submit(0, 2049, 2049)[0] == S.SH_ENOMEM    # more than the whole pool
        with pytest.raises(S.SlabHashError):
            srv.submit(5999, 2, 0)                              # outside the op arrays
        with pytest.raises(S.SlabHashError):
            srv.submit(0, 0, 0)                                 # empty
        code, t1 = srv.submit(0, 1000, 1000)
        assert code == S.SH_OK
        code2, t2 = srv.submit(1000, 1000, 1000)
        if code2 == S.SH_OK:
            assert srv.poll(t1)[0]                              # only once the first finished
        else:
            assert code2 == S.SH_EBUSY
        while not srv.poll(t1)[0]:
            pass
        if code2 != S.SH_OK:
            code2, t2 = srv.submit(1000, 1000, 1000)
            assert code2 == S.SH_OK
        while not srv.poll(t2)[0]:
            pass
        srv.stop()
        st = srv.status.cpu().numpy()[:2000]
    assert (st == 1).all()
    s = t.stats()
    assert s["live"] == 2000 and s["violations"] == 0 and s["error_word"] == 0


def test_tickets_expire_after_the_window(oracle_mod):
    """A server remembers the last 2^20 tickets: after 2^20 + 2^17 one-op requests, the first
    tickets (whose finish the load driver has read) have expired, the newest still answer, and
    every request's results are in place."""
    say("case: served ticket window")
    rng = W.SplitMix64(401)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(4099, 2048, a, b)
    keys = W.unique_keys(rng, 1 << 16)
    vals = W.value_of(keys)
    t.build(S.to_dev(keys), S.to_dev(vals))
    n = (1 << 20) + (1 << 17)
    q = keys[rng.below(n, keys.size)]
    ops = np.zeros(n, np.uint8)
    with S.Server(t, S.to_dev(ops), S.to_dev(q), S.to_dev(q)) as srv:
        adm, done = srv.replay(np.arange(n), np.ones(n, np.uint32), np.zeros(n, np.uint32),
                               np.zeros(n, np.uint64))
        with pytest.raises(S.SlabHashError):
            srv.poll(0)
        assert srv.poll(n - 1)[0]
        srv.stop()
        gv, gs = S.to_host_u32(srv.vals_out), srv.status.cpu().numpy()
    assert (done != np.iinfo(np.uint64).max).all() and (gs == 1).all()
    assert (gv == W.value_of(q)).all()

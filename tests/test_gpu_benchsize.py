"""GPU parity at the sizes the benchmark reports, in its launch configuration:
  - the batched form on the benchmark's own workload (256 tables with 2^10 .. 2^20 keys, one
    mixed batch of 2^6 .. 2^16 ops per table per round): its first round in one batched launch
    and its second through a captured graph, every op against its table's oracle, then every
    table's contents;
  - the served form on a resident 2^24-key table under Poisson arrivals with Zipf-shared keys:
    real-time linearizability of every search, and the final table equal to the oracle's;
  - the bulk build and both searches of 2^22 keys at every bucket count of the utilisation sweep;
  - the HBM-resident 2^26-key build and searches: every search result exact, and every bucket's
    live, deleted and slab counts equal to what the oracle's hash and the slab capacity give.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import autotune as A
from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_multi import build, check_round, make_tables
from test_gpu_parity import assert_same_table, make, search_both

pytestmark = pytest.mark.gpu
M = S.SH_SLAB_PAIRS
EMPTY = 0xFFFFFFFF
# largest bucket counts whose Binomial-model utilisation reaches 0.2 .. 0.8 for 2^22 keys
SWEEP_B = [654181, 436670, 327431, 261962, 217316, 176200, 55174]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


@pytest.mark.parametrize("B", SWEEP_B)
def test_bulk_2p22_every_sweep_point(oracle_mod, B):
    say("case: bulk n=2^22 B=%d" % B)
    wl = W.bulk(seed=11, n=1 << 22, prime=S.SH_HASH_PRIME)
    t, o = make(oracle_mod, B, wl.hash_a, wl.hash_b, S.pool_slabs_bound(1 << 22))
    st = t.build(S.to_dev(wl["keys"]), S.to_dev(wl["vals"]))
    assert (st.cpu().numpy() == o.replace(wl["keys"], wl["vals"])).all()
    search_both(t, o, wl["q_hit"])
    search_both(t, o, wl["q_miss"])
    assert_same_table(t, o)


def test_batched_benchmark_workload(oracle_mod):
    """The benchmark's batched workload (seed, table sizes, batch lengths and mix as it runs
    them): round 0 as one batched launch, round 1 as a graph replay, each op checked against
    its table's oracle, then all 256 tables' contents."""
    say("case: batched benchmark workload, 256 tables (generating inputs)")
    mr = W.multi_rounds(seed=31, T=256, n_lo=1 << 10, n_hi=1 << 20, len_lo=1 << 6,
                        len_hi=1 << 16, rounds=20, fractions=(0.3, 0.1, 0.3, 0.3),
                        prime=S.SH_HASH_PRIME)
    params = make_tables(mr)
    say("  building 256 tables, %d keys" % sum(k.size for k in mr.init_keys))
    m = S.MultiSlabHash(params)
    oracles = [oracle_mod.Oracle(p.num_buckets, M, p.hash_a, p.hash_b) for p in params]
    build(m, mr, oracles)
    T = len(params)
    desc0 = S.to_dev(S.pack_batch_descs(mr.offsets[0], mr.lengths[0], range(T)))
    gv, gs = m.mixed(desc0, T, S.to_dev(mr.ops[0]), S.to_dev(mr.keys[0]), S.to_dev(mr.vals[0]))
    say("  round 0: %d ops in one launch; checking" % mr.keys[0].size)
    check_round(mr, 0, oracles, S.to_host_u32(gv), gs.cpu().numpy())
    # round 1 through a captured graph, replayed on buffers holding the round's inputs
    n1 = mr.keys[1].size
    ops, keys, vals = S.to_dev(mr.ops[1]), S.to_dev(mr.keys[1]), S.to_dev(mr.vals[1])
    vout = torch.empty(n1, dtype=torch.int32, device="cuda")
    sout = torch.empty(n1, dtype=torch.uint8, device="cuda")
    desc = torch.empty_like(desc0)
    g = S.sh_multi_graph(m.handle, desc, T, ops, keys, vals, vout, sout)
    try:
        desc.copy_(S.to_dev(S.pack_batch_descs(mr.offsets[1], mr.lengths[1], range(T))))
        S.sh_graph_launch(g)
        torch.cuda.synchronize()
    finally:
        S.sh_graph_destroy(g)
    say("  round 1: %d ops as a graph replay; checking" % n1)
    check_round(mr, 1, oracles, S.to_host_u32(vout), sout.cpu().numpy())
    say("  comparing 256 tables")
    for t in range(T):
        assert_same_table(m.tables[t], oracles[t])


def served_states(sr, init_sorted):
    """Per op: its key's (found, value) before and after the key's one mutation (equal for keys
    no request mutates), for initial values value_of(key). Vectorised over all ops."""
    keys = sr.keys
    n = keys.size
    pos = np.minimum(np.searchsorted(init_sorted, keys), init_sorted.size - 1)
    pre_f = (init_sorted[pos] == keys).astype(np.uint8)
    pre_v = np.where(pre_f == 1, W.value_of(keys), np.uint32(EMPTY)).astype(np.uint32)
    post_f, post_v = pre_f.copy(), pre_v.copy()
    mi = np.flatnonzero(sr.ops != W.OP_SEARCH)
    order = np.argsort(keys[mi], kind="stable")
    mk = keys[mi][order]
    mop = mi[order]
    assert (np.diff(mk.astype(np.int64)) != 0).all(), "a key mutated twice"
    p = np.minimum(np.searchsorted(mk, keys), max(mk.size - 1, 0))
    has = mk[p] == keys
    m_op = mop[p]
    ins = has & (sr.ops[m_op] == W.OP_INSERT)
    dele = has & (sr.ops[m_op] == W.OP_DELETE)
    post_f[ins], post_v[ins] = 1, sr.vals[m_op[ins]]
    post_f[dele], post_v[dele] = 0, EMPTY
    return pre_f, pre_v, post_f, post_v


def test_served_2p24_real_time(oracle_mod):
    """A resident 2^24-key table served under Poisson arrivals: 10/5/85 insert/delete/search
    requests of log-uniform length in [1, 2^16], Zipf(1.1) searches over the initial keys."""
    say("case: served, 2^24-key table (generating inputs)")
    seed, n_keys, n_req = 43, 1 << 24, 1500
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    init = W.distinct_keys(seed, 0, n_keys)
    fresh = W.distinct_keys(seed, n_keys, n_keys // 4)
    sr = W.served_requests(seed + 1, init, n_req, 1, 1 << 16, fractions=(0.10, 0.05, 0.85),
                           zipf_s=1.1, shuffle_ranking=False, fresh_keys=fresh)
    n_final = n_keys + int(sr.inserts.sum())
    B = A.buckets_for_utilisation(n_final, 0.6)
    t = S.SlabHash(B, A.pool_slabs_for(n_final, B) + (1 << 18), a, b)
    vals0 = W.value_of(init)
    assert bool((t.build(S.to_dev(init), S.to_dev(vals0)) == 1).all())
    ops, keys, vals = S.to_dev(sr.ops), S.to_dev(sr.keys), S.to_dev(sr.vals)
    # arrivals at about the server's rate, so that requests overlap on the device
    arrivals = W.poisson_arrivals(W.SplitMix64(seed + 7), n_req, 4.0e5)
    say("  serving %d requests, %d ops" % (n_req, sr.keys.size))
    with S.Server(t, ops, keys, vals) as srv:
        adm, done = srv.replay(sr.offsets, sr.lengths, sr.inserts, arrivals)
        srv.stop()
        gv, gs = S.to_host_u32(srv.vals_out), srv.status.cpu().numpy()
    assert (done != np.iinfo(np.uint64).max).all()
    adm, done = adm.astype(np.int64), done.astype(np.int64)
    mut = sr.ops != W.OP_SEARCH
    assert (gs[mut] == 1).all()
    pre_f, pre_v, post_f, post_v = served_states(sr, np.sort(init))
    q = np.searchsorted(sr.offsets, np.arange(sr.keys.size), side="right") - 1
    r = sr.mutator_of(sr.keys)
    srch = ~mut
    ok_pre = (gs == pre_f) & ((gs == 0) | (gv == pre_v))
    ok_post = (gs == post_f) & ((gs == 0) | (gv == post_v))
    assert ok_pre[srch & (r < 0)].all()
    m = srch & (r >= 0)
    rr = np.maximum(r, 0)
    before = m & (done[q] < adm[rr])
    after = m & (adm[q] > done[rr])
    assert ok_pre[before].all(), "saw a mutation from a request admitted after it finished"
    assert ok_post[after].all(), "missed a mutation of a request that finished before it"
    assert (ok_pre | ok_post)[m].all()
    say("  searches of mutated keys: %d before, %d after, %d overlapping" % (
        int(before.sum()), int(after.sum()), int((m & ~before & ~after).sum())))
    o = oracle_mod.Oracle(B, M, a, b)
    o.replace(init, vals0)
    o.mixed(sr.ops, sr.keys, sr.vals)
    say("  comparing the final table")
    assert_same_table(t, o)


def test_hbm_resident_2p26(oracle_mod):
    """The benchmark's 2^26-key workload (bulk build at utilisation 0.6, then 2^26 all-hit and
    2^26 all-miss searches) in its launch configuration. Buckets are independent, so the whole
    table is pinned without a 2^26-entry oracle: each bucket's live count is the number of keys
    the oracle's hash sends there, its slab count max(1, ceil(live / 31)) (a build fills slabs in
    order), no deleted slots, the pool holding exactly the overflow slabs; every hit returns its
    key's value and every miss is absent."""
    say("case: HBM-resident build and searches, n=2^26")
    n, seed = 1 << 26, 61
    keys = W.distinct_keys(seed, 0, n)
    miss = W.distinct_keys(seed, n, n)
    perm = W.SplitMix64(seed + 1).permutation(n)
    a, b = W.hash_params(W.SplitMix64(seed + 2), S.SH_HASH_PRIME)
    B = A.buckets_for_utilisation(n, 0.6)
    t = S.SlabHash(B, A.pool_slabs_for(n, B), a, b)
    vals = W.value_of(keys)
    st = t.build(S.to_dev(keys), S.to_dev(vals))
    assert bool((st == 1).all())
    qh = keys[perm]
    v, f = t.search(S.to_dev(qh))
    assert bool((f == 1).all()) and (S.to_host_u32(v) == vals[perm]).all()
    del v, f
    v, f = t.search(S.to_dev(miss))
    assert not bool(f.any()) and bool((v == -1).all())
    del v, f
    counts = torch.empty(3 * B, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    viol = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.sh_dump(t.handle, None, None, None, counts, cnt, viol)
    c = S.to_host_u32(counts).reshape(-1, 3).astype(np.int64)
    assert int(viol.item()) == 0 and int(cnt.item()) == n
    live = np.bincount(oracle_mod.Oracle(B, M, a, b).bucket_of(keys).astype(np.int64),
                       minlength=B)
    assert (c[:, 0] == live).all() and not c[:, 1].any()
    assert (c[:, 2] == np.maximum(1, (live + M - 1) // M)).all()
    su = t.stats()
    assert su["pool_allocated"] == int((c[:, 2] - 1).sum()) and su["violations"] == 0
    assert su["live"] == n and su["error_word"] == 0


"""GPU parity of the batched form: many tables, one launch (and its graph replays), against one
oracle per table; and equality with the launch-per-table form."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import autotune as A
from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import linearize as LZ
from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu
M = S.SH_SLAB_PAIRS
GAMMA = (0.3, 0.1, 0.3, 0.3)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def make_tables(mr, target_u=0.6):
    T = len(mr.init_keys)
    params = []
    for t in range(T):
        occ = int(mr.final_occupancy[t])
        B = A.buckets_for_utilisation(occ, target_u)
        params.append(S.ShParams(B, A.pool_slabs_for(occ, B), int(mr.hash_a[t]),
                                 int(mr.hash_b[t])))
    return params


def build(m, mr, oracles=None):
    for t, tb in enumerate(m.tables):
        st = tb.build(S.to_dev(mr.init_keys[t]), S.to_dev(mr.init_vals[t]))
        assert bool((st == 1).all())
        if oracles is not None:
            oracles[t].replace(mr.init_keys[t], mr.init_vals[t])


def check_round(mr, r, oracles, gv, gs):
    for t, o in enumerate(oracles):
        a, n = int(mr.offsets[r][t]), int(mr.lengths[r][t])
        ops, k, v = mr.ops[r][a:a + n], mr.keys[r][a:a + n], mr.vals[r][a:a + n]
        pre_v, pre_f, _ = o.search(k)
        ov, ost = o.mixed(ops, k, v)
        post_v, post_f, _ = o.search(k)
        LZ.check_single_mutation_batch(ops, k, gv[a:a + n], gs[a:a + n], pre_f, pre_v, post_f,
                                       post_v, ost)


def test_one_launch_many_tables(oracle_mod):
    say("case: multi T=24 rounds=3")
    mr = W.multi_rounds(seed=21, T=24, n_lo=64, n_hi=1 << 14, len_lo=1, len_hi=1 << 12,
                        rounds=3, fractions=GAMMA, prime=S.SH_HASH_PRIME)
    params = make_tables(mr)
    m = S.MultiSlabHash(params)
    oracles = [oracle_mod.Oracle(p.num_buckets, M, p.hash_a, p.hash_b) for p in params]
    build(m, mr, oracles)
    for r in range(3):
        desc = S.to_dev(S.pack_batch_descs(mr.offsets[r], mr.lengths[r], range(24)))
        gv, gs = m.mixed(desc, 24, S.to_dev(mr.ops[r]), S.to_dev(mr.keys[r]),
                         S.to_dev(mr.vals[r]))
        check_round(mr, r, oracles, S.to_host_u32(gv), gs.cpu().numpy())
    for t in range(24):
        assert_same_table(m.tables[t], oracles[t])


def test_batched_equals_launch_per_table(oracle_mod):
    """The same rounds through one batched launch and through one sh_mixed launch per table give
    identical final tables and identical results for every op whose result is unique."""
    say("case: multi vs per-table")
    mr = W.multi_rounds(seed=22, T=16, n_lo=256, n_hi=1 << 13, len_lo=16, len_hi=1 << 11,
                        rounds=2, fractions=GAMMA, prime=S.SH_HASH_PRIME)
    params = make_tables(mr)
    m1, m2 = S.MultiSlabHash(params), S.MultiSlabHash(params)
    oracles = [oracle_mod.Oracle(p.num_buckets, M, p.hash_a, p.hash_b) for p in params]
    build(m1, mr, oracles)
    build(m2, mr)
    for r in range(2):
        ops, keys, vals = S.to_dev(mr.ops[r]), S.to_dev(mr.keys[r]), S.to_dev(mr.vals[r])
        desc = S.to_dev(S.pack_batch_descs(mr.offsets[r], mr.lengths[r], range(16)))
        gv1, gs1 = m1.mixed(desc, 16, ops, keys, vals)
        gv2 = torch.empty_like(gv1)
        gs2 = torch.empty_like(gs1)
        S.sh_multi_mixed_each(m2.handle, S.pack_batch_descs(mr.offsets[r], mr.lengths[r],
                                                            range(16)),
                              ops, keys, vals, gv2, gs2)
        g1v, g1s = S.to_host_u32(gv1), gs1.cpu().numpy()
        g2v, g2s = S.to_host_u32(gv2), gs2.cpu().numpy()
        check_round(mr, r, oracles, g1v, g1s)
        mut = mr.ops[r] != 0
        assert (g1s[mut] == g2s[mut]).all()
    for t in range(16):
        b1, k1, v1, c1, x1 = m1.tables[t].dump()
        b2, k2, v2, c2, x2 = m2.tables[t].dump()
        assert x1 == x2 == 0
        assert (b1 == b2).all() and (k1 == k2).all() and (v1 == v2).all() and (c1 == c2).all()


def test_graph_replays_with_new_inputs(oracle_mod):
    """Capture one batched launch, then replay it on fresh descriptors and ops copied into the
    same buffers, with eager work and synchronisations between replays; every replay is
    checked against the oracles."""
    say("case: graph replays")
    R = 4
    mr = W.multi_rounds(seed=23, T=20, n_lo=128, n_hi=1 << 13, len_lo=8, len_hi=1 << 11,
                        rounds=R, fractions=GAMMA, prime=S.SH_HASH_PRIME)
    params = make_tables(mr)
    m = S.MultiSlabHash(params)
    oracles = [oracle_mod.Oracle(p.num_buckets, M, p.hash_a, p.hash_b) for p in params]
    build(m, mr, oracles)
    cap = max(k.size for k in mr.keys)
    ops_b = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    keys_b = torch.zeros(cap, dtype=torch.int32, device="cuda")
    vals_b = torch.zeros(cap, dtype=torch.int32, device="cuda")
    vo = torch.empty(cap, dtype=torch.int32, device="cuda")
    so = torch.empty(cap, dtype=torch.uint8, device="cuda")
    desc_b = torch.zeros(2 * 20, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g = S.sh_multi_graph(m.handle, desc_b, 20, ops_b, keys_b, vals_b, vo, so)
    try:
        for r in range(R):
            n = mr.keys[r].size
            ops_b[:n].copy_(S.to_dev(mr.ops[r]))
            keys_b[:n].copy_(S.to_dev(mr.keys[r]))
            vals_b[:n].copy_(S.to_dev(mr.vals[r]))
            desc_b.copy_(S.to_dev(S.pack_batch_descs(mr.offsets[r], mr.lengths[r], range(20))))
            S.sh_graph_launch(g)
            torch.cuda.synchronize()
            check_round(mr, r, oracles, S.to_host_u32(vo)[:n], so.cpu().numpy()[:n])
            # eager work between replays: a search through the single-table call
            t0 = r % 20
            q = mr.init_keys[t0][:50]
            v, f = m.tables[t0].search(S.to_dev(q))
            ov, of, _ = oracles[t0].search(q)
            assert (f.cpu().numpy() == of).all() and (S.to_host_u32(v) == ov).all()
            torch.cuda.synchronize()
    finally:
        S.sh_graph_destroy(g)
    for t in range(20):
        assert_same_table(m.tables[t], oracles[t])


def test_descriptor_edge_cases(oracle_mod):
    """Empty descriptors, several descriptors on one table in one launch, a single descriptor,
    a descriptor naming a missing table and one reaching past the op arrays."""
    say("case: descriptor edges")
    rng = W.SplitMix64(77)
    params, oracles, keys0 = [], [], []
    for t in range(3):
        a, b = W.hash_params(rng, S.SH_HASH_PRIME)
        params.append(S.ShParams(37 + t, 3 * 2048, a, b))
        oracles.append(oracle_mod.Oracle(37 + t, M, a, b))
    m = S.MultiSlabHash(params)
    # table 1 gets two batches on disjoint fresh keys; tables 0 and 2 get empty descriptors too
    k1 = W.unique_keys(rng, 3000)
    ops = np.full(3000, W.OP_INSERT, np.uint8)
    vals = W.value_of(k1)
    descs = S.pack_batch_descs([0, 0, 1000, 3000, 1000], [0, 1000, 2000, 0, 0], [0, 1, 1, 2, 0])
    gv, gs = m.mixed(S.to_dev(descs), 5, S.to_dev(ops), S.to_dev(k1), S.to_dev(vals))
    assert bool((gs == 1).all())
    oracles[1].replace(k1, vals)
    for t in range(3):
        assert_same_table(m.tables[t], oracles[t])
    # one descriptor covering a search batch
    gv, gs = m.mixed(S.to_dev(S.pack_batch_descs([0], [3000], [1])), 1,
                     S.to_dev(np.zeros(3000, np.uint8)), S.to_dev(k1), S.to_dev(vals))
    assert bool((gs == 1).all()) and (S.to_host_u32(gv) == vals).all()
    # table 7 does not exist: skipped; a range past the arrays is clipped to them
    sent = 0xAB
    gv = torch.full((3000,), 5, dtype=torch.int32, device="cuda")
    gs = torch.full((3000,), sent, dtype=torch.uint8, device="cuda")
    S.sh_multi_mixed(m.handle, S.to_dev(S.pack_batch_descs([0, 2500], [100, 10 ** 6], [7, 1])), 2,
                     S.to_dev(np.zeros(3000, np.uint8)), S.to_dev(k1), S.to_dev(vals), gv, gs)
    gs = gs.cpu().numpy()
    assert (gs[:100] == sent).all() and (gs[100:2500] == sent).all()
    assert (gs[2500:] == 1).all() and (S.to_host_u32(gv)[2500:] == vals[2500:]).all()

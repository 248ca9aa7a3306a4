"""GPU parity at the benchmark's full sizes and launch configuration: 2^22-key bulk build and
all-hit / all-miss searches, and incremental growth to 2^24 keys with concurrent mixed batches
at checkpoints. Every output is compared with the oracle (the oracle handles these sizes in
seconds)."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import linearize as LZ
from test_gpu_parity import assert_same_table, make, search_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


@pytest.mark.parametrize("B", [217316, 55174])
def test_bulk_2p22(oracle_mod, B):
    say("case: bulk n=2^22 B=%d" % B)
    wl = W.bulk(seed=11, n=1 << 22, prime=S.SH_HASH_PRIME)
    t, o = make(oracle_mod, B, wl.hash_a, wl.hash_b, S.pool_slabs_bound(1 << 22))
    st = t.build(S.to_dev(wl["keys"]), S.to_dev(wl["vals"]))
    assert (st.cpu().numpy() == o.replace(wl["keys"], wl["vals"])).all()
    search_both(t, o, wl["q_hit"])
    search_both(t, o, wl["q_miss"])
    assert_same_table(t, o)


def test_growth_to_2p24_with_mixed_checkpoints(oracle_mod):
    say("case: growth to 2^24, B=793240, mixed batches at 2^20, 2^22, 2^24")
    B = 793240
    rng = W.SplitMix64(3)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    total = 1 << 24
    keys = W.unique_keys(rng, total)
    vals = W.value_of(keys)
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(1 << 16, (0.2, 0.2, 0.3, 0.3))
    per_cp = 2
    fresh = W.unique_keys(rng, 3 * per_cp * n_ins + n_miss, exclude=keys)
    absent = fresh[3 * per_cp * n_ins:]
    t, o = make(oracle_mod, B, a, b, S.pool_slabs_bound(total + 3 * per_cp * n_ins))
    g = 1 << 16
    grown = 0
    present = np.empty(0, np.uint32)
    fi = 0
    for cp in (1 << 20, 1 << 22, 1 << 24):
        kd, vd = S.to_dev(keys[grown:cp]), S.to_dev(vals[grown:cp])
        for s in range(0, cp - grown, g):
            st = t.insert(kd[s:s + g], vd[s:s + g])
            assert bool((st == 1).all())
        o.replace(keys[grown:cp], vals[grown:cp])
        present = np.concatenate([present, keys[grown:cp]])
        grown = cp
        say("  grown to %d" % cp)
        for _ in range(per_cp):
            ops, bk, bv = W.mixed_batch(rng, present, fresh[fi * n_ins:(fi + 1) * n_ins],
                                        absent, n_ins, n_del, n_hit, n_miss)
            fi += 1
            pre_v, pre_f, _ = o.search(bk)
            gv, gs = t.mixed(S.to_dev(ops), S.to_dev(bk), S.to_dev(bv))
            ov, ost = o.mixed(ops, bk, bv)
            post_v, post_f, _ = o.search(bk)
            LZ.check_single_mutation_batch(ops, bk, S.to_host_u32(gv), gs.cpu().numpy(),
                                           pre_f, pre_v, post_f, post_v, ost)
            dels = bk[ops == 2]
            present = np.concatenate([present[~np.isin(present, dels)], bk[ops == 1]])
    assert_same_table(t, o)


def test_growth_with_all_three_distributions(oracle_mod):
    """The concurrent benchmark's workload at reduced size: growth in insert batches, and at
    each checkpoint mixed batches of Gamma0, Gamma1 and Gamma2, every batch checked per key
    against the oracle and the final table compared in full."""
    say("case: growth to 2^19 with Gamma0/1/2 batches at 2^17 and 2^19")
    total, batch, B = 1 << 19, 1 << 14, 24787
    g = W.growth_checkpoints(61, total, batch, [1 << 17, 1 << 19], 2, 1 << 14,
                             S.SH_HASH_PRIME)
    t, o = make(oracle_mod, B, g.hash_a, g.hash_b,
                S.pool_slabs_bound(total + g.mixed_inserts))
    kd, vd = S.to_dev(g.keys), S.to_dev(g.vals)
    grown = 0
    for cp, per_cp in zip(g.checkpoints, g.mixed):
        for s0 in range(grown, cp, batch):
            st = t.insert(kd[s0:s0 + batch], vd[s0:s0 + batch])
            assert bool((st == 1).all())
        o.replace(g.keys[grown:cp], g.vals[grown:cp])
        grown = cp
        for name, batches in per_cp:
            say("  %d keys, %s" % (cp, name))
            for ops, bk, bv in batches:
                pre_v, pre_f, _ = o.search(bk)
                gv, gs = t.mixed(S.to_dev(ops), S.to_dev(bk), S.to_dev(bv))
                ov, ost = o.mixed(ops, bk, bv)
                post_v, post_f, _ = o.search(bk)
                LZ.check_single_mutation_batch(ops, bk, S.to_host_u32(gv), gs.cpu().numpy(),
                                               pre_f, pre_v, post_f, post_v, ost)
    assert_same_table(t, o)

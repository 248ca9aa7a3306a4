"""GPU parity for the benchmark's own step, with its inputs, table and default launch shapes:
reset, bulk build of 2^22 pairs into B = 217,316 buckets, 2^22 all-hit and 2^22 all-miss
searches, then 16 Gamma1 mixed batches of 2^16 ops on the same table. The step runs twice, the
second time after `sh_reset` of the table the first left behind, as the timed loop does. Builds
and searches are compared element by element with the oracle, each mixed batch is checked for
linearizability against the oracle's states before and after it, and the final table must
equal the oracle's."""
import sys

import numpy as np
import pytest
import torch

import bench
from paper_1710_11246_amd import slabhash as S

import linearize as LZ
from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def test_bench_step_twice(oracle_mod):
    say("case: benchmark step x2, n=2^22 B=%d, 16 mixed batches of 2^16" % bench.B_FOR_UTIL[0.6])
    wl, batches = bench.make_inputs(0.6)
    B = bench.B_FOR_UTIL[0.6]
    n_ins = int((batches[0][0] == 1).sum())
    pool = S.pool_slabs_bound(bench.N_KEYS + n_ins * bench.MIX_BATCHES)
    t = S.SlabHash(B, pool, wl.hash_a, wl.hash_b)
    keys, vals = S.to_dev(wl["keys"]), S.to_dev(wl["vals"])
    q_hit, q_miss = S.to_dev(wl["q_hit"]), S.to_dev(wl["q_miss"])
    mix_dev = [(S.to_dev(o), S.to_dev(k), S.to_dev(v)) for o, k, v in batches]
    for step in range(2):
        say("  step %d" % step)
        t.reset()
        o = oracle_mod.Oracle(B, S.SH_SLAB_PAIRS, wl.hash_a, wl.hash_b)
        st = t.build(keys, vals)
        assert (st.cpu().numpy() == o.replace(wl["keys"], wl["vals"])).all()
        for q_np, q_dev in ((wl["q_hit"], q_hit), (wl["q_miss"], q_miss)):
            v, f = t.search(q_dev)
            ov, of, _ = o.search(q_np)
            assert (f.cpu().numpy() == of).all()
            assert (S.to_host_u32(v) == ov).all()
        for bi, ((ops, bk, bv), (d_o, d_k, d_v)) in enumerate(zip(batches, mix_dev)):
            pre_v, pre_f, _ = o.search(bk)
            gv, gs = t.mixed(d_o, d_k, d_v)
            ost = o.mixed(ops, bk, bv)[1]
            post_v, post_f, _ = o.search(bk)
            LZ.check_single_mutation_batch(ops, bk, S.to_host_u32(gv), gs.cpu().numpy(),
                                           pre_f, pre_v, post_f, post_v, ost)
        st_tab = assert_same_table(t, o)
        assert st_tab["error_word"] == 0
        say("  step %d ok: %d live, %d tombstones, %d pool slabs" %
            (step, st_tab["live"], st_tab["tombstones"], st_tab["pool_allocated"]))

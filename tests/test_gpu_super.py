"""GPU parity of the super-block hierarchy ("Dynamic memory allocation"): tables whose own pool
(super block 0) is one block, with further super blocks registered, grow through them. Every
result and the final table match the oracle, whose pool is the super blocks' total; the host
reads every super block's slabs and bitmaps (host_walk) and checks the lists' addresses, the
allocator bits and the free slabs; the pool is exhausted only when every super block is full."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

import host_walk as HW
from test_gpu_multi import build, check_round, make_tables
from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu
M = S.SH_SLAB_PAIRS


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def super_use(t):
    """Set allocator bits per super block, read on the host."""
    _, pools, bms = HW.raw_parts(t, t.supers)
    return [int(np.unpackbits(bm.reshape(-1).view(np.uint8)).sum()) for bm in bms]


@pytest.mark.parametrize("mode", ["pairs", "duplicates", "keys_only"])
def test_growth_through_super_blocks(oracle_mod, mode):
    say("case: growth through super blocks, %s" % mode)
    dup, ko = mode == "duplicates", mode == "keys_only"
    rng = W.SplitMix64(1401)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    B = 61
    t = S.SlabHash(B, 2048, a, b, duplicates=dup, keys_only=ko)
    for slabs in (2048, 2048, 4096):
        t.add_super_block(slabs)
    cap = 2048 + 2048 + 2048 + 4096
    per = 62 if ko else M
    n = (B + 5000) * per                         # about 5000 pool slabs: three super blocks
    keys = W.unique_keys(rng, n)
    keys = keys[keys != np.uint32(0xFFFFFFFE)]
    vals = keys if ko else W.value_of(keys)
    o = oracle_mod.Oracle(B, per, a, b, duplicates=dup, pool_slabs=cap)
    st = t.insert(S.to_dev(keys), None if ko else S.to_dev(vals))
    assert (st.cpu().numpy() == o.replace(keys, vals)).all()
    s = t.stats()
    assert s["pool_capacity"] == cap and s["error_word"] == 0
    use = super_use(t)
    say("  slabs in use per super block: %s" % use)
    assert use[0] >= 2048 - 64 and use[1] > 0 and use[2] > 0 and use[3] == 0
    assert_same_table(t, o)
    # searches, deletes and a mixed batch over lists that cross super blocks
    v, f = t.search(S.to_dev(keys))
    ov, of, _ = o.search(keys)
    assert (f.cpu().numpy() == of).all() and (S.to_host_u32(v) == ov).all()
    gone = keys[::3]
    assert (t.delete(S.to_dev(gone)).cpu().numpy() == o.delete(gone)).all()
    more = W.unique_keys(rng, 40 * per, exclude=keys)
    more = more[more != np.uint32(0xFFFFFFFE)]
    ops = np.concatenate([np.full(more.size, W.OP_INSERT), np.full(keys.size // 3, W.OP_SEARCH)])
    kk = np.concatenate([more, keys[1::3][: keys.size // 3]]).astype(np.uint32)
    vv = kk if ko else W.value_of(kk)
    perm = rng.permutation(kk.size)
    ops, kk, vv = ops[perm].astype(np.uint8), kk[perm], vv[perm]
    gv, gs = t.mixed(S.to_dev(ops), S.to_dev(kk), S.to_dev(vv))
    ovv, ost = o.mixed(ops, kk, vv)
    assert (gs.cpu().numpy() == ost).all() and (S.to_host_u32(gv) == ovv).all()
    assert_same_table(t, o)
    # FLUSH frees slabs in every super block; a reset empties them all and keeps them registered
    t.flush()
    o.flush_all()
    assert_same_table(t, o)
    t.reset()
    torch.cuda.synchronize()
    assert all(u == 0 for u in super_use(t))
    for mem in t.supers:
        r = mem.cpu().numpy()
        nsl = HW.super_slabs(r.size)
        assert (r[:nsl * 256] == 0xFF).all() and (r[nsl * 256:nsl * 256 + nsl // 8] == 0).all()
    o2 = oracle_mod.Oracle(B, per, a, b, duplicates=dup, pool_slabs=cap)
    assert (t.insert(S.to_dev(keys), None if ko else S.to_dev(vals)).cpu().numpy() ==
            o2.replace(keys, vals)).all()
    assert_same_table(t, o2)


def test_exhaustion_only_when_every_super_block_is_full(oracle_mod):
    say("case: exhaustion across super blocks")
    rng = W.SplitMix64(1402)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    B = 8
    t = S.SlabHash(B, 2048, a, b)
    t.add_super_block(2048)
    cap = 4096
    n = (B + cap) * M + 5000
    keys = W.unique_keys(rng, n)
    vals = W.value_of(keys)
    st = t.insert(S.to_dev(keys), S.to_dev(vals)).cpu().numpy()
    s = t.stats()
    assert s["error_word"] & S.SH_ERR_POOL_EXHAUSTED
    assert s["pool_allocated"] == cap and super_use(t) == [2048, 2048]
    assert set(np.unique(st).tolist()) <= {0, 1} and (st == 0).sum() >= 5000
    v, f = t.search(S.to_dev(keys))
    assert (f.cpu().numpy() == (st == 1)).all()
    assert (S.to_host_u32(v)[st == 1] == vals[st == 1]).all()
    HW.check_structure(t)


def test_batched_tables_grow_through_super_blocks(oracle_mod):
    """A table of the batched form with no pool of its own and a registered super block: its
    build and one batched launch over every table take all their slabs from the super block."""
    say("case: batched tables with super blocks")
    GAMMA = (0.6, 0.0, 0.2, 0.2)
    mr = W.multi_rounds(seed=1403, T=6, n_lo=1 << 12, n_hi=1 << 14, len_lo=1 << 14,
                        len_hi=1 << 15, rounds=1, fractions=GAMMA, prime=S.SH_HASH_PRIME)
    params = make_tables(mr)
    params[0] = S.ShParams(7, 0, params[0].hash_a, params[0].hash_b)
    m = S.MultiSlabHash(params)
    mem = torch.empty(S.sh_super_block_bytes(8192), dtype=torch.uint8, device="cuda")
    S.sh_add_super_block(m.tables[0].handle, mem)
    oracles = [oracle_mod.Oracle(p.num_buckets, M, p.hash_a, p.hash_b) for p in params]
    build(m, mr, oracles)
    desc = S.to_dev(S.pack_batch_descs(mr.offsets[0], mr.lengths[0], range(6)))
    gv, gs = m.mixed(desc, 6, S.to_dev(mr.ops[0]), S.to_dev(mr.keys[0]), S.to_dev(mr.vals[0]))
    check_round(mr, 0, oracles, S.to_host_u32(gv), gs.cpu().numpy())
    s = m.tables[0].stats()
    assert s["pool_capacity"] == 8192 and s["pool_allocated"] > 0 and s["error_word"] == 0
    for t in range(6):
        assert_same_table(m.tables[t], oracles[t])


def test_super_block_arguments():
    t = S.SlabHash(4, 2048, 3, 5)
    small = torch.empty(S.sh_super_block_bytes(2048) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SlabHashError):
        S.sh_add_super_block(t.handle, small)        # less than one block
    mem = torch.empty(S.sh_super_block_bytes(2048) + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SlabHashError):
        S.sh_add_super_block(t.handle, mem[1:])       # not 256-byte aligned
    for _ in range(31):
        t.add_super_block(2048)
    with pytest.raises(S.SlabHashError):
        t.add_super_block(2048)                       # 32 super blocks at most
    assert t.stats()["pool_capacity"] == 32 * 2048
